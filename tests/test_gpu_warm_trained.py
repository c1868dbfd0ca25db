"""What the trained warm start gains over the plain method, judged on the generator's analytic
displacements (the 512 x 512 workload: drift <= 8 px per frame, non-rigid <= 1.5 px, 5 counts).

Neighbour displacements reach ~20 px, beyond what four levels recover from the identity for some
pairs; the network's prediction starts those pairs in the right basin. Accuracy is the RMS error
against the truth over the interior; "equal accuracy" means the warm result is no worse than the
cold one by more than 0.05 px RMS.
"""
import os

import numpy as np
import pytest

from synth import CONFIGS, ground_truth, ground_truth_pair, make_series

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "paper_1712_02533_amd", "weights", "warmstart_512.safetensors")
BORDER = 24


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def say(*a):
    print("[trained]", *a, flush=True)


def _rms(a):
    return float(np.sqrt((a[:, BORDER:-BORDER, BORDER:-BORDER] ** 2).mean()))


@pytest.fixture(scope="module")
def case():
    torch = _torch()
    import paper_1712_02533_amd as P
    from dataclasses import replace
    spec = replace(CONFIGS["series512"]["spec"], n_frames=48, seed=150)  # not a training seed
    s = make_series(spec, workers=8)
    frames = torch.tensor(s.frames, device="cuda")
    net = P.WarmStartNet()
    net.load(WEIGHTS)
    return s, frames, net


def test_trained_warm_start_pairs(case):
    torch = _torch()
    import paper_1712_02533_amd as P
    s, frames, net = case
    params = P.Params(levels=4, scan="brent_kung")
    ref = np.arange(s.frames.shape[0] - 1, dtype=np.int32)
    cold, cst = P.register_pairs(frames, ref, ref + 1, params=params)
    out = {}
    for mode in ("refine", "skip"):
        P.set_warm_start(net, mode=mode)
        try:
            out[mode] = P.register_pairs(frames, ref, ref + 1, params=params)
        finally:
            P.set_warm_start(None)
    sample = list(range(0, len(ref), 4))
    errs = {"cold": [], "refine": [], "skip": []}
    for m in sample:
        g = ground_truth_pair(s, m, m + 1)
        errs["cold"].append(_rms(cold[m].cpu().numpy() - g))
        for mode in ("refine", "skip"):
            errs[mode].append(_rms(out[mode][0][m].cpu().numpy() - g))
    for k in errs:
        errs[k] = np.array(errs[k])
        say("%-6s: mean RMS error %.3f px, pairs off by > 1 px: %d of %d, fallbacks %s" %
            (k, errs[k].mean(), (errs[k] > 1.0).sum(), len(sample),
             "-" if k == "cold" else sum(1 for x in out[k][1] if x.flags & 4)))
    # the gain: fewer pairs in a wrong basin, and no loss of accuracy on average
    for mode in ("refine", "skip"):
        assert (errs[mode] > 1.0).sum() < (errs["cold"] > 1.0).sum()
        assert errs[mode].mean() <= errs["cold"].mean() + 0.05
    # where the plain method reaches the truth, the warm start stays as accurate on average
    good = errs["cold"] < 0.5
    assert good.sum() >= len(sample) // 3
    assert errs["refine"][good].mean() <= errs["cold"][good].mean() + 0.05
    # and pair by pair: where cold is within 0.5 px of the truth, no warm pair is worse by more
    # than 0.05 px (the judge falls back to the cold start when the warm result is worse)
    for mode in ("refine", "skip"):
        worse = errs[mode][good] - errs["cold"][good]
        say("%-6s: per-pair excess over cold where cold < 0.5 px: max %.4f px over %d pairs"
            % (mode, worse.max(), good.sum()))
        assert worse.max() <= 0.05


def test_trained_warm_start_series_accuracy(case):
    torch = _torch()
    import paper_1712_02533_amd as P
    s, frames, net = case
    params = P.Params(levels=4, scan="brent_kung")
    cold, _, _ = P.prefix_register_series(frames, params=params)
    P.set_warm_start(net, mode="refine")
    try:
        warm, st, ops = P.prefix_register_series(frames, params=params, want_op_stats=True)
    finally:
        P.set_warm_start(None)
    ks = list(range(4, s.frames.shape[0], 8))
    ec, ew = [], []
    for k in ks:
        g = ground_truth(s, k)
        ec.append(_rms(cold[k].cpu().numpy() - g))
        ew.append(_rms(warm[k].cpu().numpy() - g))
    ec, ew = np.array(ec), np.array(ew)
    say("series phi_0k error vs truth (px), k=%s" % ks)
    say("  cold %s" % np.round(ec, 3))
    say("  warm %s" % np.round(ew, 3))
    assert ew.mean() <= ec.mean() + 0.05
