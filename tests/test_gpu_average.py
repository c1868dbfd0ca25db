"""Series averaging on the GPU (pprs_series_average) against the FP64 oracle: small frames in
full, the 512-frame 512 x 512 workload on sampled pixels, the degenerate single frame, and the
purpose of the step: the average of a registered noisy series is closer to the clean object
than any one frame."""
import numpy as np
import pytest

import oracle as O
from synth import SeriesSpec, make_series
from synth.blobs import _clean_frame

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def say(*a):
    print("[average]", *a, flush=True)


def _smooth_u(rng, N, H, W, amp):
    r, c = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    u = np.zeros((N, 2, H, W))
    for i in range(1, N):
        for k in range(2):
            a, b, ph = rng.uniform(0.02, 0.1), rng.uniform(0.02, 0.1), rng.uniform(0, 6.3)
            u[i, k] = amp * np.sin(a * c + b * r + ph) + rng.uniform(-amp, amp)
    return u


def test_average_matches_oracle_small():
    """7 frames of 64 x 96 (not square), displacements up to 10 px so that many samples are
    clamped at the borders. FP32 samples summed in FP64: 1e-5 of the value range."""
    torch = _torch()
    import paper_1712_02533_amd as P
    rng = np.random.default_rng(41)
    N, H, W = 7, 64, 96
    f = rng.uniform(0, 20, size=(N, H, W)).astype(np.float32)
    u = _smooth_u(rng, N, H, W, 5.0).astype(np.float32)
    say("frames", (N, H, W))
    got = P.series_average(torch.tensor(f, device="cuda"), torch.tensor(u, device="cuda"))
    ref = O.series_average(f, u)
    err = np.abs(got.cpu().numpy() - ref).max()
    say("  max abs err", err)
    assert err < 1e-5 * 20


def test_average_full_size_sampled():
    """512 frames of 512 x 512 (the series workload's size) on 256 sampled pixels."""
    torch = _torch()
    import paper_1712_02533_amd as P
    rng = np.random.default_rng(42)
    N, H = 512, 512
    f = torch.rand((N, H, H), device="cuda") * 10
    u = torch.tensor(_smooth_u(rng, 8, H, H, 8.0), dtype=torch.float32, device="cuda")
    u = u.repeat(N // 8, 1, 1, 1)
    u[0].zero_()
    say("frames", (N, H, H))
    got = P.series_average(f, u).cpu().numpy()
    rows, cols = rng.integers(0, H, 256), rng.integers(0, H, 256)
    cols[:8] = [0, H - 1, 0, H - 1, 1, H - 2, 255, 256]
    rows[:8] = [0, 0, H - 1, H - 1, 1, H - 2, 256, 255]
    ref = O.series_average(f.cpu().numpy(), u.cpu().numpy(), pixels=(rows, cols))
    err = np.abs(got[rows, cols] - ref).max()
    say("  max abs err on 256 pixels", err)
    assert err < 1e-5 * 10


def test_average_single_frame_is_the_frame_and_bad_shapes_raise():
    torch = _torch()
    import paper_1712_02533_amd as P
    f = torch.rand((1, 33, 40), device="cuda")
    u = torch.zeros((1, 2, 33, 40), device="cuda")
    a = P.series_average(f, u)
    # exact away from the last row and column; there the sample is v00 + 1 * (v01 - v00),
    # within one rounding of v01
    assert torch.equal(a[:-1, :-1], f[0, :-1, :-1])
    assert float((a - f[0]).abs().max()) < 1e-6
    with pytest.raises(P.PprsError):
        P.series_average(f, torch.zeros((1, 2, 33, 41), device="cuda"))
    with pytest.raises(P.PprsError):
        P.series_average(torch.rand((2, 1, 40), device="cuda"),
                         torch.zeros((2, 2, 1, 40), device="cuda"))


def test_average_of_registered_series_beats_single_frames():
    """A noisy 16-frame series (5 counts, drift <= 4 px, non-rigid <= 1 px) registered on the
    GPU and averaged: the average correlates with the clean first frame better than frame 0."""
    torch = _torch()
    import paper_1712_02533_amd as P
    spec = SeriesSpec(16, 128, 4.0, 1.0, 5.0, 43)
    s = make_series(spec)
    frames = torch.tensor(s.frames, device="cuda")
    u, _, _ = P.prefix_register_series(frames, params=P.Params(levels=2, scan="brent_kung"))
    avg = P.series_average(frames, u).cpu().numpy()
    clean = _clean_frame(spec, s.origin, s.amps, s.lattice_lo, s.shifts[0], s.sines[0])

    def ncc(a, b):
        m = 12
        a, b = a[m:-m, m:-m].ravel(), b[m:-m, m:-m].ravel()
        a, b = a - a.mean(), b - b.mean()
        return float((a * b).sum() / np.sqrt((a * a).sum() * (b * b).sum()))

    n_avg, n_0 = ncc(avg, clean), ncc(s.frames[0], clean)
    say("  NCC with the clean frame: average %.4f, frame 0 %.4f" % (n_avg, n_0))
    assert n_avg > n_0 + 0.05
