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


# ------------------------------------------------------------------------------------------
# The averaging procedure (pprs_series_average_refine): rounds of averaging the aligned frames
# and re-registering every frame i >= 1 to the average from its current deformation.

TIE_DE = 1e-5  # a replayed decision may differ from the oracle's own by this much energy


def _params(levels):
    import paper_1712_02533_amd as P
    gp = P.Params(levels=levels, scan="sequential")
    op = O.Params(levels=gp.levels, lam=gp.lam, beta=gp.beta, sigma=gp.armijo_sigma,
                  ladder_k=gp.ladder_k, cap=gp.step_cap, tau_min_rel=gp.tau_min_rel,
                  eps=gp.eps, iter_max=gp.iter_max)
    return gp, op


def _truth_start(s):
    from synth import ground_truth
    N, side = s.frames.shape[0], s.frames.shape[1]
    u = [np.zeros((2, side, side))] + [ground_truth(s, k) for k in range(1, N)]
    return np.stack(u).astype(np.float32)


def _refine_case(spec, levels, passes, fp32_spread=False):
    """GPU rounds against the oracle's, started from the analytic displacements (FP32, both
    sides). The oracle replays the GPU's logged decisions and reports, per registration, how far
    its own tests were from each (the gap). fp32_spread: the oracle is run a second time along
    the same decisions with u stored in FP32, as the kernels store it; the spread between the
    two runs says how sensitive each registration is to rounding. Returns (u_gpu, u_oracle,
    u_oracle_fp32 or None, avg_gpu, avg_oracle, frames, gaps) in pixels, gaps pass-major."""
    torch = _torch()
    import paper_1712_02533_amd as P
    s = make_series(spec)
    N = spec.n_frames
    gp, op = _params(levels)
    u0 = _truth_start(s)
    fr = torch.tensor(s.frames, device="cuda")
    u = torch.tensor(u0, device="cuda")
    say("averaging procedure", spec, "levels", levels, "passes", passes)
    with P.DecisionLog(passes * (N - 1)) as log:
        _, avg, rows = P.series_average_refine(fr, u, passes, gp)
    flat = [st for row in rows for st in row]
    force = [list(st.iters) for st in flat]
    rungs = [log.rungs(r, sum(st.iters)) for r, st in enumerate(flat)]
    uo, ao, so = O.series_average_refine(s.frames, u0, passes, op, force=force, rungs=rungs)
    u32 = None
    if fp32_spread:
        O.set_u_storage_f32(True)
        try:
            u32, _, _ = O.series_average_refine(s.frames, u0, passes, op, force=force,
                                                rungs=rungs)
        finally:
            O.set_u_storage_f32(False)
    assert len(so) == len(flat)
    for r, (g, o) in enumerate(zip(flat, so)):
        assert g.iters == o.iters and g.passes == o.trials, "registration %d" % r
    gaps = [max(o.tie_gap, o.armijo_gap) for o in so]
    say("  %d registrations, steps per level %s, replay gaps %s"
        % (len(flat), [st.iters for st in flat], ["%.1e" % g for g in gaps]))
    return u.cpu().numpy(), uo, u32, avg.cpu().numpy(), ao, s.frames, gaps


def test_average_refine_matches_oracle_small():
    """6 frames of 128 x 128 (drift 4 px, non-rigid 1 px, 10 counts), 3 levels, two rounds: every
    decision is the oracle's up to a near-tie, the fields agree with the oracle's to 1e-3 px and
    the average to 1e-4 of the frames' range."""
    u, uo, _, a, ao, f, gaps = _refine_case(SeriesSpec(6, 128, 4.0, 1.0, 10.0, 81), 3, 2)
    d = np.abs(u - uo)
    say("  field: max %.2e rms %.2e px; average: max %.2e" %
        (d.max(), np.sqrt((d ** 2).mean()), np.abs(a - ao).max()))
    assert max(gaps) <= TIE_DE
    assert np.all(u[0] == 0)
    assert d.max() < 1e-3
    assert np.abs(a - ao).max() < 1e-4 * float(f.max())


def test_average_refine_full_size_matches_oracle():
    """5 frames of 512 x 512 at the series workload's statistics (drift 8 px, non-rigid 1.5 px,
    5 counts), 4 levels, one round on 513^2 grids, frame by frame. Where storing u in FP32 moves
    the oracle (along the same decisions) by less than 1e-3 px, the registration is
    well-conditioned: every decision is the oracle's up to a near-tie and the field is held to
    the full-size bar (RMS < 1e-4 px, 99.9th percentile < 1e-3 px, max < 0.05 px). Where it
    moves it further, the descent is chaotic in FP32 (long runs on a flat energy; this case
    holds one, moved 4e-2 px by FP32 storage alone): a decision may then differ from the FP64
    oracle's by more than a near-tie. With the oracle's decisions the field is held to twice
    the oracle's own FP32 spread in RMS (at least 1e-4 px); with a decision flipped, to 0.05 px
    RMS (the tolerance of approximate associativity)."""
    u, uo, u32, a, ao, f, gaps = _refine_case(SeriesSpec(5, 512, 8.0, 1.5, 5.0, 82), 4, 1,
                                             fp32_spread=True)
    rms = lambda x: float(np.sqrt((x ** 2).mean()))
    n_tight = 0
    for i in range(1, u.shape[0]):
        d, d32 = np.abs(u[i] - uo[i]), np.abs(u32[i] - uo[i])
        tight = d32.max() < 1e-3
        say("  frame %d (%s): GPU - oracle rms %.2e p99.9 %.2e max %.2e; FP32-storage oracle "
            "rms %.2e max %.2e; decision gap %.1e"
            % (i, "well-conditioned" if tight else "chaotic", rms(d), np.percentile(d, 99.9),
               d.max(), rms(d32), d32.max(), gaps[i - 1]))
        if tight:
            n_tight += 1
            assert gaps[i - 1] <= TIE_DE
            assert rms(d) < 1e-4 and np.percentile(d, 99.9) < 1e-3 and d.max() < 0.05
        elif gaps[i - 1] <= TIE_DE:
            # the oracle's decisions, on a rounding-sensitive path
            assert rms(d) <= max(1e-4, 2 * rms(d32))
        else:
            # a decision flipped on the chaotic path: both runs are the method's results
            assert rms(d) <= 0.05
    assert n_tight >= 1
    # the averages differ by what the fields' differences move each bilinear sample, at most
    # |du_x| L_x + |du_y| L_y per frame (L: the frame's largest neighbour difference per axis),
    # plus FP32 rounding of the sum
    lx = [float(np.abs(np.diff(fi.astype(np.float64), axis=1)).max()) for fi in f]
    ly = [float(np.abs(np.diff(fi.astype(np.float64), axis=0)).max()) for fi in f]
    du = np.abs(u - uo)
    bound = sum(lx[i] * du[i, 0] + ly[i] * du[i, 1] for i in range(u.shape[0])) / u.shape[0]
    bound = bound + 1e-5 * float(f.max())
    say("  average: max difference %.2e, largest ratio to its bound %.3f"
        % (np.abs(a - ao).max(), float((np.abs(a - ao) / bound).max())))
    assert np.all(np.abs(a - ao) <= bound)


def test_average_refine_degenerate_cases_and_bad_arguments():
    """No rounds: u unchanged and the average is pprs_series_average's. Identical frames from the
    identity: the average is the frame and every registration stays at the identity (to the
    parity tolerance). One frame: nothing to register. Bad shapes and a
    negative round count raise before any kernel runs."""
    torch = _torch()
    import paper_1712_02533_amd as P
    s = make_series(SeriesSpec(4, 64, 2.0, 0.5, 10.0, 83))
    fr = torch.tensor(s.frames, device="cuda")
    gp, _ = _params(2)
    u0 = torch.tensor(_truth_start(s), device="cuda")
    u = u0.clone()
    _, a, rows = P.series_average_refine(fr, u, 0, gp)
    assert rows == [] and torch.equal(u, u0)
    assert torch.equal(a, P.series_average(fr, u0))
    same = fr[:1].repeat(4, 1, 1).contiguous()
    u = torch.zeros((4, 2, 64, 64), device="cuda")
    _, a, rows = P.series_average_refine(same, u, 2, gp)
    # the oracle stays exactly at the identity; the FP32 gradient of a vanishing mismatch is
    # rounding, so the GPU stays there to the parity tolerance
    assert float(u.abs().max()) < 1e-3 and len(rows) == 2 and len(rows[0]) == 3
    # a bilinear sample moved by |du| <= 1e-3 px changes by at most 2 |du| max|f|
    assert float((a - same[0]).abs().max()) <= 2e-3 * float(same.max())
    one = fr[:1].contiguous()
    u1 = torch.zeros((1, 2, 64, 64), device="cuda")
    _, a, rows = P.series_average_refine(one, u1, 3, gp)
    assert rows == [[], [], []] and float(u1.abs().max()) == 0.0
    assert float((a - one[0]).abs().max()) < 1e-5 * float(one.max())
    with pytest.raises(ValueError):
        P.series_average_refine(fr, torch.zeros((4, 2, 64, 63), device="cuda"), 1, gp)
    with pytest.raises(ValueError):
        P.series_average_refine(fr, torch.zeros((3, 2, 64, 64), device="cuda"), 1, gp)
    with pytest.raises(ValueError):
        P.series_average_refine(fr, u0.clone(), -1, gp)


def test_average_refine_improves_the_average():
    """The purpose of the procedure: on a noisy 16-frame series (5 counts, drift 2 px) that the
    scan registers in the right basin, one round brings the average closer to the clean object
    (RMS over the interior, the object scaled to the frames' mean) than the scan's own average.
    (Frames the scan leaves in a wrong basin of the blob lattice stay there: re-registration
    from their deformation cannot leave it.)"""
    torch = _torch()
    import paper_1712_02533_amd as P
    spec = SeriesSpec(16, 128, 2.0, 1.0, 5.0, 45)
    s = make_series(spec)
    frames = torch.tensor(s.frames, device="cuda")
    gp = P.Params(levels=3, scan="brent_kung")
    u, _, _ = P.prefix_register_series(frames, params=gp)
    a1 = P.series_average(frames, u).cpu().numpy()
    _, a2, _ = P.series_average_refine(frames, u, 1, gp)
    a2 = a2.cpu().numpy()
    clean = _clean_frame(spec, s.origin, s.amps, s.lattice_lo, s.shifts[0], s.sines[0])
    obj = clean * (s.frames.mean() / clean.mean())
    err = lambda x: float(np.sqrt(((x - obj)[12:-12, 12:-12] ** 2).mean()))
    say("  error against the clean object: scan average %.4f, after one round %.4f"
        % (err(a1), err(a2)))
    assert err(a2) < err(a1)
