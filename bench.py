#!/usr/bin/env python3
"""Benchmark: series registration (512 frames of 512 x 512, 4 levels, Brent-Kung scan) on one
MI355X. A step is one complete series registration: frame pyramids, the N-1 neighbour
registrations and every B application of the scan, with the frames already in HBM.

Prints one JSON line: registrations/s (A + B applications per second), the series time, the
roofline of the dominant kernel (algorithmic bytes / HIP-event time of its launches, taken in
extra steps after the timed ones because events around every launch slow the series), the
same series with the learned warm start (both modes, with the network's MFMA throughput) and
the FP64 CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "frame-pair registrations/s and series scan time (512², N=512), warm vs cold"
HBM_PEAK_GBS = 8000.0
SCAN_NAMES = {"sequential": "sequential", "brent_kung": "Brent-Kung", "kogge_stone": "Kogge-Stone",
              "sklansky": "Sklansky", "general": "general-strategy", "blelloch": "Blelloch",
              "reduce_then_scan": "reduce-then-scan"}
WORKLOADS = {
    "series512": dict(name="512 frames of 512x512, drift<=8 px, non-rigid<=1.5 px, 5 counts; "
                    "4 levels; Brent-Kung scan; cold start",
               spec=("series512",)),
    "series256": dict(name="64 frames of 256x256, drift<=4 px, non-rigid<=1 px, 10 counts; "
                    "3 levels; Brent-Kung scan; cold start", spec=("series256",)),
    "tiny64": dict(name="8 frames of 64x64, drift<=2 px, 20 counts; 2 levels; sequential scan",
               spec=("tiny64",)),
    "paper": dict(name="4096 frames of 1024x1024, drift<=2 px, 10 counts; rigid operator; "
                       "3 levels (the paper's levels 8-10); Brent-Kung scan", spec=None),
    "mixed": dict(name="16 independent series in one run: sides {128,256,512,1024}, 32-512 "
                    "frames, drift<=8 px, non-rigid<=1.5 px, 2-20 counts; coarsest level 6; "
                    "Brent-Kung scans; segmented slot pool", spec=None),
}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def profile_figure(kernel, key):
    """A per-launch figure of `kernel` (hbm_bytes_per_launch: calibrated FETCH_SIZE +
    WRITE_SIZE; valu_insts_per_launch: SQ_INSTS_VALU) from the committed rocprofv3 counter
    summary profiles/counters_<kernel>.md, if it was taken for the current kernel source."""
    path = os.path.join(ROOT, "profiles", "counters_%s.md" % kernel)
    if not os.path.exists(path):
        return None
    try:
        import hashlib
        rec = {}
        for line in open(path):
            line = line.strip()
            if ":" in line and line.split(":")[0] in ("kernel", "kernels_hip_sha256", key):
                k, v = line.split(":", 1)
                rec[k.strip()] = v.strip()
        src = open(os.path.join(ROOT, "paper_1712_02533_amd", "csrc", "kernels.hip"), "rb").read()
        if rec.get("kernels_hip_sha256") != hashlib.sha256(src).hexdigest():
            return None
        return float(rec[key])
    except Exception:
        return None


# VALU issue peak of MI355X without packed FP32: 256 CUs x 4 SIMDs, a wave64 instruction
# occupying a 16-lane SIMD for 4 cycles, at 2.4 GHz (the same rate gives the 78.6 TFLOP/s of
# non-packed FMA)
VALU_PEAK_GINST = 256 * 4 * 2.4e9 / 4 / 1e9


def stream_bandwidth(torch, dev, gib=2, reps=3):
    """Achievable HBM bandwidth beside the 8 TB/s specification: the best of `reps` device
    copies of `gib` GiB (read + write counted), timed with events on torch's stream, which is
    where the copy runs."""
    n = (gib << 30) // 4
    a = torch.empty(n, device=dev)
    b = torch.empty_like(a)
    a.fill_(1.0)
    best = float("inf")
    for _ in range(reps + 1):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del a, b
    return 2.0 * (gib << 30) / (best * 1e-3) / 1e9


def kernel_roofline(kt, stream, traffic):
    """Per-kind figures and the roofline object of the dominant kernel kind (most event time)
    from P.kernel_timing() output {kind: (ms, launches, algorithmic bytes)}. traffic: read the
    calibrated counter figure from profiles/ (taken on the 512-frame series only)."""
    log("device copy (2 GiB each way): %.0f GB/s" % stream)
    kernels = {}
    for name, (ms, launches, byts) in kt.items():
        if launches:
            kernels[name] = dict(ms=round(ms, 3), launches=launches,
                                 gbs=round(byts / (ms * 1e-3) / 1e9, 1) if ms > 0 else None)
    cand = {k: v for k, v in kt.items() if v[2] > 0}
    dom = max(cand, key=lambda k: cand[k][0])
    ms, launches, byts = kt[dom]
    achieved = byts / (ms * 1e-3) / 1e9
    roofline = dict(bound="hbm", kernel=dom, achieved=round(achieved, 1), peak=HBM_PEAK_GBS,
                    unit="GB/s", frac=round(achieved / HBM_PEAK_GBS, 4),
                    traffic=profile_figure(dom, "hbm_bytes_per_launch") if traffic else None,
                    launches=launches, avg_launch_us=round(1e3 * ms / launches, 2),
                    bytes_per_launch=byts / launches, stream_gbs=round(stream, 1),
                    frac_of_stream=round(achieved / stream, 4))
    # the issue-rate view of the same launches: the kernel's wave64 VALU instructions per
    # launch (counted by rocprofv3 on this workload) over the live average launch time
    insts = profile_figure(dom, "valu_insts_per_launch") if traffic else None
    if insts:
        ginst = insts / (ms * 1e-3 / launches) / 1e9
        roofline["valu_issue"] = dict(achieved=round(ginst, 1), peak=VALU_PEAK_GINST,
                                      unit="G wave64 VALU instructions/s",
                                      frac=round(ginst / VALU_PEAK_GINST, 4),
                                      insts_per_launch=insts)
    return roofline, kernels


def cpu_baseline(series, cfg, n_a, threads, scan):
    """The FP64 oracle timed on a bounded sample of the same series: n_a neighbour
    registrations (frames m, m+1), then the first scan level's B applications over them
    (frames j-1 and j+1 from the composition of the two neighbour results), each on its own
    host thread, `threads` at a time. From the mean A and B times it estimates the oracle's whole
    series time on the same threads, level by level of the schedule (ceil(width / threads)
    rounds of a level's mean op time), and reports one-thread registration times."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    import oracle as O
    import paper_1712_02533_amd as P
    gp = P.Params(levels=cfg["levels"], scan=scan)
    op = O.Params(levels=gp.levels, lam=gp.lam, beta=gp.beta, sigma=gp.armijo_sigma,
                  ladder_k=gp.ladder_k, cap=gp.step_cap, tau_min_rel=gp.tau_min_rel, eps=gp.eps,
                  iter_max=gp.iter_max)
    frames = series.frames
    N = len(frames)
    n_a = max(2, min(n_a, N - 1))
    nodes = [O.frame_to_nodes(f) for f in frames[:n_a + 1]]
    res = {}

    def a_op(m):
        t = time.perf_counter()
        u, _, _ = O.register(nodes[m], nodes[m + 1], op)
        res[m] = u
        return time.perf_counter() - t

    def b_op(j):
        t = time.perf_counter()
        O.register(nodes[j - 1], nodes[j + 1], op, u0=O.compose(res[j - 1], res[j]))
        return time.perf_counter() - t

    O._load()
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        ta = list(ex.map(a_op, range(n_a)))
        tb = list(ex.map(b_op, range(1, n_a, 2)))
    dt = time.perf_counter() - t0
    n_ops = len(ta) + len(tb)
    # whole-series estimate: the schedule's levels, each ceil(width / threads) rounds
    plan, n_lv = P.scan_plan(scan, N - 1)
    widths = [sum(1 for x in plan if x[2] == lv) for lv in range(n_lv)]
    ma, mb = float(np.mean(ta)), float(np.mean(tb))
    est = -(-(N - 1) // threads) * ma + sum(-(-w // threads) * mb for w in widths)
    return dict(value=round(n_ops / dt, 3), unit="registrations/s", cores=threads, kind="oracle",
                sample="%d neighbour registrations and the %d B applications of the first scan "
                       "level over them (frames 0..%d of the same series), FP64, one "
                       "registration per host thread, %d threads, %.1f s" %
                       (len(ta), len(tb), n_a, threads, dt),
                one_thread_s=dict(a=round(ma, 2), b=round(mb, 2)),
                series_estimate_s=round(est, 1),
                series_estimate_method="sum over the %d scan levels (and the neighbour batch) "
                                       "of ceil(level width / %d) x the sample's mean A or B "
                                       "time; %d registrations" %
                                       (n_lv, threads, N - 1 + len(plan)))


# multiply-adds x 2 of one forward pass of the warm-start network (3x3 convolutions)
CNN_LAYERS = [(64, 64, 2), (32, 128, 64), (16, 256, 128), (32, 128, 384), (64, 64, 192),
              (128, 2, 66)]  # (output side, Cout, Cin)
CNN_FLOP_PER_PAIR = sum(2 * h * h * co * 9 * ci for h, co, ci in CNN_LAYERS)
# what the forward executes: the layers after a 2x upsampling (L4, L5, L6) read their
# upsampled channels at the source resolution through folded weights, 4 source pixels per
# output instead of 9 taps (upsampled channels: 256 of L4's 384, 128 of L5's 192, 64 of L6's 66)
CNN_UPSAMPLED_CIN = [0, 0, 0, 256, 128, 64]
CNN_FLOP_PER_PAIR_EXECUTED = sum(2 * h * h * co * (4 * cu + 9 * (ci - cu))
                                 for (h, co, ci), cu in zip(CNN_LAYERS, CNN_UPSAMPLED_CIN))
# one training sample: the forward pass, the weight gradients of every layer and the data
# gradients of every layer but the first (each a product of the forward's size)
CNN_TRAIN_FLOP_PER_SAMPLE = 3 * CNN_FLOP_PER_PAIR - 2 * 64 * 64 * 64 * 9 * 2
MFMA_BF16_PEAK_TFLOPS = 2500.0


def truth_sample(series, n_sample=16, workers=8):
    """The analytic displacements phi_0k (pixels) of n_sample frames spread over the series."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    from synth import ground_truth
    N = len(series.frames)
    ks = sorted(set(int(k) for k in np.linspace(1, N - 1, n_sample)))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        gts = list(ex.map(lambda k: ground_truth(series, k), ks))
    return ks, gts


def accuracy(u, ks, gts, side):
    """Per sampled frame: RMS error (px) against the analytic displacement over the interior
    (a border of the largest displacement + 6 px left out, where the frames do not overlap)."""
    import numpy as np
    out = []
    for k, gt in zip(ks, gts):
        b = min(int(np.abs(gt).max()) + 6, side // 4)
        d = u[k].cpu().numpy()[:, b:-b, b:-b] - gt[:, b:-b, b:-b]
        out.append(float(np.sqrt((d ** 2).mean())))
    return np.array(out)


def average_rounds(P, torch, series, frames, out, avg, params, rounds=2, truth=None):
    """The series averaging procedure after the scan: each round averages the aligned frames
    and re-registers frames 1.. to the average from their current deformation. Reports each
    round's time, the average's RMS error against the clean object (the first frame's
    noise-free image scaled to the frames' mean count, interior only) and, with truth = (ks,
    gts), the registrations' accuracy against the analytic displacements of those frames."""
    import numpy as np
    from synth.blobs import _clean_frame
    spec = series.spec
    clean = _clean_frame(spec, series.origin, series.amps, series.lattice_lo, series.shifts[0],
                         series.sines[0])
    obj = clean * (float(series.frames.mean()) / float(clean.mean()))
    b = 24
    err = lambda a: float(np.sqrt(((a.cpu().numpy() - obj)[b:-b, b:-b] ** 2).mean()))

    def acc(u):
        if truth is None:
            return None, None, None
        a = accuracy(u, truth[0], truth[1], spec.side)
        # the common drift: the mean signed error of the sampled frames within 1 px (a shift
        # all frames share moves the average off frame 0's coordinates)
        dr = []
        for k, gt, e in zip(truth[0], truth[1], a):
            if e <= 1.0:
                bb = min(int(np.abs(gt).max()) + 6, spec.side // 4)
                dr.append((u[k].cpu().numpy()[:, bb:-bb, bb:-bb] - gt[:, bb:-bb, bb:-bb])
                          .mean(axis=(1, 2)))
        drift = [round(float(x), 4) for x in np.mean(dr, axis=0)] if dr else None
        return round(float(a.mean()), 4), int((a > 1.0).sum()), drift

    a0, o0, d0 = acc(out)
    res = dict(err_scan_average=round(err(avg), 4), acc_rms_px_scan=a0, frames_over_1px_scan=o0,
               drift_px_scan=d0, rounds=[])
    u = out.clone()
    for _ in range(rounds):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, a, rows = P.series_average_refine(frames, u, 1, params)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0)
        steps = float(np.mean([sum(st.iters) for st in rows[0]]))
        ar, ov, dr = acc(u)
        res["rounds"].append(dict(ms=round(ms, 1), registrations=len(rows[0]),
                                  mean_steps=round(steps, 1), err=round(err(a), 4),
                                  acc_rms_px=ar, frames_over_1px=ov, drift_px=dr))
        log("averaging round: %.1f ms, %d registrations (%.1f steps each), average's error "
            "against the clean object %.4f (scan average %.4f); accuracy against the truth %s "
            "px (scan %s), frames off by more than 1 px: %s (scan %s), common drift %s px "
            "(scan %s)" % (ms, len(rows[0]), steps, err(a), res["err_scan_average"], ar, a0,
                           ov, o0, dr, d0))
    return res


def warm_runs(P, series, frames, out, params, args, regs_per_step, cold_ms):
    """The same series with the learned warm start (both modes): throughput, accuracy against
    the analytic displacement beside the cold run's on sampled frames, the judge's decisions,
    difference to the cold result, and the network's forward and training throughput."""
    import numpy as np
    import torch
    cold = out.clone()
    net = P.WarmStartNet()
    net.load(args.weights)
    side = frames.shape[-1]
    t0 = time.perf_counter()
    ks, gts = truth_sample(series)
    acc_cold = accuracy(cold, ks, gts, side)
    log("truth of %d sampled frames in %.1f s; cold accuracy %.4f px RMS (mean over frames)"
        % (len(ks), time.perf_counter() - t0, acc_cold.mean()))
    good = acc_cold <= 0.5   # frames the cold method recovers
    M = frames.shape[0] - 1
    res = dict(sampled_frames=ks, cold=dict(ms_per_step=round(cold_ms, 1),
                                             acc_rms_px=round(float(acc_cold.mean()), 4),
                                             acc_rms_px_per_frame=[round(x, 4) for x in acc_cold],
                                             frames_within_0_5px=int(good.sum())))
    for mode in ("refine", "skip"):
        P.set_warm_start(net, mode=mode)
        try:
            w = torch.empty_like(out)
            P.prefix_register_series(frames, params=params, out=w)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                _, st, ops = P.prefix_register_series(frames, params=params, out=w,
                                                      want_op_stats=True)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / args.steps
        finally:
            P.set_warm_start(None)
        acc = accuracy(w, ks, gts, side)
        d = (w - cold)[:, :, 16:-16, 16:-16]
        dg = (w - cold)[[k for k, g in zip(ks, good) if g]][:, :, 16:-16, 16:-16]
        res[mode] = dict(value=round(regs_per_step / dt, 3), ms_per_step=round(1e3 * dt, 1),
                         acc_rms_px=round(float(acc.mean()), 4),
                         acc_rms_px_per_frame=[round(x, 4) for x in acc],
                         acc_minus_cold_px=round(float(acc.mean() - acc_cold.mean()), 4),
                         worst_frame_minus_cold_px=round(float((acc - acc_cold).max()), 4),
                         rms_vs_cold_px=round(float(d.pow(2).mean().sqrt()), 4),
                         rms_vs_cold_px_where_cold_within_0_5px=round(
                             float(dg.pow(2).mean().sqrt()), 4) if dg.numel() else None,
                         fallbacks=sum(1 for o in ops[:M] if o.flags & 4),
                         network_starts_b=sum(1 for o in ops[M:] if o.flags & 8))
        log("warm (%s): %.1f ms per series (cold %.1f); accuracy %.4f px (cold %.4f); "
            "%d fallbacks, %d B starts from the network" %
            (mode, 1e3 * dt, cold_ms, acc.mean(), acc_cold.mean(), res[mode]["fallbacks"],
             res[mode]["network_starts_b"]))
        if mode == "skip" and not args.no_refine:
            # the averaging procedure from the more accurate warm result
            res[mode]["average_refine"] = average_rounds(
                P, torch, series, frames, w, P.series_average(frames, w), params,
                truth=(ks, gts))
    # network forward on the series' neighbour pairs, as the warm start runs it (64 per call)
    n = frames.shape[0] - 1
    ref = np.arange(n, dtype=np.int32)
    x = P.pair_inputs(frames, ref, ref + 1)
    for b0 in range(0, n, 64):
        net.forward(x[b0:b0 + 64])
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for b0 in range(0, n, 64):
        net.forward(x[b0:b0 + 64])
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    tf = CNN_FLOP_PER_PAIR * n / (ms * 1e-3) / 1e12
    tfx = CNN_FLOP_PER_PAIR_EXECUTED * n / (ms * 1e-3) / 1e12
    res["cnn_forward"] = dict(pairs=n, ms=round(ms, 2), flop_per_pair=CNN_FLOP_PER_PAIR,
                              tflops=round(tf, 1), peak_tflops=MFMA_BF16_PEAK_TFLOPS,
                              frac=round(tf / MFMA_BF16_PEAK_TFLOPS, 4),
                              flop_per_pair_executed=CNN_FLOP_PER_PAIR_EXECUTED,
                              tflops_executed=round(tfx, 1),
                              frac_executed=round(tfx / MFMA_BF16_PEAK_TFLOPS, 4))
    log("cnn forward: %d pairs in %.2f ms, %.1f TFLOP/s (%.1f executed)" % (n, ms, tf, tfx))
    # one training step (forward, MSE, backward, Adam) on 64 samples, timed over 10 steps on a
    # separate network (the loaded one is not changed)
    trainer = P.WarmStartNet(seed=5)
    xb = x[:64].contiguous()
    tb = torch.zeros_like(xb)
    for _ in range(2):
        trainer.train_step(xb, tb, lr=1e-4)
    torch.cuda.synchronize()
    steps = 10
    e0.record()
    for _ in range(steps):
        trainer.train_step(xb, tb, lr=1e-4)
    e1.record()
    torch.cuda.synchronize()
    ms_t = e0.elapsed_time(e1) / steps
    tft = CNN_TRAIN_FLOP_PER_SAMPLE * xb.shape[0] / (ms_t * 1e-3) / 1e12
    res["cnn_train"] = dict(batch=int(xb.shape[0]), ms_per_step=round(ms_t, 2),
                            flop_per_sample=CNN_TRAIN_FLOP_PER_SAMPLE, tflops=round(tft, 1),
                            peak_tflops=MFMA_BF16_PEAK_TFLOPS,
                            frac=round(tft / MFMA_BF16_PEAK_TFLOPS, 4))
    log("cnn training step: %d samples in %.2f ms, %.1f TFLOP/s" % (xb.shape[0], ms_t, tft))
    trainer.close()
    return res


def bench_paper_rigid(args):
    """The paper's serial experiment in shape (4096 frames of about 1024^2, levels 8-10, the
    rigid operator it most likely timed), as one rigid series on one GPU. Synthetic frames."""
    import torch
    import paper_1712_02533_amd as P
    from synth import SeriesSpec, make_series
    spec = SeriesSpec(args.frames or 4096, 1024, 2.0, 0.0, 10.0, 4)
    t0 = time.perf_counter()
    series = make_series(spec, workers=min(16, os.cpu_count() or 1))
    log("generated %d frames of 1024x1024 in %.1f s" % (spec.n_frames, time.perf_counter() - t0))
    dev = torch.device("cuda", 0)
    frames = torch.tensor(series.frames, device=dev)
    del series
    params = P.Params(levels=3, scan="brent_kung")
    for w in range(args.warmup):
        _, st = P.prefix_register_series_rigid(frames, params=params)
        log("warmup %d: %.1f ms" % (w, st.ms_total))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    regs = 0
    for k in range(args.steps):
        _, st = P.prefix_register_series_rigid(frames, params=params)
        regs += st.n_ops_a + st.n_ops_b
        log("step %d: %.1f ms (prepare %.1f, scan %.1f), %d A + %d B" %
            (k, st.ms_total, st.ms_prepare, st.ms_scan, st.n_ops_a, st.n_ops_b))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(json.dumps(dict(
        metric="frame-pair registrations/s and series time, rigid operator", value=round(regs / dt, 3),
        unit="registrations/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
        ms_per_step=round(1e3 * dt / args.steps, 1), higher_is_better=True, scaling="weak",
        vs_baseline=None, dtype="f32", data="synthetic",
        config=dict(workload=WORKLOADS["paper"]["name"].replace("4096", str(spec.n_frames)),
                    frames=spec.n_frames, side=1024,
                    levels=3, scan="brent_kung", operator="rigid"))), flush=True)


def bench_uneven(args):
    """The segmented workload: batches of 16 independent series of mixed sides and lengths
    (one batch per seed, seeds 3, 4, ... one per step), each registered concurrently in one
    segmented run, cold and then with the warm start. Throughput over all batches; per-series
    latency p50/p99 pooled over the batches (5 steps give 80 samples). Frame generation and
    upload stay outside the timed runs."""
    import numpy as np
    import torch
    import paper_1712_02533_amd as P
    from synth import make_series
    from synth.blobs import uneven_batch
    dev = torch.device("cuda", 0)
    seeds = [3 + k for k in range(max(args.steps, 1))]
    batches = []
    t0 = time.perf_counter()
    for sd in seeds:
        b = uneven_batch(seed=sd)
        fr = [torch.tensor(make_series(x["spec"], workers=min(16, os.cpu_count() or 1)).frames,
                           device=dev) for x in b]
        batches.append(dict(seed=sd, frames=fr, levels=[x["levels"] for x in b],
                            outs=[torch.empty((f.shape[0], 2, f.shape[1], f.shape[2]),
                                              device=dev) for f in fr]))
        log("seed %d: %d series, %d frames (%.1f s so far)" % (
            sd, len(fr), sum(f.shape[0] for f in fr), time.perf_counter() - t0))
    params = P.Params(levels=max(max(b["levels"]) for b in batches), scan="brent_kung")

    def run_one(b):
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, st, la = P.register_series_batch(b["frames"], params=params, levels=b["levels"],
                                            outs=b["outs"])
        torch.cuda.synchronize()
        return time.perf_counter() - t, sum(x.n_ops_a + x.n_ops_b for x in st), list(la)

    def run(tag):
        lat, regs, dt = [], 0, 0.0
        for b in batches:
            d, r, la = run_one(b)
            dt += d
            regs += r
            lat += la
            log("%s seed %d: %.0f ms, latencies p50 %.0f ms, max %.0f ms"
                % (tag, b["seed"], 1e3 * d, np.percentile(la, 50), max(la)))
        return regs / dt, 1e3 * dt / len(batches), lat

    for w in range(args.warmup):
        run_one(batches[0])
    value, ms, lat = run("cold")
    roofline, kernels = None, {}
    if not args.no_timing:
        P.set_kernel_timing(True, dev)
        P.kernel_timing(reset=True, device=dev)
        run_one(batches[0])
        kt = P.kernel_timing(reset=True, device=dev)
        P.set_kernel_timing(False, dev)
        roofline, kernels = kernel_roofline(kt, stream_bandwidth(torch, dev), traffic=False)
    result = dict(
        metric=METRIC, value=round(value, 3), unit="registrations/s", n_gpus=1,
        steps=len(batches), warmup=args.warmup, ms_per_step=round(ms, 1),
        higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32", data="synthetic",
        config=dict(workload=WORKLOADS["mixed"]["name"], seeds=seeds,
                    series=sum(len(b["frames"]) for b in batches),
                    sides=[[int(f.shape[1]) for f in b["frames"]] for b in batches],
                    frames=[[int(f.shape[0]) for f in b["frames"]] for b in batches],
                    start="cold"),
        latency_ms=dict(p50=round(float(np.percentile(lat, 50)), 1),
                        p99=round(float(np.percentile(lat, 99)), 1), samples=len(lat)),
        roofline=roofline, kernels=kernels)
    weights = os.path.join(ROOT, "paper_1712_02533_amd", "weights", "warmstart_mixed.safetensors")
    if not args.no_warm and os.path.exists(weights):
        net = P.WarmStartNet()
        net.load(weights)
        P.set_warm_start(net, mode="refine")
        try:
            run_one(batches[0])
            wv, wms, wlat = run("warm")
        finally:
            P.set_warm_start(None)
        result["warm"] = dict(value=round(wv, 3), ms_per_step=round(wms, 1),
                              latency_ms=dict(p50=round(float(np.percentile(wlat, 50)), 1),
                                              p99=round(float(np.percentile(wlat, 99)), 1),
                                              samples=len(wlat)))
    print(json.dumps(result), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="series512", choices=sorted(WORKLOADS))
    ap.add_argument("--frames", type=int, default=0, help="override the series length")
    ap.add_argument("--scan", default="", help="override the scan schedule (sequential, "
                    "brent_kung, kogge_stone, sklansky, general, blelloch, reduce_then_scan)")
    ap.add_argument("--workers", type=int, default=0, help="workers P of the general and "
                    "reduce-then-scan strategies (0: ceil(sqrt(N-1)))")
    ap.add_argument("--cpu-ops", type=int, default=0, help="oracle sample size (0 = auto)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-timing", action="store_true", help="no per-kernel HIP events")
    ap.add_argument("--no-warm", action="store_true", help="skip the warm-start runs")
    ap.add_argument("--no-refine", action="store_true",
                    help="skip the rounds of the series averaging procedure")
    ap.add_argument("--no-tune", action="store_true", help="default launch shape, no autotuning")
    ap.add_argument("--no-rigid", action="store_true", help="skip the rigid-operator series")
    ap.add_argument("--weights", default=os.path.join(ROOT, "paper_1712_02533_amd", "weights",
                                                      "warmstart_512.safetensors"))
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    if args.config == "mixed":
        return bench_uneven(args)
    if args.config == "paper":
        return bench_paper_rigid(args)
    import numpy as np
    import torch
    import paper_1712_02533_amd as P
    from synth import CONFIGS, make_series
    from dataclasses import replace

    cfg = CONFIGS[args.config]
    spec = cfg["spec"]
    if args.frames:
        spec = replace(spec, n_frames=args.frames)
    # host threads of the CPU baseline: all cores of this host, at most 16 (the host share one
    # GPU's box gives a run)
    nthreads = min(16, os.cpu_count() or 1)
    t0 = time.perf_counter()
    series = make_series(spec, workers=nthreads)
    log("generated %d frames of %dx%d in %.1f s" % (spec.n_frames, spec.side, spec.side,
                                                     time.perf_counter() - t0))
    dev = torch.device("cuda", 0)
    frames = torch.tensor(series.frames, device=dev)
    out = torch.empty((spec.n_frames, 2, spec.side, spec.side), device=dev)
    scan = args.scan or cfg["scan"]
    params = P.Params(levels=cfg["levels"], scan=scan, scan_workers=args.workers)
    # a plain device copy of known size (256 MiB read + 256 MiB written), untimed: profiler
    # counters of this kernel calibrate the HBM byte counters of the registration kernels
    calib = torch.empty(64 << 20, device=dev)
    calib.copy_(torch.ones_like(calib))
    del calib
    tuning = None
    if not args.no_tune:
        from paper_1712_02533_amd import autotune
        t0 = time.perf_counter()
        tuning = autotune.tune(frames, params, cache=os.path.join(
            os.environ.get("TMPDIR", "/tmp"), "pprs_tuning_bench.json"), log=log)
        log("autotuned launch shape in %.1f s: %s" % (time.perf_counter() - t0, tuning))
    for w in range(args.warmup):
        _, st, _ = P.prefix_register_series(frames, params=params, out=out)
        log("warmup %d: %.1f ms, %d A + %d B ops" % (w, st.ms_total, st.n_ops_a, st.n_ops_b))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for k in range(args.steps):
        _, st, _ = P.prefix_register_series(frames, params=params, out=out)
        stats.append(st)
        log("step %d: %.1f ms (prepare %.1f, preprocess %.1f, scan %.1f), flags %d" %
            (k, st.ms_total, st.ms_prepare, st.ms_preprocess, st.ms_scan, st.flags_or))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    regs = sum(s.n_ops_a + s.n_ops_b for s in stats)
    value = regs / elapsed
    ms_per_step = 1e3 * elapsed / args.steps
    # per-kernel HIP events bracket every launch, which slows the series: they run in steps of
    # their own after the timed ones (same work, same launches)
    timing = not args.no_timing
    if timing:
        P.set_kernel_timing(True, dev)
        P.kernel_timing(reset=True, device=dev)
        for k in range(max(1, min(args.steps, 2))):
            P.prefix_register_series(frames, params=params, out=out)
        torch.cuda.synchronize()
        kt = P.kernel_timing(reset=True, device=dev)
        P.set_kernel_timing(False, dev)

    roofline = None
    kernels = {}
    if timing:
        # measured here only with timing on: the counter runs (no timing) keep the 256 MiB
        # calibration copy as their largest copy
        roofline, kernels = kernel_roofline(kt, stream_bandwidth(torch, dev), traffic=True)
    result = dict(
        metric=METRIC, value=round(value, 3), unit="registrations/s", n_gpus=1,
        steps=args.steps, warmup=args.warmup, ms_per_step=round(ms_per_step, 1),
        higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32",
        data="synthetic",
        config=dict(workload=WORKLOADS[args.config]["name"].replace(
                        "Brent-Kung scan", SCAN_NAMES[scan] + " scan"), frames=spec.n_frames,
                    side=spec.side, levels=cfg["levels"], scan=scan, start="cold",
                    **(dict(scan_workers=args.workers)
                       if scan in ("general", "reduce_then_scan") else {}),
                    tuning=tuning,
                    registrations_per_step=stats[0].n_ops_a + stats[0].n_ops_b),
        series_scan_s=round(ms_per_step / 1e3, 3),
        roofline=roofline, kernels=kernels,
        node_steps=stats[0].node_steps, node_passes=stats[0].node_passes,
    )
    # series averaging of the registered frames (the scan's consumer): u 8 B + frame 4 B per
    # pixel and frame, plus the average written once
    avg = torch.empty((spec.side, spec.side), device=dev)
    P.series_average(frames, out, avg)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 5
    for _ in range(reps):
        P.series_average(frames, out, avg)
    torch.cuda.synchronize()
    ams = 1e3 * (time.perf_counter() - t0) / reps
    abytes = spec.n_frames * spec.side * spec.side * 12 + spec.side * spec.side * 4
    result["average"] = dict(ms=round(ams, 3), bytes=abytes,
                             gbs=round(abytes / (ams * 1e-3) / 1e9, 1))
    log("series average: %.3f ms, %.0f GB/s" % (ams, abytes / (ams * 1e-3) / 1e9))
    if not args.no_refine:
        truth = truth_sample(series, n_sample=16, workers=nthreads) if spec.side >= 128 else None
        result["average_refine"] = average_rounds(P, torch, series, frames, out, avg, params,
                                                  truth=truth)
    if not args.no_rigid and scan not in ("blelloch", "reduce_then_scan"):
        # the same frames through the rigid operator (three parameters per registration)
        rp = P.Params(levels=cfg["levels"], scan=scan, scan_workers=args.workers)
        P.prefix_register_series_rigid(frames, params=rp)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rs = None
        for _ in range(2):
            _, rs = P.prefix_register_series_rigid(frames, params=rp)
        rms = 1e3 * (time.perf_counter() - t0) / 2
        rregs = rs.n_ops_a + rs.n_ops_b
        result["rigid"] = dict(ms_per_step=round(rms, 1), value=round(rregs / (rms * 1e-3), 3),
                               unit="registrations/s", registrations_per_step=rregs)
        log("rigid series: %.1f ms, %d registrations" % (rms, rregs))
    if not args.no_warm and os.path.exists(args.weights) and spec.side >= 128:
        result["warm"] = warm_runs(P, series, frames, out, params, args,
                                   stats[0].n_ops_a + stats[0].n_ops_b, ms_per_step)
    if not args.no_cpu:
        n_a = args.cpu_ops or nthreads
        log("cpu baseline: oracle on %d neighbour registrations and their B applications, "
            "%d threads" % (n_a, nthreads))
        result["cpu_baseline"] = cpu_baseline(series, cfg, n_a, nthreads, scan)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
