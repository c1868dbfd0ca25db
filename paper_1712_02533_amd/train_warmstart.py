"""Training driver of the learned warm start.

Data: neighbour pairs (m, m+1) of synthetic series with the statistics of the 512-frame
512 x 512 workload (drift <= 8 px, non-rigid <= 1.5 px, 5 counts per pixel), one series per
seed from 100 on. Inputs are the level-7 normalised frames of a pair (pair_inputs); targets are
the displacements the plain (cold-start) method finds for the pair at full resolution,
restricted to level 7 and expressed in level-7 cells (level7_targets). All network arithmetic
(forward, backward, Adam) runs in the library's kernels; torch only holds device buffers and
gathers mini-batches.

Augmentation: the 8 symmetries of the square act on a pair and its displacement together
(a flip of the x axis negates the x component; a transpose swaps the components).

    python -m paper_1712_02533_amd.train_warmstart --series 40 --minutes 8 \
        --out weights/warmstart_512.safetensors
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def log(*a):
    print("[train]", *a, flush=True)


def series_specs(n_series, n_frames, seed0, mix):
    """(SeriesSpec, levels) per training series. Default: the 512 x 512 workload's statistics,
    one seed each from seed0. mix: sides drawn from {128, 256, 512, 1024} and mean counts from
    U[2, 20] (the mixed-size batch workload), coarsest level 6."""
    from dataclasses import replace
    from synth import CONFIGS, SeriesSpec
    if not mix:
        base = CONFIGS["series512"]["spec"]
        return [(replace(base, n_frames=n_frames, seed=seed0 + i), CONFIGS["series512"]["levels"])
                for i in range(n_series)]
    rng = np.random.Generator(np.random.PCG64(seed0))
    out = []
    for i in range(n_series):
        side = int([128, 256, 512, 1024][i % 4])
        mu = float(rng.uniform(2.0, 20.0))
        out.append((SeriesSpec(n_frames, side, 8.0, 1.5, mu, seed0 + i),
                    int(np.log2(side)) - 6 + 1))
    return out


def make_dataset(specs, device, workers):
    """Inputs X [P, 128, 128, 2] and targets T [P, 128, 128, 2] on the device."""
    import torch
    import paper_1712_02533_amd as P
    from synth import make_series
    n_series = len(specs)
    X, T = [], []
    last = None
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=1) as ex:
        fut = ex.submit(make_series, specs[0][0], True, workers)
        for i in range(n_series):
            s = fut.result()
            if i + 1 < n_series:
                fut = ex.submit(make_series, specs[i + 1][0], True, workers)
            frames = torch.tensor(s.frames, device=device)
            n_frames = frames.shape[0]
            params = P.Params(levels=specs[i][1], scan="brent_kung")
            ref = np.arange(n_frames - 1, dtype=np.int32)
            u, st = P.register_pairs(frames, ref, ref + 1, params=params)
            X.append(P.pair_inputs(frames, ref, ref + 1))
            T.append(P.level7_targets(u))
            del u
            last = frames
            log("series %d/%d (side %d, seed %d): %d pairs, %.0f s" %
                (i + 1, n_series, specs[i][0].side, specs[i][0].seed, n_frames - 1,
                 time.perf_counter() - t0))
    return torch.cat(X), torch.cat(T), last


def dihedral(x, t, k):
    """Applies symmetry k (0..7) of the square to inputs and targets [B, H, W, 2] (x, y)."""
    import torch
    if k & 1:   # flip x: columns reversed, x component negated
        x = torch.flip(x, dims=[2])
        t = torch.flip(t, dims=[2]) * torch.tensor([-1.0, 1.0], device=t.device)
    if k & 2:   # flip y
        x = torch.flip(x, dims=[1])
        t = torch.flip(t, dims=[1]) * torch.tensor([1.0, -1.0], device=t.device)
    if k & 4:   # transpose: swap x and y
        x = x.transpose(1, 2)
        t = t.transpose(1, 2).flip(dims=[3])
    return x.contiguous(), t.contiguous()


def evaluate(net, X, T, batch, margin=4):
    """RMS error (level-7 cells) over the interior and the share of samples whose largest
    error stays below half a cell."""
    se, n, good = 0.0, 0, 0
    for b0 in range(0, X.shape[0], batch):
        y = net.forward(X[b0:b0 + batch])
        d = (y - T[b0:b0 + batch])[:, margin:-margin, margin:-margin, :]
        se += float((d * d).sum())
        n += d.numel()
        good += int((d.abs().amax(dim=(1, 2, 3)) < 0.5).sum())
    return float(np.sqrt(se / n)), good / X.shape[0]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--series", type=int, default=40)
    ap.add_argument("--frames", type=int, default=512)
    ap.add_argument("--seed0", type=int, default=100)
    ap.add_argument("--val-series", type=int, default=2)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--minutes", type=float, default=8.0, help="training time budget")
    ap.add_argument("--max-epochs", type=int, default=200)
    ap.add_argument("--init", default="", help="start from these weights")
    ap.add_argument("--net-seed", type=int, default=1)
    ap.add_argument("--out", default="")
    ap.add_argument("--eval-only", action="store_true",
                    help="compare warm and cold on one series (seed --seed0) with --init")
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--mix", action="store_true",
                    help="series of mixed sides and counts (the mixed-size batch workload)")
    args = ap.parse_args()
    if args.eval_only:
        return evaluate_only(args)
    if not args.out:
        ap.error("--out is required for training")

    import torch
    import paper_1712_02533_amd as P
    dev = torch.device("cuda", 0)
    params = P.Params(levels=4, scan="brent_kung")
    specs = series_specs(args.series, args.frames, args.seed0, args.mix)
    X, T, val_frames = make_dataset(specs, dev, args.workers)
    n_val = args.val_series * (args.frames - 1)
    Xv, Tv = X[-n_val:], T[-n_val:]
    Xt, Tt = X[:-n_val], T[:-n_val]
    log("train %d pairs, validation %d pairs; target RMS %.3f cells" %
        (Xt.shape[0], Xv.shape[0], float(Tt.pow(2).mean().sqrt())))

    net = P.WarmStartNet(seed=args.net_seed, device=dev)
    if args.init:
        net.load(args.init)
    rng = np.random.default_rng(args.net_seed)
    steps_per_epoch = Xt.shape[0] // args.batch
    budget = args.minutes * 60.0
    total_steps = steps_per_epoch * args.max_epochs
    history = []
    t0 = time.perf_counter()
    step = 0
    best = (float("inf"), None)
    for epoch in range(args.max_epochs):
        perm = torch.tensor(rng.permutation(Xt.shape[0]), device=dev)
        sym = rng.integers(0, 8, steps_per_epoch)
        run = 0.0
        te = time.perf_counter()
        for b in range(steps_per_epoch):
            idx = perm[b * args.batch:(b + 1) * args.batch]
            x, t = dihedral(Xt[idx], Tt[idx], int(sym[b]))
            # cosine decay over the expected number of steps within the time budget
            elapsed = time.perf_counter() - t0
            frac = min(1.0, elapsed / budget)
            lr = args.lr * (0.02 + 0.98 * 0.5 * (1 + np.cos(np.pi * frac)))
            run += net.train_step(x, t, lr=float(lr))
            step += 1
        dt = time.perf_counter() - te
        rms, good = evaluate(net, Xv, Tv, 64)
        history.append(dict(epoch=epoch, train_loss=run / steps_per_epoch, val_rms_cells=rms,
                            val_good=good, seconds=dt))
        log("epoch %d: loss %.4f, val RMS %.4f cells (%.3f px at 512), %.1f%% within 0.5 "
            "cell, %.1f s (%.0f samples/s)" % (epoch, run / steps_per_epoch, rms, rms * 4,
                                                100 * good, dt, steps_per_epoch * args.batch / dt))
        if rms < best[0]:
            best = (rms, net.get_params())
            if epoch % 5 == 0:
                _save(args.out, best[1], dict(partial=True, epoch=epoch, best_val_rms_cells=rms))
        if time.perf_counter() - t0 > budget or step >= total_steps:
            break
    meta = dict(series=args.series, frames=args.frames, seeds=[args.seed0,
                args.seed0 + args.series - 1], val_series=args.val_series, batch=args.batch,
                sides=sorted({sp.side for sp, _ in specs}), mix=args.mix,
                lr=args.lr, epochs=len(history), best_val_rms_cells=best[0],
                train_seconds=time.perf_counter() - t0, history=history)
    _save(args.out, best[1], meta)
    log("saved %s (best val RMS %.4f cells)" % (args.out, best[0]))
    net.set_params(best[1])
    meta["warm_vs_cold"] = warm_vs_cold(
        net, val_frames, P.Params(levels=specs[-1][1], scan="brent_kung"))[0]
    _save(args.out, best[1], meta)


def warm_vs_cold(net, frames, params, border=16):
    """Neighbour registrations of a validation series, cold and warm (both modes): time,
    fallbacks and the RMS difference (pixels) over the interior."""
    import torch
    import paper_1712_02533_amd as P
    ref = np.arange(frames.shape[0] - 1, dtype=np.int32)
    out = {}
    for mode in ("cold", "refine", "skip", "cold"):
        P.set_warm_start(None if mode == "cold" else net, mode="refine" if mode == "cold" else mode)
        torch.cuda.synchronize()
        t = time.perf_counter()
        u, st = P.register_pairs(frames, ref, ref + 1, params=params)
        torch.cuda.synchronize()
        out[mode] = (u, st, time.perf_counter() - t)   # the second cold run is timed warm
    P.set_warm_start(None)
    res = dict(pairs=len(ref), cold_s=out["cold"][2],
               cold_iters=np.sum([s.iters for s in out["cold"][1]], axis=0).tolist())
    for mode in ("refine", "skip"):
        d = (out[mode][0] - out["cold"][0])[:, :, border:-border, border:-border]
        per_pair = d.pow(2).mean(dim=(1, 2, 3)).sqrt().cpu().numpy()
        res[mode] = dict(seconds=out[mode][2], rms_px=float(d.pow(2).mean().sqrt()),
                         pairs_over_005=int((per_pair > 0.05).sum()),
                         worst_pair_rms_px=float(per_pair.max()),
                         fallbacks=sum(1 for s in out[mode][1] if s.flags & 4),
                         iters=np.sum([s.iters for s in out[mode][1]], axis=0).tolist())
    log("warm vs cold on %d validation pairs: %s" % (len(ref), json.dumps(res)))
    return res, out


def evaluate_only(args):
    """Warm vs cold of saved weights on fresh series (seed args.seed0): one series with the
    512 x 512 workload's statistics, or with --mix one per side of the mixed workload. Accuracy
    against the generator's analytic displacement on a sample of pairs."""
    import torch
    import paper_1712_02533_amd as P
    from synth import make_series, ground_truth_pair
    dev = torch.device("cuda", 0)
    net = P.WarmStartNet(device=dev)
    net.load(args.init)
    results = []
    specs = series_specs(4 if args.mix else 1, args.frames, args.seed0, args.mix)
    for spec, levels in specs:
        params = P.Params(levels=levels, scan="brent_kung")
        series = make_series(spec, workers=args.workers)
        frames = torch.tensor(series.frames, device=dev)
        n = spec.n_frames
        ref = np.arange(n - 1, dtype=np.int32)
        X = P.pair_inputs(frames, ref, ref + 1)
        u, _ = P.register_pairs(frames, ref, ref + 1, params=params)
        rms, good = evaluate(net, X, P.level7_targets(u), 64)
        log("side %d seed %d: prediction RMS %.4f cells, %.1f%% within 0.5 cell" %
            (spec.side, spec.seed, rms, 100 * good))
        res, out = warm_vs_cold(net, frames, params)
        res.update(side=spec.side, seed=spec.seed, prediction_rms_cells=rms,
                   prediction_within_half_cell=good)
        b = max(8, spec.side // 20)
        sample = list(range(0, len(ref), max(1, len(ref) // 16)))[:16]
        err = {k: [] for k in ("cold", "refine", "skip")}
        for m in sample:
            g = torch.tensor(ground_truth_pair(series, m, m + 1), device=dev, dtype=torch.float32)
            for mode in err:
                e = (out[mode][0][m] - g)[:, b:-b, b:-b]
                err[mode].append(float(e.pow(2).mean().sqrt()))
        res["truth_rms_px"] = {k: dict(mean=float(np.mean(v)), off_by_1px=int(np.sum(
            np.array(v) > 1.0)), pairs=len(v)) for k, v in err.items()}
        log("side %d: RMS error vs truth %s" % (spec.side, json.dumps(res["truth_rms_px"])))
        results.append(res)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(results, f, indent=1)


def _save(path, params, meta):
    from safetensors.numpy import save_file
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    save_file({"params": np.ascontiguousarray(params, dtype=np.float32)}, path)
    with open(os.path.splitext(path)[0] + ".json", "w") as f:
        json.dump(meta, f, indent=1)


if __name__ == "__main__":
    main()
