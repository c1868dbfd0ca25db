"""Autotuner of the launch shape (pprs_tuning) for a series workload.

The launch shape never changes a result (the library sums every tile's partials in a fixed
order and each slot's decisions are its own), so the tuner is free to pick the fastest:
coordinate descent over the knobs, each candidate timed with HIP events on a series with the
statistics of the target (a prefix of the caller's frames), best of `repeats` runs. The choice
is cached per (side, levels, scan, frames) in a JSON file.

    from paper_1712_02533_amd import autotune
    best = autotune.tune(frames, params)        # applies and returns the best shape
"""
from __future__ import annotations

import json
import os
import time

CANDIDATES = {
    "ladder_rungs": [2, 1],
    "tile_grad": [0, 3, 4, 2],
    "smooth_lines": [32, 8, 16],
    "pool_group": [16, 32, 8],
    "grid_grad": [8192, 4096, 2048],
    "grid_energy": [8192, 16384, 4096],
    "grid_smooth": [8192, 16384, 4096],
    "pool_slots": [256, 512, 1024],
}
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "pprs", "tuning.json")


def _key(frames, params):
    N, H, _ = frames.shape
    return "side%d_levels%d_scan%s_frames%d" % (H, params.levels, params.scan, N)


def _time_series(P, frames, params, repeats):
    import torch
    best = float("inf")
    for _ in range(repeats):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P.prefix_register_series(frames, params=params)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    return best


def tune(frames, params, max_frames: int = 128, repeats: int = 2, cache: str | None = None,
         log=None, apply: bool = True) -> dict:
    """Finds the fastest launch shape for series like `frames` (device [N, H, W]) with
    `params`; tunes on the first `max_frames` frames. Returns the shape (and applies it)."""
    import paper_1712_02533_amd as P
    cache = cache or DEFAULT_CACHE
    sub = frames[:max_frames].contiguous()
    key = _key(sub, params)
    table = {}
    if os.path.exists(cache):
        try:
            table = json.load(open(cache))
        except (OSError, ValueError):
            table = {}
    if key in table:
        best = table[key]["tuning"]
        if apply:
            P.set_tuning(best)
        return best
    say = log or (lambda *a: None)
    cur = P.get_tuning()
    P.prefix_register_series(sub, params=params)        # warm-up: allocations, first launches
    base = _time_series(P, sub, params, repeats)
    say("autotune %s: default %.1f ms" % (key, 1e3 * base))
    best_t = base
    for knob, values in CANDIDATES.items():
        for v in values:
            if v == cur[knob]:
                continue
            trial = dict(cur, **{knob: v})
            P.set_tuning(trial)
            t = _time_series(P, sub, params, repeats)
            say("  %s=%d: %.1f ms" % (knob, v, 1e3 * t))
            if t < best_t * 0.99:
                best_t, cur = t, trial
        P.set_tuning(cur)
    say("autotune %s: %.1f ms -> %.1f ms with %s" % (key, 1e3 * base, 1e3 * best_t, cur))
    table[key] = dict(tuning=cur, ms=1e3 * best_t, default_ms=1e3 * base)
    try:
        os.makedirs(os.path.dirname(cache), exist_ok=True)
        with open(cache, "w") as f:
            json.dump(table, f, indent=1)
    except OSError:
        pass
    if not apply:
        P.set_tuning({k: 0 for k in cur})
    return cur
