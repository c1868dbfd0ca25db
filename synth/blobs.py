"""Blob-lattice micrograph series generator.

A frame is a square lattice of Gaussian blobs (the "object") seen through a per-frame rigid
drift and a smooth non-rigid displacement, then sampled with Poisson counting noise. It stands
in for the HRTEM frame series the paper registers (Electron microscopy data section), which is
not available. The draw order below is part of the definition: a given seed always yields the
same frames.

Coordinates: pixel (row r, column c) sits at the point (x, y) = (c, r) in pixel units, which is
also the position of grid node (r, c) at the finest level. Displacements are (x, y) pairs.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

N_SINES = 4


@dataclass(frozen=True)
class SeriesSpec:
    n_frames: int
    side: int
    drift: float            # D: per-frame translation drawn from U[-D, D]^2 (px)
    warp_amp: float         # A: 4 sinusoids with amplitudes U[0, A/4] each (px)
    mean_counts: float      # mu: mean Poisson count of frame 0; <= 0 means noise-free
    seed: int
    spacing: float = 6.0    # lattice spacing (px)
    blob_sigma: float = 1.5 # Gaussian blob width (px)
    wavelength: tuple = (32.0, 128.0)


@dataclass
class Series:
    spec: SeriesSpec
    frames: np.ndarray                 # [N, side, side] float32 counts (or clean intensities)
    shifts: np.ndarray                 # [N, 2] per-frame translation t_k (x, y) px
    sines: np.ndarray                  # [N, 4, 6]: alpha, Lambda, n_angle, e_angle, theta, unused
    origin: np.ndarray = field(repr=False, default=None)
    amps: np.ndarray = field(repr=False, default=None)
    lattice_lo: tuple = (0, 0)
    kappa: float = 1.0


def _warp(sines_k: np.ndarray, x: np.ndarray, y: np.ndarray):
    """s_k(x): sum of N_SINES sinusoids alpha * e * sin(2 pi <n, x> / Lambda + theta)."""
    sx = np.zeros_like(x)
    sy = np.zeros_like(y)
    for m in range(N_SINES):
        alpha, lam, an, ae, th = sines_k[m, :5]
        if alpha == 0.0:
            continue
        ph = 2.0 * math.pi * (math.cos(an) * x + math.sin(an) * y) / lam + th
        s = np.sin(ph)
        sx += alpha * math.cos(ae) * s
        sy += alpha * math.sin(ae) * s
    return sx, sy


def _lattice(spec: SeriesSpec, origin, amps, lo, px, py):
    """L(p) = sum of a_pq exp(-|p - c_pq|^2 / (2 sigma^2)) over the 4x4 blobs nearest to p
    (every blob within 5 sigma of p for the default spacing and width)."""
    s = spec.spacing
    inv2s2 = 1.0 / (2.0 * spec.blob_sigma ** 2)
    fx = (px - origin[0]) / s
    fy = (py - origin[1]) / s
    ix0 = np.floor(fx).astype(np.int64)
    iy0 = np.floor(fy).astype(np.int64)
    rx = (fx - ix0) * s          # offset of p from blob column ix0 (px)
    ry = (fy - iy0) * s
    ny, nx = amps.shape
    jx0 = ix0 - lo[0]
    jy0 = iy0 - lo[1]
    if jx0.min() - 1 < 0 or jx0.max() + 2 >= nx or jy0.min() - 1 < 0 or jy0.max() + 2 >= ny:
        raise ValueError("lattice margin too small for the requested displacement")
    offs = (-1, 0, 1, 2)
    ex = [np.exp(-(rx - s * d) ** 2 * inv2s2) for d in offs]
    ey = [np.exp(-(ry - s * d) ** 2 * inv2s2) for d in offs]
    flat = amps.ravel()
    base = jy0 * nx + jx0
    out = np.zeros_like(px)
    for a, dy in enumerate(offs):
        row = np.zeros_like(px)
        for b, dx in enumerate(offs):
            row += flat[base + (dy * nx + dx)] * ex[b]
        out += row * ey[a]
    return out


def _clean_frame(spec, origin, amps, lo, shift, sines_k):
    side = spec.side
    r, c = np.meshgrid(np.arange(side, dtype=np.float64), np.arange(side, dtype=np.float64),
                       indexing="ij")
    sx, sy = _warp(sines_k, c, r)
    return _lattice(spec, origin, amps, lo, c - shift[0] - sx, r - shift[1] - sy)


def _noise_rng(spec: SeriesSpec, k: int) -> np.random.Generator:
    """Counting noise of frame k comes from its own stream, so frames can be drawn in any order."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([spec.seed, 7919, k])))


def make_series(spec: SeriesSpec, noise: bool = True, workers: int = 0) -> Series:
    """Draw a series. The main stream gives the lattice origin, the blob amplitudes, then per
    frame the shift and the sinusoid parameters. Frame k's Poisson counts (scaled so that frame 0
    has mean `mean_counts`) come from a stream of its own. `workers` > 1 evaluates frames on
    that many threads; the result does not depend on it."""
    rng = np.random.Generator(np.random.PCG64(spec.seed))
    s = spec.spacing
    origin = rng.uniform(0.0, s, size=2)
    margin = spec.drift + spec.warp_amp + 5.0 * spec.blob_sigma + 3.0 * s
    lo_i = int(math.floor((-margin - s) / s)) - 1
    hi_i = int(math.ceil((spec.side - 1 + margin + s) / s)) + 1
    count = hi_i - lo_i + 1
    amps = rng.uniform(0.5, 1.0, size=(count, count))
    lo = (lo_i, lo_i)
    shifts = np.zeros((spec.n_frames, 2))
    sines = np.zeros((spec.n_frames, N_SINES, 6))
    for k in range(spec.n_frames):
        shifts[k] = rng.uniform(-spec.drift, spec.drift, size=2)
        for m in range(N_SINES):
            sines[k, m, 0] = rng.uniform(0.0, spec.warp_amp / N_SINES)
            sines[k, m, 1] = rng.uniform(spec.wavelength[0], spec.wavelength[1])
            sines[k, m, 2] = rng.uniform(0.0, 2.0 * math.pi)
            sines[k, m, 3] = rng.uniform(0.0, 2.0 * math.pi)
            sines[k, m, 4] = rng.uniform(0.0, 2.0 * math.pi)
    frames = np.empty((spec.n_frames, spec.side, spec.side), dtype=np.float32)
    use_noise = noise and spec.mean_counts > 0
    clean0 = _clean_frame(spec, origin, amps, lo, shifts[0], sines[0])
    kappa = spec.mean_counts / clean0.mean() if use_noise else 1.0

    def one(k):
        clean = clean0 if k == 0 else _clean_frame(spec, origin, amps, lo, shifts[k], sines[k])
        if use_noise:
            frames[k] = _noise_rng(spec, k).poisson(kappa * clean).astype(np.float32)
        else:
            frames[k] = clean.astype(np.float32)

    if workers and workers > 1 and spec.n_frames > 1:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(max_workers=workers) as ex:
            list(ex.map(one, range(spec.n_frames)))
    else:
        for k in range(spec.n_frames):
            one(k)
    return Series(spec, frames, shifts, sines, origin, amps, lo, kappa)


def ground_truth(series: Series, k: int, iters: int = 60) -> np.ndarray:
    """Analytic u_{0,k} in pixels, shape [2, side, side] (plane 0: x, plane 1: y).

    phi_{0,k}(x) = y solves y = x + t_k - t_0 - s_0(x) + s_k(y), so that frame k sampled at
    phi(x) shows what frame 0 shows at x. Solved by fixed-point iteration (s_k is a
    contraction because its Lipschitz constant is below 0.3 for the specified amplitudes).
    """
    side = series.spec.side
    r, c = np.meshgrid(np.arange(side, dtype=np.float64), np.arange(side, dtype=np.float64),
                       indexing="ij")
    t = series.shifts
    s0x, s0y = _warp(series.sines[0], c, r)
    bx = c + t[k, 0] - t[0, 0] - s0x
    by = r + t[k, 1] - t[0, 1] - s0y
    yx, yy = bx.copy(), by.copy()
    for _ in range(iters):
        skx, sky = _warp(series.sines[k], yx, yy)
        yx, yy = bx + skx, by + sky
    return np.stack([yx - c, yy - r])


def ground_truth_pair(series: Series, i: int, k: int, iters: int = 60) -> np.ndarray:
    """Analytic u_{i,k} in pixels, [2, side, side]: y = x + t_k - t_i - s_i(x) + s_k(y), so that
    frame k sampled at x + u(x) shows what frame i shows at x (same fixed point as above)."""
    side = series.spec.side
    r, c = np.meshgrid(np.arange(side, dtype=np.float64), np.arange(side, dtype=np.float64),
                       indexing="ij")
    t = series.shifts
    six, siy = _warp(series.sines[i], c, r)
    bx = c + t[k, 0] - t[i, 0] - six
    by = r + t[k, 1] - t[i, 1] - siy
    yx, yy = bx.copy(), by.copy()
    for _ in range(iters):
        skx, sky = _warp(series.sines[k], yx, yy)
        yx, yy = bx + skx, by + sky
    return np.stack([yx - c, yy - r])


# Workload recipes. Levels are listed finest first; "scan" is the schedule of the series step.
CONFIGS = {
    "tiny64": dict(spec=SeriesSpec(8, 64, 2.0, 0.0, 20.0, 0), levels=2, scan="sequential"),
    "series256": dict(spec=SeriesSpec(64, 256, 4.0, 1.0, 10.0, 1), levels=3, scan="brent_kung"),
    "series512": dict(spec=SeriesSpec(512, 512, 8.0, 1.5, 5.0, 2), levels=4, scan="brent_kung"),
}


def config_spec(name: str):
    return CONFIGS[name]


def uneven_batch(seed: int = 3, n_series: int = 16):
    """Config of 16 independent series with mixed sides and lengths (segmented scan input)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(n_series):
        side = int(rng.choice([128, 256, 512, 1024]))
        n = int(rng.integers(32, 513))
        mu = float(rng.uniform(2.0, 20.0))
        sub_seed = int(rng.integers(0, 2 ** 31 - 1))
        levels = int(math.log2(side)) - 6 + 1
        out.append(dict(spec=SeriesSpec(n, side, 8.0, 1.5, mu, sub_seed), levels=levels,
                        scan="brent_kung"))
    return out
