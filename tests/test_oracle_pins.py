"""Pins of the FP64 oracle against what the paper and mathematics fix (no GPU).

Every test checks the oracle against something other than itself: closed-form integrals,
library routines (scipy's bilinear interpolation with edge replication, dense numpy solves,
numerically integrated hat functions), invariants (NCC bounds, Armijo decrease, monotone
energy), values printed in the paper (tests/golden/paper_values.json) and the analytic ground
truth of the synthetic generator.
"""
import json
import os

import numpy as np
import pytest
from scipy import ndimage

import oracle as O
from synth import SeriesSpec, ground_truth, make_series

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
GP = np.array([(1 - 1 / np.sqrt(3)) / 2, (1 + 1 / np.sqrt(3)) / 2])


def grid(n):
    x = np.linspace(0.0, 1.0, n)
    X, Y = np.meshgrid(x, x)  # X varies along columns (x), Y along rows (y)
    return X, Y


# ------------------------------------------------------------------------------------------
# Restriction / prolongation (Multilevel section)

@pytest.mark.parametrize("n", [5, 9, 17, 33])
def test_restriction_constants_and_affine_interior(n):
    X, Y = grid(n)
    c = np.full((n, n), 3.25)
    assert np.allclose(O.restrict(c), 3.25, atol=1e-14)
    f = 0.7 * X - 1.3 * Y + 0.2
    r = O.restrict(f)
    Xc, Yc = grid((n - 1) // 2 + 1)
    assert np.abs(r - (0.7 * Xc - 1.3 * Yc + 0.2))[1:-1, 1:-1].max() < 1e-13


def test_restriction_interior_matches_library_correlation():
    rng = np.random.default_rng(1)
    f = rng.normal(size=(17, 17))
    k = np.outer([1, 2, 1], [1, 2, 1]) / 16.0
    full = ndimage.correlate(f, k, mode="constant")
    ref = full[::2, ::2]
    assert np.abs(O.restrict(f) - ref)[1:-1, 1:-1].max() < 1e-13


@pytest.mark.parametrize("nc", [3, 5, 9, 17])
def test_prolongation_exact_for_affine_and_inverse_of_restriction(nc):
    Xc, Yc = grid(nc)
    nf = 2 * (nc - 1) + 1
    Xf, Yf = grid(nf)
    f = -0.4 * Xc + 2.1 * Yc + 0.5
    p = O.prolong(f)
    assert np.abs(p - (-0.4 * Xf + 2.1 * Yf + 0.5)).max() < 1e-13
    assert np.abs(O.restrict(p) - f)[1:-1, 1:-1].max() < 1e-13


def test_prolongation_matches_library_bilinear_zoom():
    rng = np.random.default_rng(2)
    c = rng.normal(size=(9, 9))
    ref = ndimage.zoom(c, (17 - 1) / (9 - 1) + 1e-12, order=1, grid_mode=False)
    ref = ndimage.map_coordinates(c, np.mgrid[0:17, 0:17] / 2.0, order=1)
    assert np.abs(O.prolong(c) - ref).max() < 1e-13


# ------------------------------------------------------------------------------------------
# Clamped bilinear evaluation

def test_bilinear_affine_exact_and_nodes_and_clamp():
    n = 9
    X, Y = grid(n)
    g = 1.5 * X - 0.25 * Y + 0.125
    rng = np.random.default_rng(3)
    for _ in range(50):
        px, py = rng.uniform(0, 1, 2)
        v, gx, gy = O.bilinear(g, px, py)
        assert abs(v - (1.5 * px - 0.25 * py + 0.125)) < 1e-13
        assert abs(gx - 1.5) < 1e-12 and abs(gy + 0.25) < 1e-12
    h = 1.0 / (n - 1)
    f = rng.normal(size=(n, n))
    for a in range(n):
        for b in range(n):
            assert O.bilinear(f, b * h, a * h)[0] == f[a, b]
    # outside the domain: replicated value, zero derivative across the violated axis
    v, gx, gy = O.bilinear(g, 1.7, 0.5)
    assert abs(v - (1.5 - 0.125 + 0.125)) < 1e-13 and gx == 0.0 and abs(gy + 0.25) < 1e-12
    v, gx, gy = O.bilinear(g, 0.5, -0.3)
    assert abs(v - (0.75 + 0.125)) < 1e-13 and gy == 0.0


def test_bilinear_matches_library_with_edge_replication():
    rng = np.random.default_rng(4)
    n = 17
    f = rng.normal(size=(n, n))
    pts = rng.uniform(-0.2, 1.2, size=(200, 2))
    h = 1.0 / (n - 1)
    ref = ndimage.map_coordinates(f, [np.clip(pts[:, 1] / h, 0, n - 1),
                                      np.clip(pts[:, 0] / h, 0, n - 1)], order=1, mode="nearest")
    got = np.array([O.bilinear(f, px, py)[0] for px, py in pts])
    assert np.abs(got - ref).max() < 1e-12


# ------------------------------------------------------------------------------------------
# FE matrices (Spatial discretization section)

def _hat_matrices_1d(n):
    """M1, K1 by numerical integration of the 1-D hat functions (5-point Gauss per cell)."""
    h = 1.0 / (n - 1)
    xg, wg = np.polynomial.legendre.leggauss(5)
    M = np.zeros((n, n))
    K = np.zeros((n, n))
    for c in range(n - 1):
        x = c * h + (xg + 1) / 2 * h
        w = wg / 2 * h
        phi = {c: 1 - (x - c * h) / h, c + 1: (x - c * h) / h}
        dphi = {c: -1 / h, c + 1: 1 / h}
        for i in phi:
            for j in phi:
                M[i, j] += np.sum(w * phi[i] * phi[j])
                K[i, j] += np.sum(w * dphi[i] * dphi[j])
    return M, K


@pytest.mark.parametrize("n", [3, 5, 9])
def test_mass_and_stiffness_match_integrated_basis(n):
    M1, K1 = _hat_matrices_1d(n)
    M = np.kron(M1, M1)
    K = np.kron(K1, M1) + np.kron(M1, K1)
    rng = np.random.default_rng(5)
    f = rng.normal(size=(n, n))
    assert np.abs(O.mass_apply(f).ravel() - M @ f.ravel()).max() < 1e-13
    assert np.abs(O.stiff_apply(f).ravel() - K @ f.ravel()).max() < 1e-12


def test_fe_integrals_closed_forms():
    n = 17
    X, Y = grid(n)
    one = np.ones((n, n))
    assert abs(O.mass_apply(one).sum() - 1.0) < 1e-14           # |Omega| = 1
    assert abs((O.mass_apply(X) * one).sum() - 0.5) < 1e-14     # int x = 1/2
    xy = X * Y
    assert abs((xy * O.mass_apply(xy)).sum() - 1.0 / 9.0) < 1e-14  # int (xy)^2 = 1/9
    u = 2.0 * X + 3.0 * Y
    assert abs((u * O.stiff_apply(u)).sum() - 13.0) < 1e-11     # int |grad u|^2
    assert abs((xy * O.stiff_apply(xy)).sum() - 2.0 / 3.0) < 1e-12
    assert np.abs(O.stiff_apply(one)).max() < 1e-11             # constants have no energy


# ------------------------------------------------------------------------------------------
# Normalisation, NCC, energy

def _frames(side=16, seed=7, drift=1.0, noise=0.0):
    s = make_series(SeriesSpec(2, side, drift, 0.0, noise, seed))
    return s, O.frame_to_nodes(s.frames[0]), O.frame_to_nodes(s.frames[1])


def _energy_numpy(R, T, u, lam):
    """Independent quadrature energy with scipy's bilinear interpolation (edge replication)."""
    n = R.shape[0]
    h = 1.0 / (n - 1)
    Rn, m, sg = O.normalize(R)
    a, b, p, q = np.meshgrid(np.arange(n - 1), np.arange(n - 1), [0, 1], [0, 1], indexing="ij")
    rows = a + GP[p]
    cols = b + GP[q]
    ux = ndimage.map_coordinates(u[0], [rows, cols], order=1)
    uy = ndimage.map_coordinates(u[1], [rows, cols], order=1)
    rq = ndimage.map_coordinates(Rn, [rows, cols], order=1)
    tr = np.clip(rows + uy / h, 0, n - 1)
    tc = np.clip(cols + ux / h, 0, n - 1)
    tq = ndimage.map_coordinates(T, [tr, tc], order=1, mode="nearest")
    w = h * h / 4
    mean = w * tq.sum()
    sig = np.sqrt(w * ((tq - mean) ** 2).sum())
    ncc = w * (rq * (tq - mean)).sum() / sig
    M1, K1 = _hat_matrices_1d(n)
    K = np.kron(K1, M1) + np.kron(M1, K1)
    reg = sum(u[c].ravel() @ K @ u[c].ravel() for c in range(2))
    return -ncc + 0.5 * lam * reg, ncc


def test_energy_matches_independent_quadrature():
    _, R, T = _frames()
    n = R.shape[0]
    rng = np.random.default_rng(8)
    for trial in range(3):
        u = rng.normal(0, 1.5 / (n - 1), size=(2, n, n))
        e, ncc = O.energy(R, T, u, 0.37)
        e2, ncc2 = _energy_numpy(R, T, u, 0.37)
        assert abs(ncc - ncc2) < 1e-12 and abs(e - e2) < 1e-11


def test_ncc_invariants_and_bounds():
    _, R, T = _frames()
    n = R.shape[0]
    z = np.zeros((2, n, n))
    assert abs(O.energy(R, R, z, 1.0)[1] - 1.0) < 1e-13            # perfect match
    assert abs(O.energy(R, 3.0 * R + 7.0, z, 1.0)[1] - 1.0) < 1e-13
    assert abs(O.energy(R, -2.0 * R + 1.0, z, 1.0)[1] + 1.0) < 1e-13  # sign(a)
    rng = np.random.default_rng(9)
    for _ in range(5):
        u = rng.normal(0, 2.0 / (n - 1), size=(2, n, n))
        ncc = O.energy(R, T, u, 0.0)[1]
        assert GOLD["ncc_bounds"]["min"] <= ncc <= GOLD["ncc_bounds"]["max"]
    # at u = 0 the 2x2 Gauss rule is exact for Q1 x Q1: NCC = R~^T M T~ (mass-matrix form)
    M1, _ = _hat_matrices_1d(n)
    M = np.kron(M1, M1)
    Rn = O.normalize(R)[0].ravel()
    Tn = O.normalize(T)[0].ravel()
    assert abs(O.energy(R, T, z, 0.0)[1] - Rn @ M @ Tn) < 1e-13
    # constant displacements carry no Dirichlet energy
    e0 = O.energy(R, T, np.full((2, n, n), 0.013), 5.0)
    e1 = O.energy(R, T, np.full((2, n, n), 0.013), 0.0)
    assert abs(e0[0] - e1[0]) < 1e-13


def _rectangle(n, cx, sigma_px=1.5):
    """Smoothed 0.5 x 0.5 rectangle with its lower-left corner at (cx, 0.25)."""
    X, Y = grid(n)
    side = n - 1
    inside = ((X >= cx) & (X <= cx + 0.5) & (Y >= 0.25) & (Y <= 0.75)).astype(float)
    return ndimage.gaussian_filter(inside, sigma_px, mode="nearest")


def test_rectangle_worked_example_sign_convention():
    """f1(x + G) = f0(x) with G = (0.25, 0) for the centred / right-shifted rectangle."""
    ex = GOLD["rectangle_example"]
    n = 65
    f0 = _rectangle(n, ex["lower_left_f0"][0])
    f1 = _rectangle(n, ex["lower_left_f1"][0])
    G = np.array(ex["G"])
    up = np.stack([np.full((n, n), G[0]), np.full((n, n), G[1])])
    e_plus, ncc_plus = O.energy(f0, f1, up, 1.0)
    e_minus, _ = O.energy(f0, f1, -up, 1.0)
    assert e_plus < e_minus
    # along the x-translation line the energy is lowest at +G (sign convention f1(x+G) = f0(x));
    # the rectangle of f1 touches the right border, so the clamped sample is not a perfect match
    ts = np.linspace(-0.4, 0.4, 65)
    es = [O.energy(f0, f1, np.stack([np.full((n, n), t), np.zeros((n, n))]), 1.0)[0] for t in ts]
    assert abs(ts[int(np.argmin(es))] - G[0]) <= 1.0 / (n - 1) + 1e-12
    u, st, _ = O.register(f0, f1, O.Params(levels=4, lam=10.0, eps=1e-6))
    X, Y = grid(n)
    inside = (X >= 0.3) & (X <= 0.7) & (Y >= 0.3) & (Y <= 0.7)
    # registering from the identity finds +G inside the rectangle (within 2 of its 16 px; the
    # rectangle of f1 touches the border, where clamped sampling pulls the field)
    assert abs(u[0][inside].mean() - G[0]) < 2.0 / (n - 1)
    assert abs(u[1][inside].mean() - G[1]) < 2.0 / (n - 1)


# ------------------------------------------------------------------------------------------
# Gradient and metric

def test_gradient_matches_central_differences():
    _, R, T = _frames(side=16, seed=3)
    n = R.shape[0]
    rng = np.random.default_rng(0)
    u = rng.normal(0, 0.3 / (n - 1), size=(2, n, n))
    lam = 0.7
    G = O.gradient(R, T, u, lam)
    fd = np.zeros_like(u)
    eps = 1e-7
    for c in range(2):
        for i in range(n):
            for j in range(n):
                up = u.copy()
                up[c, i, j] += eps
                um = u.copy()
                um[c, i, j] -= eps
                fd[c, i, j] = (O.energy(R, T, up, lam)[0] - O.energy(R, T, um, lam)[0]) / (2 * eps)
    assert np.abs(G - fd).max() < 1e-6 * np.abs(G).max()


@pytest.mark.parametrize("n,beta", [(5, 0.0), (9, 1.0), (9, 3.0)])
def test_metric_solve_matches_dense(n, beta):
    M1, K1 = _hat_matrices_1d(n)
    h = 1.0 / (n - 1)
    S1 = M1 + (beta * h) ** 2 * K1
    A = np.kron(S1, S1)
    rng = np.random.default_rng(11)
    g = rng.normal(size=(n, n))
    d = O.smooth(g, beta)
    assert np.abs(d.ravel() - np.linalg.solve(A, g.ravel())).max() < 1e-10 * np.abs(d).max()
    assert g.ravel() @ d.ravel() > 0


# ------------------------------------------------------------------------------------------
# Gradient flow and operator A

def test_armijo_and_monotone_energy_trace():
    s, R, T = _frames(side=32, seed=5, drift=1.5, noise=20.0)
    p = O.Params(levels=2, lam=10.0, eps=1e-6)
    _, st, tr = O.register(R, T, p, trace_cap=4000)
    assert len(tr) > 3
    sigma = GOLD["armijo_sigma"]["value"]
    for level, step, tau, e0, e1, gtd, tmax, passes in tr:
        if tau > 0:
            assert e1 <= e0 - sigma * tau * gtd + 1e-15        # sufficient decrease
            assert tau <= tmax * (1 + 1e-12)
        else:
            assert e1 == e0
    # energy never increases within a level
    for lv in np.unique(tr[:, 0]):
        t = tr[tr[:, 0] == lv]
        assert np.all(np.diff(np.concatenate([t[:1, 3], t[:, 4]])) <= 1e-15)


def _replay_level_state(R, T, p, u0, k):
    """State of the one-level flow after its first k accepted steps (the flow is deterministic,
    so capping iter_max at k stops it exactly there)."""
    if k == 0:
        return np.array(u0, dtype=np.float64)
    q = O.Params(**{**p.__dict__, "iter_max": k})
    return O.gradient_flow(R, T, u0, q)[0]


@pytest.mark.parametrize("seed,drift,noise,cap", [(21, 1.5, 20.0, 1.0), (22, 2.5, 0.0, 1.0),
                                                  (23, 2.0, 20.0, 64.0)])
def test_line_search_takes_the_largest_passing_step(seed, drift, noise, cap):
    """Armijo with widening (Gradient flow subsection): the accepted step is the largest step of
    the ladder top * 2^-j that satisfies the sufficient-decrease test, top = min(2^K tau_prev,
    tau_max), tau_max = cap h / max|d|. Every state of the flow is rebuilt and the direction,
    G.d and every rung larger than the accepted one are re-evaluated with the pinned energy,
    gradient and metric solve: a ladder walked smallest-first, a wrong top or a wrong tau_max
    fails here. A cap of 64 cells makes the first pass of the ladder fail, so the later passes
    (each 2K+1 halvings below the previous one) are checked too."""
    _, R, T = _frames(side=32, seed=seed, drift=drift, noise=noise)
    n = R.shape[0]
    h = 1.0 / (n - 1)
    p = O.Params(levels=1, lam=10.0, eps=1e-7, iter_max=40, cap=cap)
    u0 = np.zeros((2, n, n))
    _, steps, _, _, tr, _ = O.gradient_flow(R, T, u0, p)
    assert steps >= 8
    sigma, K = p.sigma, p.ladder_k
    tau_prev = np.inf
    below_top = multi_pass = 0
    for k, (_, step, tau, e0, e1, gtd, tmax, passes) in enumerate(tr):
        assert step == k
        u = _replay_level_state(R, T, p, u0, k)
        E = O.energy(R, T, u, p.lam)[0]
        G = O.gradient(R, T, u, p.lam)
        d = np.stack([O.smooth(G[c], p.beta) for c in range(2)])
        assert abs(E - e0) <= 1e-13
        assert abs((G * d).sum() - gtd) <= 1e-12 * abs(gtd)
        assert abs(p.cap * h / np.abs(d).max() - tmax) <= 1e-12 * tmax
        top = min(2.0 ** K * tau_prev, tmax)
        armijo = lambda t: O.energy(R, T, u - t * d, p.lam)[0] <= E - sigma * t * gtd
        if tau == 0:                                    # exhausted: every rung failed
            assert all(not armijo(top * 2.0 ** -j) for j in range(int(passes) * (2 * K + 1)))
            break
        j = np.log2(top / tau)
        assert abs(j - round(j)) < 1e-9                 # a rung of the ladder
        j = int(round(j))
        assert (2 * K + 1) * (passes - 1) <= j < (2 * K + 1) * passes
        assert armijo(tau) and abs(O.energy(R, T, u - tau * d, p.lam)[0] - e1) <= 1e-13
        for jj in range(j):                             # every larger rung was tried and failed
            assert not armijo(top * 2.0 ** -jj)
        below_top += j > 0
        multi_pass += passes > 1
        tau_prev = tau
    assert below_top >= 1                               # the maximality check did bite
    assert cap == 1.0 or multi_pass >= 1


def test_stopping_rule_energy_decrease_and_iteration_cap():
    """Stopping criteria (end of the Image registration chapter): a level stops after the first
    accepted step whose energy decrease E_k - E_{k+1} falls below eps, or after iter_max
    accepted steps, or when the line search fails. Every other step of a level decreases the
    energy by at least eps."""
    s, R, T = _frames(side=64, seed=31, drift=2.0, noise=20.0)
    for eps in (3e-4, 1e-5):
        p = O.Params(levels=3, lam=10.0, eps=eps)
        _, st, tr = O.register(R, T, p, trace_cap=8000)
        for li, lv in enumerate(range(6 - p.levels + 1, 7)):
            t = tr[tr[:, 0] == lv]
            assert len(t) == st.iters[li] + (1 if len(t) and t[-1, 2] == 0 else 0)
            dec = t[:, 3] - t[:, 4]
            acc = t[t[:, 2] > 0]
            assert np.all(acc[:-1, 3] - acc[:-1, 4] >= eps)     # non-final steps: >= eps
            last = t[-1]
            assert (last[2] == 0 or dec[-1] < eps or st.iters[li] == p.iter_max)
    # the cap: with iter_max = 3 every level takes exactly three steps and is flagged
    p = O.Params(levels=3, lam=10.0, eps=1e-12, iter_max=3)
    _, st, tr = O.register(R, T, p, trace_cap=100)
    assert st.iters == [3, 3, 3] and st.flags & 1


def test_replayed_stopping_decisions():
    """The test switch that replays stopping decisions: given the flow's own step counts it
    reproduces the flow bit for bit; given one more step on a level it takes exactly that step
    (a decrease below eps, which the energy test would have refused) and nothing else changes
    on the coarser levels."""
    s, R, T = _frames(side=64, seed=32, drift=2.0, noise=20.0)
    p = O.Params(levels=3, lam=10.0, eps=3e-4)
    u, st, tr = O.register(R, T, p, trace_cap=4000)
    uf, stf, trf = O.register(R, T, p, trace_cap=4000, force=st.iters)
    assert np.array_equal(u, uf) and st.iters == stf.iters and st.trials == stf.trials
    assert stf.tie_gap == 0.0                   # every replayed decision is the test's own
    more = list(st.iters)
    more[1] += 1
    um, stm, trm = O.register(R, T, p, trace_cap=4000, force=[None, more[1], None])
    assert stm.iters[0] == st.iters[0] and stm.iters[1] == more[1]
    lv = trm[trm[:, 0] == 5]
    assert lv[-1, 3] - lv[-1, 4] < p.eps                        # the replayed extra step
    assert not np.array_equal(um, u)
    # the gap is how far the energy test was from continuing where the flow itself stopped
    own = tr[tr[:, 0] == 5]
    assert stm.tie_gap == pytest.approx(p.eps - (own[-1, 3] - own[-1, 4]), rel=1e-12)


def test_replayed_line_search_decisions():
    """The test switch that replays line-search decisions: the flow's own ladder positions (with
    its step counts) reproduce it bit for bit with both gaps 0; replaying one step a rung lower
    than the largest passing one takes that smaller step and reports in armijo_gap how far the
    Armijo test was from accepting the rung above it (its sufficient-decrease margin)."""
    s, R, T = _frames(side=64, seed=33, drift=2.0, noise=20.0)
    p = O.Params(levels=3, lam=10.0, eps=3e-4)
    u, st, tr = O.register(R, T, p, trace_cap=4000)
    J = O.trace_rungs(tr, p)
    assert len(J) == sum(st.iters)
    ur, sr, trr = O.register(R, T, p, trace_cap=4000, force=st.iters, rungs=J)
    assert np.array_equal(u, ur) and sr.iters == st.iters and sr.trials == st.trials
    assert sr.tie_gap == 0.0 and sr.armijo_gap == 0.0
    k = 3                                     # a step of the coarsest level
    J2 = list(J)
    J2[k] += 1
    um, sm, trm = O.register(R, T, p, trace_cap=4000, force=st.iters, rungs=J2)
    assert trm[k, 2] == pytest.approx(tr[k, 2] / 2, rel=1e-15)     # half the step was taken
    assert sm.iters == st.iters and not np.array_equal(um, u)
    margin = (tr[k, 3] - p.sigma * tr[k, 2] * tr[k, 5]) - tr[k, 4]  # the refused rung's margin
    assert sm.armijo_gap >= margin > 0


def test_identical_frames_give_identity():
    _, R, _ = _frames(side=32, seed=6, noise=20.0)
    u, st, _ = O.register(R, R, O.Params(levels=3))
    assert np.all(u == 0.0)


@pytest.mark.parametrize("seed", [100, 101, 102])
def test_known_translation_recovered(seed):
    spec = SeriesSpec(2, 64, 1.5, 0.0, 0.0, seed)
    s = make_series(spec)
    u, st, _ = O.register(O.frame_to_nodes(s.frames[0]), O.frame_to_nodes(s.frames[1]),
                          O.Params(levels=3, lam=10.0, eps=3e-4))
    gt = ground_truth(s, 1)
    err = O.u_to_pixels(u, 64) - gt
    b = 8
    assert np.sqrt((err[:, b:-b, b:-b] ** 2).mean()) < 0.05


@pytest.mark.parametrize("seed", [300, 301, 302, 303])
def test_known_integer_translation_recovered_under_noise(seed):
    """A known translation under Poisson noise at a mean of 20 counts (the blob-lattice
    generator of the 64^2 configuration; two crops of one frame, shifted by a whole number of
    pixels, each with its own noise): recovered within 0.05 px RMS over the interior. At a whole
    pixel the bilinear template is sampled at its nodes at the truth, so the interpolation bias
    of the method (next test) is absent and only noise and the stopping rule remain."""
    side = 64
    s = make_series(SeriesSpec(1, 96, 0.0, 0.0, 0.0, seed))
    img = s.frames[0].astype(np.float64)
    rng = np.random.default_rng(seed)
    d = rng.integers(-2, 3, size=2)
    R = img[16:16 + side, 16:16 + side]
    T = img[16 + d[1]:16 + d[1] + side, 16 + d[0]:16 + d[0] + side]   # T(x) = R(x + d)
    k = 20.0 / img.mean()
    R = rng.poisson(k * R).astype(np.float64)
    T = rng.poisson(k * T).astype(np.float64)
    u, _, _ = O.register(O.frame_to_nodes(R), O.frame_to_nodes(T),
                         O.Params(levels=2, lam=10.0, eps=3e-4))
    err = O.u_to_pixels(u, side)[:, 8:-8, 8:-8] + d[:, None, None]      # truth: u = -d
    assert np.sqrt((err ** 2).mean()) < 0.05


def test_known_translation_recovered_under_noise():
    """The 64^2 configuration's pairs (drift U[-2, 2] px, Poisson noise at a mean of 20 counts,
    2 levels, the library defaults lambda = 10, eps = 3e-4): the recovered translation (the
    field's mean over the interior) lies within 0.1 px of t_1 - t_0 on every pair and within
    0.06 px RMS over the pairs. The bar is wider than 0.05 px because bilinear interpolation of
    the template biases the NCC optimum towards whole-pixel shifts (measured without noise on
    the same pairs: 0.04 px RMS); a dropped term or a sign error moves it by pixels."""
    errs = []
    for seed in range(100, 108):
        s = make_series(SeriesSpec(2, 64, 2.0, 0.0, 20.0, seed))
        u, _, _ = O.register(O.frame_to_nodes(s.frames[0]), O.frame_to_nodes(s.frames[1]),
                             O.Params(levels=2, lam=10.0, eps=3e-4))
        gt = ground_truth(s, 1)
        b = int(np.abs(gt).max() + 3 * 1.5 + 1)
        e = (O.u_to_pixels(u, 64) - gt)[:, b:-b, b:-b].mean(axis=(1, 2))
        errs.append(np.abs(e).max())
    errs = np.array(errs)
    assert errs.max() < 0.1 and np.sqrt((errs ** 2).mean()) < 0.06


@pytest.mark.parametrize("seed", [200, 201])
def test_smooth_nonrigid_field_recovered(seed):
    spec = SeriesSpec(2, 128, 1.0, 1.0, 0.0, seed)
    s = make_series(spec)
    u, st, _ = O.register(O.frame_to_nodes(s.frames[0]), O.frame_to_nodes(s.frames[1]),
                          O.Params(levels=3, lam=1.0, eps=1e-6))
    gt = ground_truth(s, 1)
    err = O.u_to_pixels(u, 128) - gt
    b = int(np.abs(gt).max() + 3 * 1.5 + 2)
    assert np.sqrt((err[:, b:-b, b:-b] ** 2).mean()) < 0.05


# RMS error against the analytic field over the interior on four 128^2 pairs (drift 1 px,
# non-rigid amplitude 1 px, no noise, 3 levels), per (lambda, eps): the bar each setting must
# meet on every pair (measured maxima: 0.087, 0.072, 0.071, 0.060 px). The library defaults are
# lambda = 10, eps = 3e-4; smaller eps and lambda trade work for accuracy down to the 0.05 px
# the tighter settings reach on most pairs.
NONRIGID_TABLE = [((10.0, 3e-4), 0.10), ((10.0, 1e-6), 0.08), ((1.0, 3e-4), 0.08),
                  ((1.0, 1e-6), 0.07)]


@pytest.mark.parametrize("setting,bar", NONRIGID_TABLE)
def test_smooth_nonrigid_accuracy_table(setting, bar):
    """Smooth non-rigid recovery at the library defaults and at tighter settings: every pair
    within the table's bar, and at most half the RMS of the field's non-rigid part (what is
    left after its mean translation), so the non-rigid part is recovered and not only the
    shift."""
    lam, eps = setting
    for seed in (200, 201, 202, 203):
        s = make_series(SeriesSpec(2, 128, 1.0, 1.0, 0.0, seed))
        u, _, _ = O.register(O.frame_to_nodes(s.frames[0]), O.frame_to_nodes(s.frames[1]),
                             O.Params(levels=3, lam=lam, eps=eps))
        gt = ground_truth(s, 1)
        b = int(np.abs(gt).max() + 3 * 1.5 + 2)
        g = gt[:, b:-b, b:-b]
        err = np.sqrt(((O.u_to_pixels(u, 128)[:, b:-b, b:-b] - g) ** 2).mean())
        nonrigid = np.sqrt(((g - g.mean(axis=(1, 2))[:, None, None]) ** 2).mean())
        print("lambda %g eps %g seed %d: rms err %.4f px, non-rigid part %.3f px"
              % (lam, eps, seed, err, nonrigid))
        assert err < bar and err < 0.5 * nonrigid


def test_start_level_variant_reduces_to_multilevel_and_skips_levels():
    """Started on the coarsest level with the restricted guess, the start-level variant is the
    multilevel algorithm itself; started on a finer level from the true (constant) shift it
    recovers the translation with no work on the skipped levels."""
    spec = SeriesSpec(2, 64, 1.5, 0.0, 0.0, 103)
    s = make_series(spec)
    R, T = O.frame_to_nodes(s.frames[0]), O.frame_to_nodes(s.frames[1])
    p = O.Params(levels=3, lam=10.0, eps=3e-4)
    u0 = np.zeros((2, 65, 65))
    u0[0], u0[1] = 0.4 / 64, -0.3 / 64
    ua, sa, _ = O.register(R, T, p, u0=u0)
    c = np.stack([O.restrict(O.restrict(u0[k])) for k in range(2)])
    ub, sb, _ = O.register_from(R, T, 4, c, p)
    assert np.array_equal(ua, ub) and sa.iters == sb.iters
    gt = ground_truth(s, 1)
    shift = gt[:, 32, 32]
    us = np.zeros((2, 33, 33))
    us[0], us[1] = shift[0] / 64, shift[1] / 64
    u, st, _ = O.register_from(R, T, 5, us, p)
    assert st.iters[0] == 0 and st.iters[1] >= 0
    err = O.u_to_pixels(u, 64) - gt
    assert np.sqrt((err[:, 8:-8, 8:-8] ** 2).mean()) < 0.05
    # identical frames from the identity on any start level stay exactly at the identity
    z, _, _ = O.register_from(R, R, 5, np.zeros((2, 33, 33)), p)
    assert np.all(z == 0)
    with pytest.raises(ValueError):
        O.register_from(R, T, 3, np.zeros((2, 9, 9)), p)


def test_long_registration_sensitivity_to_fp32_level_perturbation():
    """Derived tolerance for long registrations: a pair four frames' drift apart (about 230
    accepted steps over 3 levels) is sensitive to perturbations at the level of FP32
    arithmetic. Relative noise of 1e-6 and 2e-6 on the template (four draws each) leaves the
    line-search decisions unchanged on most draws; with unchanged decisions the result moves by
    up to ~2.4e-4 px RMS, ~1.1e-3 px at the 99.9th percentile and by more than 1e-3 px at
    isolated nodes (a sample point crossing a cell edge switches the one-sided bilinear gradient
    there), never by 0.05 px. The long-run bar of the GPU tests (RMS < 3e-4, 99.9th percentile
    < 2e-3, max < 0.05 px) is this envelope."""
    s = make_series(SeriesSpec(n_frames=4, side=256, drift=4.0, warp_amp=1.0,
                               mean_counts=10.0, seed=51))
    p = O.Params(levels=3, lam=10.0, beta=1.0, sigma=0.5, ladder_k=1, cap=1.0,
                 tau_min_rel=1e-4, eps=3e-4, iter_max=500)
    R, T = O.frame_to_nodes(s.frames[3]), O.frame_to_nodes(s.frames[0])
    u0, s0, _ = O.register(R, T, p)
    same, rms, p999, worst = 0, [], [], 0.0
    for amp in (1e-6, 2e-6):
        rng = np.random.default_rng(0)
        for _ in range(4):
            up, sp, _ = O.register(R, T * (1 + amp * rng.standard_normal(T.shape)), p)
            if sp.iters != s0.iters or sp.trials != s0.trials:
                continue
            same += 1
            d = np.abs(O.u_to_pixels(u0, 256) - O.u_to_pixels(up, 256))
            rms.append(float(np.sqrt((d ** 2).mean())))
            p999.append(float(np.percentile(d, 99.9)))
            worst = max(worst, float(d.max()))
    assert same >= 6
    assert max(rms) < 3e-4 and max(p999) < 2e-3 and 1e-3 < worst < 0.05
    # the envelope reaches past the former 1e-4 / 1e-3 bar
    assert max(rms) > 1e-4 and max(p999) > 1e-3


def test_constant_reference_rejected():
    n = 17
    with pytest.raises(ValueError):
        O.register(np.ones((n, n)), np.random.default_rng(0).normal(size=(n, n)), O.Params(levels=2))


# ------------------------------------------------------------------------------------------
# Composition

def test_composition_identity_constants_affine():
    n = 17
    X, Y = grid(n)
    rng = np.random.default_rng(12)
    u = rng.normal(0, 0.01, size=(2, n, n))
    z = np.zeros((2, n, n))
    assert np.array_equal(O.compose(u, z), u)
    assert np.abs(O.compose(z, u) - u).max() < 1e-15
    a = np.stack([np.full((n, n), 0.03), np.full((n, n), -0.02)])
    b = np.stack([np.full((n, n), -0.01), np.full((n, n), 0.05)])
    assert np.abs(O.compose(a, b) - (a + b)).max() < 1e-15
    # affine o affine: u1 = A1 x + c1, u2 = A2 x + c2 -> w = u1 + A2 (x + u1) + c2
    A1 = np.array([[0.01, -0.02], [0.015, 0.005]])
    A2 = np.array([[-0.01, 0.02], [0.01, 0.01]])
    c1 = np.array([0.02, 0.01])
    c2 = np.array([-0.01, 0.03])
    P = np.stack([X, Y])
    u1 = np.einsum("ij,jab->iab", A1, P) + c1[:, None, None]
    u2 = np.einsum("ij,jab->iab", A2, P) + c2[:, None, None]
    w = u1 + np.einsum("ij,jab->iab", A2, P + u1) + c2[:, None, None]
    got = O.compose(u1, u2)
    q = P + u1
    inside = (q[0] >= 0) & (q[0] <= 1) & (q[1] >= 0) & (q[1] <= 1)
    assert np.abs(got - w)[:, inside].max() < 1e-14


# ------------------------------------------------------------------------------------------
# Series registration (scan with operator B)

def test_series_identical_frames_all_zero():
    s = make_series(SeriesSpec(1, 32, 0.0, 0.0, 20.0, 13))
    fr = np.stack([O.frame_to_nodes(s.frames[0])] * 5)
    for scan in ("sequential", "brent_kung", "kogge_stone", "sklansky"):
        u, a, b, pairs = O.series(fr, O.Params(levels=2), scan=scan)
        assert np.all(u == 0.0)


@pytest.mark.parametrize("M,ops", [(8, 11), (7, 8), (1, 0), (2, 1), (5, 5), (16, 26)])
def test_series_bk_schedule_counts_and_pairs(M, ops):
    """Brent-Kung over M elements: 2M - log2(M) - 2 ops for M a power of two (table), and every
    op combines (i, j) with (j, k)."""
    s = make_series(SeriesSpec(M + 1, 16, 0.5, 0.0, 0.0, 14))
    fr = np.stack([O.frame_to_nodes(f) for f in s.frames])
    u, a, b, pairs = O.series(fr, O.Params(levels=1, iter_max=0), scan="brent_kung")
    assert len(pairs) == ops
    if M == 8:
        assert ops == GOLD["scan_figures_N8"]["brent_kung"]["ops"]
    for i, j, k in pairs:
        assert i < j < k


def _ks_expected(M):
    """Kogge-Stone section: step d = 1, 2, 4, ... combines x_{j-d} with x_j for j = d .. M-1,
    both as they were after the previous step. Tracked as frame intervals."""
    x = [(m, m + 1) for m in range(M)]
    out, d = [], 1
    while d < M:
        prev = list(x)
        for j in range(d, M):
            assert prev[j - d][1] == prev[j][0]
            out.append((prev[j - d][0], prev[j - d][1], prev[j][1]))
            x[j] = (prev[j - d][0], prev[j][1])
        d *= 2
    return out, x


def _sk_expected(M):
    """Sklansky section: step d = 1, 2, 4, ...: the upper half of every block of 2d elements
    takes the last element of the lower half as left operand."""
    x = [(m, m + 1) for m in range(M)]
    out, d = [], 1
    while d < M:
        for base in range(0, M, 2 * d):
            src = base + d - 1
            for dst in range(base + d, min(base + 2 * d, M)):
                out.append((x[src][0], x[src][1], x[dst][1]))
                x[dst] = (x[src][0], x[dst][1])
        d *= 2
    return out, x


@pytest.mark.parametrize("M", [1, 2, 5, 8, 11, 16])
@pytest.mark.parametrize("scan", ["kogge_stone", "sklansky"])
def test_series_ks_sklansky_schedule_pairs(scan, M):
    """The oracle's Kogge-Stone and Sklansky scans apply B to exactly the (i, j, k) triples the
    sections' step rules give (order within a step aside), 17 and 12 of them for 8 elements
    (figures), and end with every element covering (0, m+1)."""
    s = make_series(SeriesSpec(M + 1, 16, 0.5, 0.0, 0.0, 14))
    fr = np.stack([O.frame_to_nodes(f) for f in s.frames])
    u, a, b, pairs = O.series(fr, O.Params(levels=1, iter_max=0), scan=scan)
    exp, final = (_ks_expected if scan == "kogge_stone" else _sk_expected)(M)
    assert sorted(tuple(int(v) for v in p) for p in pairs) == sorted(exp)
    assert final == [(0, m + 1) for m in range(M)]
    if M == 8:
        assert len(pairs) == GOLD["scan_figures_N8"][scan]["ops"]


def _general_expected(M, P):
    """General strategy of the distributed chapter on P workers, tracked as frame intervals:
    worker I holds K = M // P elements, one more for the first M % P workers; local stage one
    is a serial scan in every chunk; the global stage an inclusive scan over the chunk ends
    (Brent-Kung, in place); local stage two combines the end of chunk I-1 with every other
    element of chunk I."""
    x = [(m, m + 1) for m in range(M)]
    out = []
    P = min(P, M)
    sizes = [M // P + (1 if I < M % P else 0) for I in range(P)]
    lo = [sum(sizes[:I]) for I in range(P)]
    hi = [lo[I] + sizes[I] - 1 for I in range(P)]

    def b(src, dst):
        assert x[src][1] == x[dst][0]
        out.append((x[src][0], x[src][1], x[dst][1]))
        x[dst] = (x[src][0], x[dst][1])
    for I in range(P):
        for j in range(lo[I] + 1, hi[I] + 1):
            b(j - 1, j)
    d = 1
    while d < P:                                   # up-sweep over the ends
        for j in range(2 * d - 1, P, 2 * d):
            b(hi[j - d], hi[j])
        d *= 2
    d = 1
    while d * 2 < P:
        d *= 2
    while d >= 1:                                  # down-sweep over the ends
        for j in range(3 * d - 1, P, 2 * d):
            b(hi[j - d], hi[j])
        d //= 2
    for I in range(1, P):
        for j in range(lo[I], hi[I]):
            b(hi[I - 1], j)
    return out, x


def _blelloch_expected(M):
    """Blelloch's exclusive scan (Prefix sum chapter) tracked as frame intervals, None for the
    identity element: up-sweep over the elements padded with identities to a power of two, the
    root replaced by the identity, down-sweep where the left child takes the parent and the
    parent becomes parent (.) old left child. Returns the registrations (i, j, k) in the
    chapter's order (levels in order, left to right; combinations with the identity are free)
    and the inclusive results y_m = exclusive m + 1, the last one the kept total."""
    n2 = 1
    while n2 < M:
        n2 *= 2
    a = [(m, m + 1) for m in range(M)] + [None] * (n2 - M)
    regs = []

    def comb(x, y):
        if x is None or y is None:
            return y if x is None else x
        assert x[1] == y[0]
        regs.append((x[0], x[1], y[1]))
        return (x[0], y[1])
    d = 1
    while d < n2:
        for j in range(2 * d - 1, n2, 2 * d):
            a[j] = comb(a[j - d], a[j])
        d *= 2
    total, a[n2 - 1] = a[n2 - 1], None
    d = n2 // 2
    while d >= 1:
        for j in range(2 * d - 1, n2, 2 * d):
            t = a[j - d]
            a[j - d] = a[j]
            a[j] = comb(a[j], t)
        d //= 2
    return regs, [a[m + 1] for m in range(M - 1)] + [total]


def _reduce_then_scan_expected(M, P):
    """The distributed chapter's alternative strategy on P workers, tracked as intervals:
    chunks reduced into totals, Brent-Kung over the totals in place, each chunk rescanned
    serially from the total before it."""
    P = min(P, M)
    sizes = [M // P + (1 if I < M % P else 0) for I in range(P)]
    lo = [sum(sizes[:I]) for I in range(P)]
    x = [(m, m + 1) for m in range(M)]
    T = [x[lo[I]] for I in range(P)]
    regs = []

    def comb(a, b):
        assert a[1] == b[0]
        regs.append((a[0], a[1], b[1]))
        return (a[0], b[1])
    for st in range(1, max(sizes)):
        for I in range(P):
            if st < sizes[I]:
                T[I] = comb(T[I], x[lo[I] + st])
    d = 1
    while d < P:
        for j in range(2 * d - 1, P, 2 * d):
            T[j] = comb(T[j - d], T[j])
        d *= 2
    d = 1
    while d * 2 < P:
        d *= 2
    while d >= 1:
        for j in range(3 * d - 1, P, 2 * d):
            T[j] = comb(T[j - d], T[j])
        d //= 2
    for st in range(max(sizes)):
        for I in range(P):
            if st < sizes[I] and not (st == 0 and I == 0):
                j = lo[I] + st
                x[j] = comb(T[I - 1] if st == 0 else x[j - 1], x[j])
    return regs, x


@pytest.mark.parametrize("M", [1, 2, 3, 5, 8, 11, 16])
def test_series_blelloch_pairs_and_counts(M):
    """The oracle's Blelloch scan registers exactly the chapter's non-trivial combinations, in
    its order, and ends with every element covering (0, m+1). For 8 elements the figure of the
    chapter counts 14 operator applications in 6 steps; 3 of them combine with the identity
    (the leftmost path of the down-sweep), leaving Brent-Kung's 11."""
    s = make_series(SeriesSpec(M + 1, 16, 0.5, 0.0, 0.0, 17))
    fr = np.stack([O.frame_to_nodes(f) for f in s.frames])
    u, a, b, pairs = O.series(fr, O.Params(levels=1, iter_max=0), scan="blelloch")
    exp, final = _blelloch_expected(M)
    assert [tuple(int(v) for v in p) for p in pairs] == exp
    assert final == [(0, m + 1) for m in range(M)]
    if M == 8:
        fig = GOLD["scan_figures_N8"]["blelloch"]
        assert fig["ops"] == 14 and fig["steps"] == 6
        assert len(exp) == 14 - 3 == GOLD["scan_figures_N8"]["brent_kung"]["ops"]


@pytest.mark.parametrize("M,P", [(1, 1), (5, 2), (8, 2), (8, 3), (11, 4), (16, 4)])
def test_series_reduce_then_scan_pairs(M, P):
    """The oracle's alternative strategy registers exactly the chapter's triples in its order,
    ends with every element covering (0, m+1), and does (M - P) + BK(P) + (M - 1) work."""
    s = make_series(SeriesSpec(M + 1, 16, 0.5, 0.0, 0.0, 18))
    fr = np.stack([O.frame_to_nodes(f) for f in s.frames])
    u, a, b, pairs = O.series(fr, O.Params(levels=1, iter_max=0), scan="reduce_then_scan",
                              workers=P)
    exp, final = _reduce_then_scan_expected(M, P)
    assert [tuple(int(v) for v in p) for p in pairs] == exp
    assert final == [(0, m + 1) for m in range(M)]
    bk = {1: 0, 2: 1, 3: 2, 4: 4}[min(P, M)]
    assert len(pairs) == (M - min(P, M)) + bk + (M - 1)


@pytest.mark.parametrize("M,P", [(1, 1), (5, 2), (8, 2), (8, 3), (11, 4), (16, 4), (9, 9)])
def test_series_general_strategy_pairs(M, P):
    """The oracle's general strategy applies B to exactly the (i, j, k) triples of the
    chapter's stages (order within a stage aside), ends with every element covering
    (0, m+1), and for an even division does the chapter's work: N - P in local stage one,
    the global scan's, and (P - 1)(K - 1) in local stage two (the inclusive global stage
    already finished the chunk ends)."""
    s = make_series(SeriesSpec(M + 1, 16, 0.5, 0.0, 0.0, 16))
    fr = np.stack([O.frame_to_nodes(f) for f in s.frames])
    u, a, b, pairs = O.series(fr, O.Params(levels=1, iter_max=0), scan="general", workers=P)
    exp, final = _general_expected(M, P)
    assert sorted(tuple(int(v) for v in p) for p in pairs) == sorted(exp)
    assert final == [(0, m + 1) for m in range(M)]
    if M % P == 0:
        K = M // P
        # Brent-Kung work over the P ends: 2P - 2 - log2 P for a power of two (table of the
        # Prefix sum chapter); 12 for 9 ends (7 up-sweep + 5 down-sweep, counted by hand)
        bk = {1: 0, 2: 1, 4: 4, 9: 12}[P]
        assert len(pairs) == (M - P) + bk + (P - 1) * (K - 1)
    # the default worker count is ceil(sqrt(M))
    _, _, _, pd = O.series(fr, O.Params(levels=1, iter_max=0), scan="general")
    assert len(pd) == len(_general_expected(M, int(np.ceil(np.sqrt(M))))[0])


def test_series_translation_chain_and_bk_vs_sequential():
    spec = SeriesSpec(6, 64, 1.0, 0.0, 0.0, 15)
    s = make_series(spec)
    fr = np.stack([O.frame_to_nodes(f) for f in s.frames])
    p = O.Params(levels=3, lam=10.0, eps=3e-4)
    useq, _, _, _ = O.series(fr, p, scan="sequential")
    b = 8
    for k in range(1, 6):
        gt = ground_truth(s, k)
        e = O.u_to_pixels(useq[k], 64) - gt
        assert np.sqrt((e[:, b:-b, b:-b] ** 2).mean()) < 0.1
    for scan in ("brent_kung", "kogge_stone", "sklansky", "general", "blelloch",
                 "reduce_then_scan"):
        upar, _, _, _ = O.series(fr, p, scan=scan, workers=2)
        for k in range(1, 6):
            d = O.u_to_pixels(upar[k] - useq[k], 64)
            # approximate associativity (definition in the associativity section)
            assert np.sqrt((d[:, b:-b, b:-b] ** 2).mean()) < 0.05
        assert np.all(upar[0] == 0)
    assert np.all(useq[0] == 0)


@pytest.mark.slow
def test_fp32_storage_sensitivity_at_full_size():
    """The GPU stores u in FP32. Rounding only u to FP32 after each step in this FP64 oracle
    moves the 512 x 512, 4-level result by up to ~1e-2 px at a few nodes: the gradient of the
    bilinear interpolant jumps across cell edges, and a position rounded to the other side of an
    edge takes the other cell's slope. This bounds the full-size agreement of any FP32
    implementation; the GPU parity test at full size uses the bounds measured here."""
    s = make_series(SeriesSpec(2, 512, 8.0, 1.5, 5.0, 2))
    R, T = O.frame_to_nodes(s.frames[0]), O.frame_to_nodes(s.frames[1])
    p = O.Params(levels=4, lam=10.0, eps=3e-4)
    a, sa, _ = O.register(R, T, p)
    try:
        O.set_u_storage_f32(True)
        b, sb, _ = O.register(R, T, p)
    finally:
        O.set_u_storage_f32(False)
    d = np.abs(O.u_to_pixels(a - b, 512))
    assert sa.iters == sb.iters and sa.trials == sb.trials
    assert np.sqrt((d ** 2).mean()) < 1e-4
    assert np.percentile(d, 99.9) < 1e-3
    assert 1e-3 < d.max() < 0.05


# ------------------------------------------------------------------------------------------
# Series averaging (Introduction: the aligned frames f_i o phi_{0,i} averaged)

def test_average_zero_displacement_is_plain_mean():
    rng = np.random.default_rng(31)
    f = rng.uniform(0, 10, size=(5, 12, 17))
    got = O.series_average(f, np.zeros((5, 2, 12, 17)))
    assert np.allclose(got, f.mean(axis=0), rtol=0, atol=1e-12)


def test_average_undoes_integer_shifts_inside():
    """f_i is a reference image g shifted by t_i; with u_i = t_i every aligned frame is g again,
    so the average is g wherever no sample was clamped."""
    rng = np.random.default_rng(32)
    g = rng.uniform(0, 1, size=(40, 40))
    shifts = [(0, 0), (3, -2), (-4, 1), (2, 5)]
    H = W = 40
    f = np.zeros((len(shifts), H, W))
    u = np.zeros((len(shifts), 2, H, W))
    for i, (tx, ty) in enumerate(shifts):
        for r in range(H):
            for c in range(W):
                rr, cc = min(max(r - ty, 0), H - 1), min(max(c - tx, 0), W - 1)
                f[i, r, c] = g[rr, cc]
        u[i, 0], u[i, 1] = tx, ty
    got = O.series_average(f, u)
    m = 6
    assert np.abs(got[m:-m, m:-m] - g[m:-m, m:-m]).max() < 1e-12


def test_average_half_pixel_and_clamp():
    """One frame, u = (0.5, 0): the mean of each pixel and its right neighbour (the last
    column is clamped onto itself); u = (0, 0.25): a quarter of the way to the row below;
    u = (-10, 0): the first column."""
    rng = np.random.default_rng(33)
    f = rng.uniform(0, 1, size=(1, 9, 11))
    u = np.zeros((1, 2, 9, 11))
    u[0, 0] = 0.5
    got = O.series_average(f, u)
    assert np.allclose(got[:, :-1], 0.5 * (f[0, :, :-1] + f[0, :, 1:]), atol=1e-14)
    assert np.allclose(got[:, -1], f[0, :, -1], atol=1e-14)
    u[0, 0], u[0, 1] = 0.0, 0.25
    got = O.series_average(f, u)
    assert np.allclose(got[:-1], 0.75 * f[0, :-1] + 0.25 * f[0, 1:], atol=1e-14)
    u[0, 0], u[0, 1] = -10.0, 0.0
    got = O.series_average(f, u)
    assert np.allclose(got[:, :11 - 1], f[0, :, :1], atol=1e-14)
    sel = O.series_average(f, u, pixels=(np.array([0, 8]), np.array([10, 3])))
    assert np.allclose(sel, got[[0, 8], [10, 3]], atol=1e-14)


# ------------------------------------------------------------------------------------------
# Rigid variant (definition of a rigid transformation): phi(x) = R(alpha) x + t

def test_warm_judge_reading_reduces_to_the_cold_series():
    """The warm-start judge (oracle.warm_series) on a series whose finest level (8) is above
    the judge's level 7, pinned by the two cases where it must give the plain method's series
    exactly: a guess that is not finite is rejected everywhere (every neighbour registration a
    fallback, every B application from the composition); a zero guess in REFINE mode starts every
    neighbour registration at the identity on the coarsest level, passes the NCC test on level 7
    (the registration only raises the NCC) and resumes on level 8 from that level-7 result,
    which is the cold registration's own path."""
    s = make_series(SeriesSpec(5, 256, 2.0, 0.5, 10.0, 77))
    p = O.Params(levels=3, lam=10.0, eps=3e-4)
    fr = np.stack([O.frame_to_nodes(f) for f in s.frames])
    cold, _, _, _ = O.series(fr, p, scan="brent_kung")
    g_nan = np.full((2, 129, 129), np.nan)
    u, ops = O.warm_series(fr, p, lambda i, k: g_nan, "refine")
    assert all(o["fallback"] and not o["net_start"] for o in ops[:4])
    assert not any(o["net_start"] for o in ops[4:])
    assert np.array_equal(u, cold)
    zero = np.zeros((2, 129, 129))
    u, ops = O.warm_series(fr, p, lambda i, k: zero, "refine")
    # (on this series every composition also beats the zero guess on level 7)
    assert not any(o["fallback"] or o["net_start"] for o in ops)
    assert np.array_equal(u, cold)


def test_averaging_procedure_fixed_points_and_gain():
    """The series averaging procedure (a round: average the aligned frames, register every
    frame i >= 1 to the average from its current deformation): identical frames stay at the
    identity exactly; noise-free frames started from the analytic displacements stay within
    0.05 px of them; and one round started from the series registration of a noisy series
    brings the average closer to the clean object than the single average."""
    p = O.Params(levels=2, lam=10.0, eps=3e-4)
    s = make_series(SeriesSpec(1, 64, 0.0, 0.0, 20.0, 72))
    same = np.stack([s.frames[0]] * 4)
    u, avg, _ = O.series_average_refine(same, np.zeros((4, 2, 64, 64)), 2, p)
    assert np.all(u == 0) and np.allclose(avg, s.frames[0], atol=1e-12)
    s = make_series(SeriesSpec(5, 64, 1.5, 0.5, 0.0, 73))
    gt = np.stack([np.zeros((2, 64, 64))] + [ground_truth(s, k) for k in range(1, 5)])
    u, _, _ = O.series_average_refine(s.frames, gt, 1, p)
    assert np.all(u[0] == 0)
    assert np.sqrt(((u - gt)[1:, :, 8:-8, 8:-8] ** 2).mean()) < 0.05
    for seed in (70, 71):
        s = make_series(SeriesSpec(8, 64, 1.5, 0.5, 20.0, seed))
        clean = make_series(SeriesSpec(8, 64, 1.5, 0.5, 0.0, seed))
        obj = clean.frames[0] * (s.frames.mean() / clean.frames.mean())
        fr = np.stack([O.frame_to_nodes(f) for f in s.frames])
        us, _, _, _ = O.series(fr, p, scan="brent_kung")
        u1 = np.stack([O.u_to_pixels(x, 64) for x in us])
        err = lambda a: np.sqrt(((a - obj)[8:-8, 8:-8] ** 2).mean())
        _, ar, _ = O.series_average_refine(s.frames, u1, 1, p)
        assert err(ar) < err(O.series_average(s.frames, u1))


def _rotated_pair(side, alpha, t_px, seed):
    """Frame 0 is the blob lattice L; frame 1 is L seen through the rigid map, T(y) =
    L(R(alpha)^-1 (y - t)), so that T(phi(x)) = L(x) with phi(x) = R(alpha) x + t (pixels,
    rotation about pixel (0, 0)). Noise-free."""
    from synth.blobs import _lattice
    spec = SeriesSpec(2, side, 4.0, 0.0, 0.0, seed)
    s = make_series(spec)
    r, c = np.meshgrid(np.arange(side, dtype=np.float64), np.arange(side, dtype=np.float64),
                       indexing="ij")
    ca, sa = np.cos(alpha), np.sin(alpha)
    x, y = c - t_px[0], r - t_px[1]
    f0 = _lattice(spec, s.origin, s.amps, s.lattice_lo, c, r)
    f1 = _lattice(spec, s.origin, s.amps, s.lattice_lo, ca * x + sa * y, -sa * x + ca * y)
    return f0, f1


@pytest.mark.parametrize("alpha,t", [(0.0, (2.5, -1.75)), (0.015, (1.0, 0.5)),
                                     (-0.02, (-2.0, 1.5))])
def test_rigid_recovers_known_rotation_and_shift(alpha, t):
    side = 64
    f0, f1 = _rotated_pair(side, alpha, t, 17)
    p, st = O.register_rigid(O.frame_to_nodes(f0), O.frame_to_nodes(f1),
                             O.Params(levels=3, eps=1e-9, iter_max=2000))
    got_t = p[1:] * side                      # domain units -> pixels

    def phi(a, tt, x, y):
        return (np.cos(a) * x - np.sin(a) * y + tt[0], np.sin(a) * x + np.cos(a) * y + tt[1])

    # the recovered map against the true one over the frame (its extremes are at the corners)
    err = max(np.hypot(*(np.subtract(phi(p[0], got_t, x, y), phi(alpha, t, x, y))))
              for x in (0, side) for y in (0, side))
    assert err < 0.05
    # below 1 only through the borders: clamped samples, and the replicated last node row and
    # column of the 2^L-pixel frames
    assert st.ncc > 0.97


def test_rigid_identical_frames_stay_at_identity():
    f0, _ = _rotated_pair(32, 0.0, (0.0, 0.0), 18)
    fr = O.frame_to_nodes(f0)
    p, st = O.register_rigid(fr, fr, O.Params(levels=2))
    assert np.abs(p).max() < 1e-9
    assert sum(st.iters) == 0 or np.abs(p).max() < 1e-9


def test_rigid_energy_is_the_field_energy_of_the_affine_displacement():
    """A rigid start guess evaluated through the rigid path equals the field oracle's energy of
    the same (affine) displacement at lambda = 0, and the rigid flow from there never raises
    the energy."""
    side = 32
    f0, f1 = _rotated_pair(side, 0.01, (1.0, -0.5), 19)
    R, T = O.frame_to_nodes(f0), O.frame_to_nodes(f1)
    n = side + 1
    p0 = np.array([0.004, 0.5 / side, -0.25 / side])
    yy, xx = np.meshgrid(np.arange(n) / side, np.arange(n) / side, indexing="ij")
    ca, sa = np.cos(p0[0]), np.sin(p0[0])
    u = np.stack([ca * xx - sa * yy + p0[1] - xx, sa * xx + ca * yy + p0[2] - yy])
    e_field, _ = O.energy(R, T, u, 0.0)
    p, st = O.register_rigid(R, T, O.Params(levels=1, iter_max=0), p_init=p0)
    assert np.allclose(p, p0)
    assert abs(st.energy - e_field) < 1e-12
    p2, st2 = O.register_rigid(R, T, O.Params(levels=1), p_init=p0)
    assert st2.energy <= e_field


def _rigid_series(side, N, seed, rot=0.008, shift=1.5):
    """Frames f_k = L o Phi_k^-1 for cumulative random rigid maps Phi_k (Phi_0 = identity):
    f_0 = f_k o phi_0k with phi_0k = Phi_k. Returns frames [N, side, side] and the true
    parameter rows (alpha, t0 px, t1 px) of phi_0k."""
    from synth.blobs import _lattice
    spec = SeriesSpec(2, side, 8.0, 0.0, 0.0, seed)
    s = make_series(spec)
    rng = np.random.default_rng(seed)
    r, c = np.meshgrid(np.arange(side, dtype=np.float64), np.arange(side, dtype=np.float64),
                       indexing="ij")
    frames, truth = [], []
    a, t = 0.0, np.zeros(2)
    for k in range(N):
        if k:
            a += rng.uniform(-rot, rot)
            t = t + rng.uniform(-shift, shift, size=2)
        ca, sa = np.cos(a), np.sin(a)
        x, y = c - t[0], r - t[1]
        frames.append(_lattice(spec, s.origin, s.amps, s.lattice_lo, ca * x + sa * y,
                               -sa * x + ca * y))
        truth.append([a, t[0], t[1]])
    return np.stack(frames), np.array(truth)


def test_rigid_composition_is_the_product_of_the_maps():
    """phi_jk o phi_ij in parameters against the product of homogeneous 3x3 matrices."""
    rng = np.random.default_rng(34)

    def mat(p):
        c, s = np.cos(p[0]), np.sin(p[0])
        return np.array([[c, -s, p[1]], [s, c, p[2]], [0.0, 0.0, 1.0]])

    for _ in range(20):
        u, v = rng.uniform(-1, 1, 3), rng.uniform(-1, 1, 3)
        w = O._compose_rigid(u, v)
        assert np.allclose(mat(w), mat(v) @ mat(u), atol=1e-14)
    assert np.allclose(O._compose_rigid(u, np.zeros(3)), u)


def test_rigid_series_recovers_cumulative_maps():
    side, N = 64, 6
    frames, truth = _rigid_series(side, N, 35)
    fr = np.stack([O.frame_to_nodes(f) for f in frames])
    for scan in ("sequential", "brent_kung"):
        p = O.series_rigid(fr, O.Params(levels=2, eps=1e-9, iter_max=400), scan=scan)
        assert np.all(p[0] == 0)
        for k in range(1, N):
            got = np.array([p[k, 0], p[k, 1] * side, p[k, 2] * side])
            # largest corner distance between the recovered and the true map (px)
            d = 0.0
            for x in (0, side):
                for y in (0, side):
                    ga = np.array([np.cos(got[0]) * x - np.sin(got[0]) * y + got[1],
                                   np.sin(got[0]) * x + np.cos(got[0]) * y + got[2]])
                    tr = truth[k]
                    ta = np.array([np.cos(tr[0]) * x - np.sin(tr[0]) * y + tr[1],
                                   np.sin(tr[0]) * x + np.cos(tr[0]) * y + tr[2]])
                    d = max(d, float(np.hypot(*(ga - ta))))
            assert d < 0.05, (scan, k, d)
