"""FP64 CPU oracle of the registration operator and of the series prefix scan.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline leg of the
benchmark may use it; the product path never does. It shares no code with the GPU path.

The C source (pprs_oracle.c) is compiled with gcc on first use (or by build()). Arrays cross
the boundary as C-contiguous float64 NumPy arrays. Frames are nodal grids (2^L+1)^2 and
displacements are [2, n, n] in domain units ([0,1]^2), unless a function says otherwise.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from dataclasses import dataclass, asdict

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pprs_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

TRACE_W = 8
SCAN_KINDS = {"sequential": 0, "brent_kung": 1, "kogge_stone": 2, "sklansky": 3, "general": 4,
              "blelloch": 5, "reduce_then_scan": 6}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, FP64, no fast-math)."""
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math",
           "-o", tmp, _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if (not os.path.exists(_LIB)) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        D = ctypes.POINTER(ctypes.c_double)
        I = ctypes.POINTER(ctypes.c_int)
        U8 = ctypes.POINTER(ctypes.c_ubyte)
        P = ctypes.POINTER(_CParams)
        S = ctypes.POINTER(_CStats)
        sigs = {
            "or_restrict": (None, [D, ctypes.c_int, D]),
            "or_prolong": (None, [D, ctypes.c_int, D]),
            "or_bilinear": (ctypes.c_double, [D, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                              D, D]),
            "or_mass_apply": (None, [D, ctypes.c_int, D]),
            "or_stiff_apply": (None, [D, ctypes.c_int, D]),
            "or_normalize": (ctypes.c_int, [D, ctypes.c_int, D, D, D]),
            "or_smooth": (None, [D, ctypes.c_int, ctypes.c_double, D]),
            "or_energy": (ctypes.c_double, [D, D, ctypes.c_int, D, ctypes.c_double, D]),
            "or_gradient": (ctypes.c_int, [D, D, ctypes.c_int, D, ctypes.c_double, D]),
            "or_gradient_flow": (ctypes.c_int, [D, D, ctypes.c_int, D, P, I, I, D, D,
                                                ctypes.c_int, I]),
            "or_register": (ctypes.c_int, [D, D, ctypes.c_int, D, P, D, S, D, ctypes.c_int, I]),
            "or_register_f": (ctypes.c_int, [D, D, ctypes.c_int, D, P, I, U8, ctypes.c_int, D,
                                             S, D, ctypes.c_int, I]),
            "or_register_from": (ctypes.c_int, [D, D, ctypes.c_int, ctypes.c_int, D, P, D, S, D,
                                                ctypes.c_int, I]),
            "or_compose": (None, [D, D, ctypes.c_int, D]),
            "or_register_rigid": (ctypes.c_int, [D, D, ctypes.c_int, D, P, D, S]),
            "or_register_rigid_f": (ctypes.c_int, [D, D, ctypes.c_int, D, P, I, U8,
                                                   ctypes.c_int, D, S]),
            "or_series": (ctypes.c_int, [D, ctypes.c_int, ctypes.c_int, P, ctypes.c_int,
                                         ctypes.c_int, D, S, S, I, ctypes.c_int]),
            "or_series_f": (ctypes.c_int, [D, ctypes.c_int, ctypes.c_int, P, ctypes.c_int,
                                           ctypes.c_int, I, I, U8, U8, ctypes.c_int, D, S, S,
                                           I, ctypes.c_int]),
            "or_set_u_storage_f32": (None, [ctypes.c_int]),
        }
        for name, (res, args) in sigs.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
        return lib


class _CParams(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int), ("lam", ctypes.c_double), ("beta", ctypes.c_double),
                ("sigma", ctypes.c_double), ("ladder_k", ctypes.c_int), ("cap", ctypes.c_double),
                ("tau_min_rel", ctypes.c_double), ("eps", ctypes.c_double),
                ("iter_max", ctypes.c_int)]


class _CStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int * 16), ("trials", ctypes.c_int * 16),
                ("energy", ctypes.c_double), ("ncc", ctypes.c_double), ("flags", ctypes.c_int),
                ("tie_gap", ctypes.c_double), ("armijo_gap", ctypes.c_double)]


@dataclass
class Params:
    """Parameters of operator A. Field meanings follow the C struct in pprs_oracle.c."""
    levels: int = 2
    lam: float = 0.1
    beta: float = 1.0
    sigma: float = 0.5
    ladder_k: int = 1
    cap: float = 1.0
    tau_min_rel: float = 1e-4
    eps: float = 1e-7
    iter_max: int = 500

    def c(self) -> _CParams:
        return _CParams(**asdict(self))


def _d(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# ------------------------------------------------------------------------------------------ #
# Elementary operators

def restrict(f) -> np.ndarray:
    f = _f64(f)
    n = f.shape[-1]
    nc = (n - 1) // 2 + 1
    out = np.empty((nc, nc))
    _load().or_restrict(_d(f), n, _d(out))
    return out


def prolong(c) -> np.ndarray:
    c = _f64(c)
    nc = c.shape[-1]
    nf = 2 * (nc - 1) + 1
    out = np.empty((nf, nf))
    _load().or_prolong(_d(c), nc, _d(out))
    return out


def bilinear(g, px: float, py: float):
    g = _f64(g)
    gx = ctypes.c_double()
    gy = ctypes.c_double()
    v = _load().or_bilinear(_d(g), g.shape[-1], px, py, ctypes.byref(gx), ctypes.byref(gy))
    return v, gx.value, gy.value


def mass_apply(f) -> np.ndarray:
    f = _f64(f)
    out = np.empty_like(f)
    _load().or_mass_apply(_d(f), f.shape[-1], _d(out))
    return out


def stiff_apply(f) -> np.ndarray:
    f = _f64(f)
    out = np.empty_like(f)
    _load().or_stiff_apply(_d(f), f.shape[-1], _d(out))
    return out


def normalize(f):
    """Returns (F~, mean, sigma); F~ is None when sigma == 0."""
    f = _f64(f)
    out = np.empty_like(f)
    m = ctypes.c_double()
    s = ctypes.c_double()
    rc = _load().or_normalize(_d(f), f.shape[-1], _d(out), ctypes.byref(m), ctypes.byref(s))
    return (out if rc == 0 else None), m.value, s.value


def smooth(g, beta: float) -> np.ndarray:
    g = _f64(g)
    out = np.empty_like(g)
    _load().or_smooth(_d(g), g.shape[-1], beta, _d(out))
    return out


def energy(R, T, u, lam: float):
    """Returns (E, NCC) for raw reference R, template T and displacement u [2, n, n]."""
    R, T, u = _f64(R), _f64(T), _f64(u)
    ncc = ctypes.c_double()
    e = _load().or_energy(_d(R), _d(T), R.shape[-1], _d(u), lam, ctypes.byref(ncc))
    return e, ncc.value


def gradient(R, T, u, lam: float) -> np.ndarray:
    R, T, u = _f64(R), _f64(T), _f64(u)
    G = np.empty_like(u)
    rc = _load().or_gradient(_d(R), _d(T), R.shape[-1], _d(u), lam, _d(G))
    if rc != 0:
        raise ValueError("constant reference")
    return G


def gradient_flow(R, T, u0, params: Params, trace_cap: int = 4096):
    """One level of gradient flow. Returns (u, steps, passes, energy, trace[len, 8], flags)."""
    R, T = _f64(R), _f64(T)
    u = _f64(u0).copy()
    steps = ctypes.c_int()
    passes = ctypes.c_int()
    e = ctypes.c_double()
    tr = np.zeros((trace_cap, TRACE_W))
    tl = ctypes.c_int()
    cp = params.c()
    flags = _load().or_gradient_flow(_d(R), _d(T), R.shape[-1], _d(u), ctypes.byref(cp),
                                     ctypes.byref(steps), ctypes.byref(passes), ctypes.byref(e),
                                     _d(tr), trace_cap, ctypes.byref(tl))
    if flags < 0:
        raise ValueError("constant reference")
    return u, steps.value, passes.value, e.value, tr[: tl.value], flags


@dataclass
class RegStats:
    iters: list
    trials: list
    energy: float
    ncc: float
    flags: int
    tie_gap: float = 0.0     # replayed decisions only: largest distance of the energy test
                             # from deciding a replayed stop the other way
    armijo_gap: float = 0.0  # ... and of the Armijo test from a replayed line-search choice


def _force(force, rows: int = 1):
    """Replayed stopping decisions: `rows` lists of accepted-step counts per level (coarsest
    first; None or -1 where the energy-decrease test decides) -> int32 [rows][16], or None."""
    if force is None:
        return None
    if rows == 1:
        force = [force]
    if len(force) != rows:
        raise ValueError("need %d lists of replayed step counts" % rows)
    out = np.full((rows, 16), -1, dtype=np.int32)
    for r, lst in enumerate(force):
        if lst is None:
            continue
        if len(lst) > 16:
            raise ValueError("at most 16 levels")
        out[r, :len(lst)] = [-1 if v is None else int(v) for v in lst]
    return out


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int)) if a is not None else None


def _rungs(rungs, rows: int = 1):
    """Replayed ladder positions: `rows` uint8 sequences (one per registration, each step in
    order) -> (uint8 [rows][cap], cap), or (None, 0)."""
    if rungs is None:
        return None, 0
    if rows == 1:
        rungs = [rungs]
    if len(rungs) != rows:
        raise ValueError("need %d rung sequences" % rows)
    cap = max(1, max(len(r) for r in rungs))
    out = np.zeros((rows, cap), dtype=np.uint8)
    for r, seq in enumerate(rungs):
        out[r, :len(seq)] = np.asarray(seq, dtype=np.uint8)
    return out, cap


def _up(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte)) if a is not None else None


def _stats(st: _CStats, levels: int) -> RegStats:
    return RegStats(list(st.iters[:levels]), list(st.trials[:levels]), st.energy, st.ncc,
                    st.flags, st.tie_gap, st.armijo_gap)


def register(R, T, params: Params, u0=None, trace_cap: int = 0, force=None, rungs=None):
    """Operator A on finest-level nodal frames. Returns (u [2,n,n] domain units, RegStats,
    trace).

    force (test switch): accepted-step counts per level, coarsest first; a level with a count
    takes exactly that many steps (unless its line search fails first) instead of stopping by
    the energy-decrease test. rungs (test switch): the ladder position J of every accepted step
    (levels in order), taken in place of the Armijo test's choice. They replay decisions another
    implementation took; the stats' tie_gap / armijo_gap say how far the oracle's own tests
    were from each replayed decision. Pass both, or neither: a replayed rung sequence belongs to
    one sequence of step counts."""
    R, T = _f64(R), _f64(T)
    n = R.shape[-1]
    u = np.empty((2, n, n))
    st = _CStats()
    cp = params.c()
    tr = np.zeros((max(trace_cap, 1), TRACE_W))
    tl = ctypes.c_int()
    u0p = _d(_f64(u0)) if u0 is not None else None
    keep = _f64(u0) if u0 is not None else None
    if keep is not None:
        u0p = _d(keep)
    fo = _force(force)
    ru, rc_ = _rungs(rungs)
    rc = _load().or_register_f(_d(R), _d(T), n, u0p, ctypes.byref(cp), _ip(fo), _up(ru), rc_,
                               _d(u), ctypes.byref(st), _d(tr), trace_cap, ctypes.byref(tl))
    if rc == -1:
        raise ValueError("constant reference on some level")
    if rc != 0:
        raise ValueError("invalid sizes or levels")
    return u, _stats(st, params.levels), tr[: tl.value]


def trace_rungs(trace, params: Params):
    """Ladder position J of every accepted step of a register() trace (levels in order): the
    step is top 2^-J with top = min(2^K tau_prev, tau_max) of its iteration."""
    out = []
    prev_level, tau_prev = None, np.inf
    for level, step, tau, e0, e1, gtd, tmax, passes in trace:
        if level != prev_level:
            prev_level, tau_prev = level, np.inf
        if tau <= 0:
            continue
        top = min(2.0 ** params.ladder_k * tau_prev, tmax)
        out.append(int(round(np.log2(top / tau))))
        tau_prev = tau
    return out


def register_from(R, T, start: int, u_start, params: Params, trace_cap: int = 0):
    """Operator A started on level `start` from u_start ([2, n, n] on that level, domain units);
    the coarser levels are skipped. Returns (u [2, nf, nf], RegStats, trace)."""
    R, T = _f64(R), _f64(T)
    n = R.shape[-1]
    us = _f64(u_start)
    u = np.empty((2, n, n))
    st = _CStats()
    cp = params.c()
    tr = np.zeros((max(trace_cap, 1), TRACE_W))
    tl = ctypes.c_int()
    if us.shape != (2, (1 << start) + 1, (1 << start) + 1):
        raise ValueError("u_start must be [2, 2^start+1, 2^start+1]")
    rc = _load().or_register_from(_d(R), _d(T), n, start, _d(us), ctypes.byref(cp), _d(u),
                                  ctypes.byref(st), _d(tr), trace_cap, ctypes.byref(tl))
    if rc == -1:
        raise ValueError("constant reference on some level")
    if rc != 0:
        raise ValueError("invalid sizes, levels or start level")
    return u, _stats(st, params.levels), tr[: tl.value]


def register_rigid(R, T, params: Params, p_init=None, force=None, rungs=None):
    """Rigid variant of A on finest-level nodal frames: phi(x) = R(alpha) x + t about the domain
    origin. Returns (p = [alpha, t0, t1] in radians and domain units, RegStats). force: as for
    register()."""
    R, T = _f64(R), _f64(T)
    n = R.shape[-1]
    out = np.zeros(3)
    st = _CStats()
    cp = params.c()
    pin = _f64(np.asarray(p_init, dtype=np.float64)) if p_init is not None else None
    fo = _force(force)
    ru, rc_ = _rungs(rungs)
    rc = _load().or_register_rigid_f(_d(R), _d(T), n, _d(pin) if pin is not None else None,
                                     ctypes.byref(cp), _ip(fo), _up(ru), rc_, _d(out),
                                     ctypes.byref(st))
    if rc == -1:
        raise ValueError("constant reference on some level")
    if rc != 0:
        raise ValueError("invalid sizes or levels")
    return out, _stats(st, params.levels)


def _compose_rigid(u, v):
    """phi_jk o phi_ij for parameter rows u = phi_ij, v = phi_jk (alpha, t0, t1): the rotation
    angles add, t = R(alpha_jk) t_ij + t_jk."""
    c, s = np.cos(v[0]), np.sin(v[0])
    return np.array([u[0] + v[0], c * u[1] - s * u[2] + v[1], s * u[1] + c * u[2] + v[2]])


def series_rigid(frames_nodal, params: Params, scan: str = "brent_kung", force_a=None,
                 force_b=None, rungs_a=None, rungs_b=None):
    """Series registration with the rigid operator (definition of image series registration):
    N-1 neighbour registrations, then the scan with B = rigid registration started from the
    composition of the operands' maps. Schedules: "sequential" and "brent_kung" (Prefix sum
    chapter; the standard 0-based Brent-Kung form for any element count). Returns p [N, 3]
    (phi_0i; alpha in radians, t in domain units; p[0] = 0). force_a / force_b: replayed
    step counts (see register()) per neighbour registration / per B application in schedule
    order."""
    fr = _f64(frames_nodal)
    N = fr.shape[0]
    M = N - 1
    out = np.zeros((N, 3))
    if M < 1:
        return out
    el = [[m, m + 1, register_rigid(fr[m], fr[m + 1], params,
                                    force=force_a[m] if force_a is not None else None,
                                    rungs=rungs_a[m] if rungs_a is not None else None)[0]]
          for m in range(M)]
    nb = [0]

    def apply(a, b):
        ia, ka, pa = el[a]
        ib, kb, pb = el[b]
        assert ka == ib
        fb = force_b[nb[0]] if force_b is not None else None
        rb = rungs_b[nb[0]] if rungs_b is not None else None
        nb[0] += 1
        el[b] = [ia, kb, register_rigid(fr[ia], fr[kb], params,
                                        p_init=_compose_rigid(pa, pb), force=fb, rungs=rb)[0]]

    if scan == "sequential":
        for m in range(1, M):
            apply(m - 1, m)
    elif scan == "brent_kung":
        d = 1
        while d < M:
            for j in range(2 * d - 1, M, 2 * d):
                apply(j - d, j)
            d *= 2
        top = 1
        while top * 2 < M:
            top *= 2
        d = top
        while d >= 1:
            for j in range(3 * d - 1, M, 2 * d):
                apply(j - d, j)
            d //= 2
    else:
        raise ValueError("rigid series: sequential or brent_kung")
    for m in range(M):
        assert el[m][0] == 0 and el[m][1] == m + 1
        out[m + 1] = el[m][2]
    return out


def restrict_levels(f, times: int) -> np.ndarray:
    """f ([n, n] or [2, n, n]) restricted `times` levels down (full weighting each time)."""
    g = _f64(f)
    for _ in range(times):
        g = np.stack([restrict(x) for x in g]) if g.ndim == 3 else restrict(g)
    return g


def _bk_pairs(M):
    """(left, right) of the Brent-Kung schedule over M elements, in execution order."""
    out = []
    d = 1
    while d < M:
        out += [(j - d, j) for j in range(2 * d - 1, M, 2 * d)]
        d *= 2
    top = 1
    while top * 2 < M:
        top *= 2
    d = top
    while d >= 1:
        out += [(j - d, j) for j in range(3 * d - 1, M, 2 * d)]
        d //= 2
    return out


WARM_LEVEL = 7


def warm_series(frames_nodal, params: Params, guess, mode: str = "refine",
                max_cells: float = 8.0):
    """Series registration (Brent-Kung) with the learned warm start and its judge, for a
    series whose finest level L is above 7. guess(i, k) gives the network's level-7 guess
    ([2, 129, 129], domain units) for reference i and template k. Rejected outright: a guess
    that is not finite or exceeds max_cells level-7 cells (the registration runs cold).
    Neighbour registration: the warm registration up to level 7 (mode "skip": started on level
    7 from the guess; "refine": from the guess restricted to the coarsest level) against the
    identity on level 7; an NCC no lower than the identity's resumes on level 8 from the
    prolongated level-7 result, else the registration runs cold. B application: the
    composition of its operands and the guess for its own pair, both restricted to / given on
    level 7 and compared by their energy there; the lower starts the registration (on level 7
    in "skip" mode, restricted to the coarsest level in "refine" mode).
    Returns (u [N, 2, n, n], per-op dicts (pair, fallback, net_start) in execution order)."""
    fr = _f64(frames_nodal)
    N, nf = fr.shape[0], fr.shape[-1]
    L = int(round(np.log2(nf - 1)))
    m0 = L - params.levels + 1
    if not (m0 <= WARM_LEVEL < L):
        raise ValueError("the judge needs m0 <= 7 < L")
    p7 = Params(**{**params.__dict__, "levels": WARM_LEVEL - m0 + 1})
    R7 = [restrict_levels(f, L - WARM_LEVEL) for f in fr]
    n7 = (1 << WARM_LEVEL) + 1
    skip = mode == "skip"

    def ok(g):
        return np.all(np.isfinite(g)) and np.abs(g).max() * (n7 - 1) <= max_cells

    def start_from(i, k, g7):
        """A from a level-7 guess: on level 7 (skip) or restricted to m0 (refine)."""
        if skip:
            return register_from(fr[i], fr[k], WARM_LEVEL, g7, params)[0]
        return register_from(fr[i], fr[k], m0, restrict_levels(g7, WARM_LEVEL - m0), params)[0]

    ops = []
    u = np.zeros((N, 2, nf, nf))
    el = []
    for m in range(N - 1):
        g = guess(m, m + 1)
        rec = dict(pair=(m, m + 1), fallback=False, net_start=False)
        if ok(g):
            if skip:
                w, sw, _ = register_from(R7[m], R7[m + 1], WARM_LEVEL, g, p7)
            else:
                w, sw, _ = register_from(R7[m], R7[m + 1], m0,
                                         restrict_levels(g, WARM_LEVEL - m0), p7)
            ncc_id = energy(R7[m], R7[m + 1], np.zeros((2, n7, n7)), params.lam)[1]
            if sw.ncc >= ncc_id:
                u8 = np.stack([prolong(w[c]) for c in range(2)])
                res = register_from(fr[m], fr[m + 1], WARM_LEVEL + 1, u8, params)[0]
            else:
                rec["fallback"] = True
                res = register(fr[m], fr[m + 1], params)[0]
        else:
            rec["fallback"] = True
            res = register(fr[m], fr[m + 1], params)[0]
        ops.append(rec)
        el.append([m, m + 1, res])
    for a, b in _bk_pairs(N - 1):
        i, j, ua = el[a]
        j2, k, ub = el[b]
        assert j == j2
        comp = compose(ua, ub)
        g = guess(i, k)
        rec = dict(pair=(i, k), fallback=False, net_start=False)
        use_net = False
        if ok(g):
            c7 = restrict_levels(comp, L - WARM_LEVEL)
            e_c = energy(R7[i], R7[k], c7, params.lam)[0]
            e_n = energy(R7[i], R7[k], g, params.lam)[0]
            use_net = e_n < e_c
        if use_net:
            rec["net_start"] = True
            res = start_from(i, k, g)
        elif skip:
            res = register_from(fr[i], fr[k], WARM_LEVEL,
                                restrict_levels(comp, L - WARM_LEVEL), params)[0]
        else:
            res = register(fr[i], fr[k], params, u0=comp)[0]
        ops.append(rec)
        el[b] = [i, k, res]
    for m in range(N - 1):
        assert el[m][0] == 0 and el[m][1] == m + 1
        u[m + 1] = el[m][2]
    return u, ops


def set_u_storage_f32(on: bool) -> None:
    """Test switch: round the displacement to FP32 after every accepted step (process-wide)."""
    _load().or_set_u_storage_f32(1 if on else 0)


def compose(uij, ujk) -> np.ndarray:
    uij, ujk = _f64(uij), _f64(ujk)
    out = np.empty_like(uij)
    _load().or_compose(_d(uij), _d(ujk), uij.shape[-1], _d(out))
    return out


def series(frames_nodal, params: Params, scan: str = "brent_kung", threads: int = 0,
           workers: int = 0, force_a=None, force_b=None, rungs_a=None, rungs_b=None):
    """Series registration as an inclusive scan with operator B (workers: P of the general
    strategy, 0 for ceil(sqrt(N-1))). force_a (N-1 lists) and force_b (one list per B
    application in schedule order): replayed step counts; rungs_a / rungs_b: replayed ladder
    positions, one sequence per registration; see register().

    frames_nodal: [N, n, n]. Returns (u [N, 2, n, n] domain units with u[0] = 0, a_stats,
    b_stats, b_pairs [(i, j, k)] in execution order)."""
    fr = _f64(frames_nodal)
    N, n = fr.shape[0], fr.shape[-1]
    u = np.zeros((N, 2, n, n))
    a_st = (_CStats * max(N - 1, 1))()
    # B ops: at most 2(M-1) for sequential and Brent-Kung, M log2 M for Kogge-Stone and Sklansky
    M = max(N - 1, 1)
    cap = 2 * M + M * max(1, int(np.ceil(np.log2(M))))
    b_st = (_CStats * cap)()
    pairs = np.zeros(3 * cap, dtype=np.int32)
    cp = params.c()
    fa = _force(force_a, N - 1) if force_a is not None else None
    fb = None
    if force_b is not None:
        fb = np.full((cap, 16), -1, dtype=np.int32)
        if len(force_b) > cap:
            raise ValueError("too many B lists")
        fb[:len(force_b)] = _force(force_b, len(force_b))
    ra = rb = None
    rcap = 0
    if rungs_a is not None or rungs_b is not None:
        seqs = list(rungs_a or [[]] * (N - 1)) + list(rungs_b or [])
        rcap = max(1, max(len(x) for x in seqs))
        ra = np.zeros((max(N - 1, 1), rcap), dtype=np.uint8)
        rb = np.zeros((cap, rcap), dtype=np.uint8)
        for m, x in enumerate(rungs_a or []):
            ra[m, :len(x)] = np.asarray(x, dtype=np.uint8)
        for m, x in enumerate(rungs_b or []):
            rb[m, :len(x)] = np.asarray(x, dtype=np.uint8)
        if rungs_a is None:
            ra = None
        if rungs_b is None:
            rb = None
    rc = _load().or_series_f(_d(fr), N, n, ctypes.byref(cp), SCAN_KINDS[scan], workers,
                             _ip(fa), _ip(fb), _up(ra), _up(rb), rcap, _d(u), a_st, b_st,
                             pairs.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), threads)
    if rc < 0:
        raise ValueError("oracle series failed with %d" % rc)
    a = [_stats(a_st[m], params.levels) for m in range(N - 1)]
    b = [_stats(b_st[m], params.levels) for m in range(rc)]
    return u, a, b, [tuple(pairs[3 * m: 3 * m + 3]) for m in range(rc)]


def series_average(frames, u, pixels=None):
    """Series averaging (Introduction; image series registration): the aligned frames
    f_i o phi_{0,i} averaged, avg(x) = 1/N sum_i f_i(x + u_i(x)), on the pixel grid (x is the
    column, y the row), each f_i interpolated bilinearly with the position clamped to
    [0, W-1] x [0, H-1]. frames [N, H, W], u [N, 2, H, W] in pixels. pixels: optional
    (rows, cols) integer arrays; then only those pixels are evaluated (1-D result). FP64."""
    f = np.asarray(frames, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    N, H, W = f.shape
    if pixels is None:
        r, c = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    else:
        r, c = (np.asarray(a) for a in pixels)
    acc = np.zeros(r.shape)
    for i in range(N):
        x = np.clip(c + u[i, 0][r, c], 0.0, W - 1.0)
        y = np.clip(r + u[i, 1][r, c], 0.0, H - 1.0)
        x0 = np.minimum(np.floor(x).astype(np.int64), W - 2)
        y0 = np.minimum(np.floor(y).astype(np.int64), H - 2)
        fx, fy = x - x0, y - y0
        top = (1.0 - fx) * f[i][y0, x0] + fx * f[i][y0, x0 + 1]
        bot = (1.0 - fx) * f[i][y0 + 1, x0] + fx * f[i][y0 + 1, x0 + 1]
        acc += (1.0 - fy) * top + fy * bot
    return acc / N


def series_average_refine(frames, u, passes: int, params: Params, force=None, rungs=None):
    """The series averaging procedure (Introduction; section "Registration for series of
    images": the series' result refined by further rounds of registration): each round averages
    the aligned frames (series_average) and registers every frame f_i, i >= 1, to that average
    with operator A started from its current deformation (restricted to the coarsest level, as
    the multilevel algorithm prescribes); f_0's deformation stays the identity, which keeps the
    result in f_0's coordinates. frames [N, H, W] and u [N, 2, H, W] in pixels (H = W = 2^L).
    force / rungs (test switches, as in register()): per registration, pass-major with frame 1
    first, the decisions to replay (None entries leave a registration to its own tests).
    Returns (u refined, the average of the last round's alignment, [RegStats] pass-major)."""
    f = np.asarray(frames, dtype=np.float64)
    u = np.array(u, dtype=np.float64)
    N, H, W = f.shape
    stats = []
    for q in range(passes):
        avg = series_average(f, u)
        R = frame_to_nodes(avg)
        for i in range(1, N):
            row = q * (N - 1) + i - 1
            fo = force[row] if force is not None else None
            ru = rungs[row] if rungs is not None and fo is not None else None
            u0 = np.stack([frame_to_nodes(u[i, c]) for c in range(2)]) / H
            res, st, _ = register(R, frame_to_nodes(f[i]), params, u0=u0, force=fo, rungs=ru)
            u[i] = u_to_pixels(res, H)
            stats.append(st)
    return u, series_average(f, u), stats


# ------------------------------------------------------------------------------------------ #
# Pixel frames <-> nodal grids (the API works in pixels of 2^L x 2^L frames)

def frame_to_nodes(frame) -> np.ndarray:
    """2^L x 2^L pixels -> (2^L+1)^2 nodes by replicating the last row and column."""
    f = _f64(frame)
    return np.pad(f, ((0, 1), (0, 1)), mode="edge") if (f.shape[-1] & (f.shape[-1] - 1)) == 0 \
        else f


def u_to_pixels(u_dom, side: int) -> np.ndarray:
    """Domain-unit displacement on (side+1)^2 nodes -> pixels on side x side."""
    return np.asarray(u_dom)[..., :side, :side] * side
