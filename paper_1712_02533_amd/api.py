"""ctypes binding of libpprs (include/pprs.h). Argument marshalling only.

Every function takes and returns torch tensors in device memory; the work happens in the HIP
kernels of libpprs.so on the caller's current HIP stream. Displacements are [2, H, W] float32
in pixels (plane 0: x/column, plane 1: y/row); frames are [H, W] float32 with H == W == 2^L
(or 2^L + 1).
"""
from __future__ import annotations

import ctypes
import os
import threading
from dataclasses import asdict, dataclass, field

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpprs.so")

PPRS_OK = 0
PPRS_NOT_CONVERGED = 1
SCAN_KINDS = {"sequential": 0, "brent_kung": 1, "kogge_stone": 2, "sklansky": 3, "general": 4,
              "blelloch": 5, "reduce_then_scan": 6}
MAX_LEVELS = 16


class PprsError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("pprs status %d: %s" % (status, message))
        self.status = status


class _CParams(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int), ("lam", ctypes.c_double), ("beta", ctypes.c_double),
                ("armijo_sigma", ctypes.c_double), ("ladder_k", ctypes.c_int),
                ("step_cap", ctypes.c_double), ("tau_min_rel", ctypes.c_double),
                ("eps", ctypes.c_double), ("iter_max", ctypes.c_int), ("scan", ctypes.c_int),
                ("scan_workers", ctypes.c_int), ("warm_start", ctypes.c_int),
                ("force_fallback", ctypes.c_int)]


class _CPairStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int * MAX_LEVELS), ("passes", ctypes.c_int * MAX_LEVELS),
                ("energy", ctypes.c_double), ("ncc", ctypes.c_double), ("flags", ctypes.c_int),
                ("ms", ctypes.c_float)]


class _CSeriesStats(ctypes.Structure):
    _fields_ = [("n_ops_a", ctypes.c_int), ("n_ops_b", ctypes.c_int),
                ("n_scan_levels", ctypes.c_int), ("flags_or", ctypes.c_int),
                ("ms_total", ctypes.c_double), ("ms_prepare", ctypes.c_double),
                ("ms_preprocess", ctypes.c_double), ("ms_scan", ctypes.c_double),
                ("node_steps", ctypes.c_longlong), ("node_passes", ctypes.c_longlong)]


class _CTuning(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int) for n in ("pool_slots", "pool_group", "grid_energy",
                                            "grid_grad", "grid_smooth", "grid_prolong",
                                            "tile_grad", "smooth_lines", "ladder_rungs")]


TUNING_KEYS = [n for n, _ in _CTuning._fields_]


@dataclass
class Params:
    """Mirror of pprs_params; defaults are pprs_default_params()."""
    levels: int = 4
    lam: float = 10.0
    beta: float = 1.0
    armijo_sigma: float = 0.5
    ladder_k: int = 1
    step_cap: float = 1.0
    tau_min_rel: float = 1e-4
    eps: float = 3e-4
    iter_max: int = 500
    scan: str = "brent_kung"
    scan_workers: int = 0     # P of the general strategy (0: ceil(sqrt(M)))
    warm_start: int = 1       # 1: the context's network where set (cold fallback); 0: cold
    force_fallback: int = 0   # test switch: reject every network prediction

    def c(self) -> _CParams:
        d = asdict(self)
        d["scan"] = SCAN_KINDS[d["scan"]]
        return _CParams(**d)


@dataclass
class PairStats:
    iters: list
    passes: list
    energy: float
    ncc: float
    flags: int
    ms: float = 0.0


@dataclass
class SeriesStats:
    n_ops_a: int
    n_ops_b: int
    n_scan_levels: int
    flags_or: int
    ms_total: float
    ms_prepare: float
    ms_preprocess: float
    ms_scan: float
    node_steps: int
    node_passes: int


_lib_lock = threading.Lock()
_lib_obj = None


def _lib():
    global _lib_obj
    with _lib_lock:
        if _lib_obj is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError("libpprs.so is not built (%s); run __graft_entry__.build()"
                                   % LIB_PATH)
            lib = ctypes.CDLL(LIB_PATH)
            vp = ctypes.c_void_p
            i = ctypes.c_int
            sigs = {
                "pprs_default_params": (None, [ctypes.POINTER(_CParams)]),
                "pprs_create": (i, [ctypes.POINTER(vp), i, vp]),
                "pprs_destroy": (None, [vp]),
                "pprs_last_error": (ctypes.c_char_p, []),
                "pprs_register_pair": (i, [vp, vp, vp, i, i, vp, vp, ctypes.POINTER(_CParams),
                                           ctypes.POINTER(_CPairStats)]),
                "pprs_register_pair_noalloc": (i, [vp, vp, vp, i, i, vp, vp,
                                                   ctypes.POINTER(_CParams),
                                                   ctypes.POINTER(_CPairStats)]),
                "pprs_register_pairs": (i, [vp, vp, i, i, i, vp, vp, i, vp,
                                            ctypes.POINTER(_CParams),
                                            ctypes.POINTER(_CPairStats)]),
                "pprs_compose_deformations": (i, [vp, vp, vp, vp, i, i]),
                "pprs_series_average": (i, [vp, vp, vp, i, i, i, vp]),
                "pprs_series_average_refine": (i, [vp, vp, i, i, i, vp, i,
                                                   ctypes.POINTER(_CParams), vp,
                                                   ctypes.POINTER(_CPairStats)]),
                "pprs_register_pairs_rigid": (i, [vp, vp, i, i, i, vp, vp, i, vp, vp, vp, vp]),
                "pprs_prefix_register_series_rigid": (i, [vp, vp, i, i, i, vp, vp, vp]),
                "pprs_prefix_register_series": (i, [vp, vp, i, i, i, vp,
                                                    ctypes.POINTER(_CParams),
                                                    ctypes.POINTER(_CSeriesStats),
                                                    ctypes.POINTER(_CPairStats)]),
                "pprs_scan_plan": (i, [i, i, ctypes.POINTER(ctypes.c_int), i,
                                       ctypes.POINTER(ctypes.c_int),
                                       ctypes.POINTER(ctypes.c_int)]),
                "pprs_scan_plan_p": (i, [i, i, i, ctypes.POINTER(ctypes.c_int), i,
                                         ctypes.POINTER(ctypes.c_int),
                                         ctypes.POINTER(ctypes.c_int)]),
                "pprs_scan_program": (i, [i, i, i, ctypes.POINTER(ctypes.c_int), i,
                                          ctypes.POINTER(ctypes.c_int),
                                          ctypes.POINTER(ctypes.c_int),
                                          ctypes.POINTER(ctypes.c_int),
                                          ctypes.POINTER(ctypes.c_int)]),
                "pprs_set_kernel_timing": (i, [vp, i]),
                "pprs_get_kernel_timing": (i, [vp, ctypes.POINTER(ctypes.c_double),
                                               ctypes.POINTER(ctypes.c_longlong),
                                               ctypes.POINTER(ctypes.c_double), i,
                                               ctypes.POINTER(ctypes.c_int), i]),
                "pprs_kernel_name": (ctypes.c_char_p, [i]),
                "pprs_set_pool": (i, [vp, i, i]),
                "pprs_set_metric_solve": (i, [vp, i]),
                "pprs_set_decision_log": (i, [vp, vp, i]),
                "pprs_register_series_batch": (i, [vp, i, ctypes.POINTER(vp),
                                                   ctypes.POINTER(ctypes.c_int),
                                                   ctypes.POINTER(ctypes.c_int),
                                                   ctypes.POINTER(ctypes.c_int),
                                                   ctypes.POINTER(vp), ctypes.POINTER(_CParams),
                                                   ctypes.POINTER(_CSeriesStats),
                                                   ctypes.POINTER(ctypes.c_double)]),
                "pprs_get_tuning": (i, [vp, ctypes.POINTER(_CTuning)]),
                "pprs_set_tuning": (i, [vp, ctypes.POINTER(_CTuning)]),
                "pprs_workspace_query": (i, [i, i, i, ctypes.POINTER(_CParams),
                                             ctypes.POINTER(ctypes.c_size_t)]),
                "pprs_reserve_workspace": (i, [vp, i, i, i, ctypes.POINTER(_CParams)]),
                "pprs_workspace_bytes": (i, [vp, ctypes.POINTER(ctypes.c_size_t)]),
                "pprs_prefix_register_series_batch": (i, [vp, i, ctypes.POINTER(vp),
                                                          ctypes.POINTER(ctypes.c_int),
                                                          ctypes.POINTER(ctypes.c_int),
                                                          ctypes.POINTER(ctypes.c_int),
                                                          ctypes.POINTER(vp),
                                                          ctypes.POINTER(_CParams),
                                                          ctypes.POINTER(_CSeriesStats)]),
            }
            for name, (res, args) in sigs.items():
                fn = getattr(lib, name)
                fn.restype = res
                fn.argtypes = args
            _lib_obj = lib
        return _lib_obj


def _check(status: int) -> int:
    if status < 0:
        raise PprsError(status, _lib().pprs_last_error().decode())
    return status


def default_params() -> Params:
    cp = _CParams()
    _lib().pprs_default_params(ctypes.byref(cp))
    scan = {v: k for k, v in SCAN_KINDS.items()}[cp.scan]
    return Params(cp.levels, cp.lam, cp.beta, cp.armijo_sigma, cp.ladder_k, cp.step_cap,
                  cp.tau_min_rel, cp.eps, cp.iter_max, scan, cp.scan_workers, cp.warm_start,
                  cp.force_fallback)


def scan_plan(kind: str, M: int, workers: int = 0):
    """Host-only schedule: list of (left, right, level) and the number of levels (workers: P
    of the general strategy, 0 for its default)."""
    lib = _lib()
    n = ctypes.c_int()
    lv = ctypes.c_int()
    lib.pprs_scan_plan_p(SCAN_KINDS[kind], M, workers, None, 0, ctypes.byref(n),
                         ctypes.byref(lv))
    buf = (ctypes.c_int * max(3 * n.value, 1))()
    _check(lib.pprs_scan_plan_p(SCAN_KINDS[kind], M, workers, buf, n.value, ctypes.byref(n),
                                ctypes.byref(lv)))
    return [(buf[3 * k], buf[3 * k + 1], buf[3 * k + 2]) for k in range(n.value)], lv.value


SCAN_OPS = {0: "combine", 1: "move", 2: "clear"}


def scan_program(kind: str, M: int, workers: int = 0):
    """Host-only schedule as a program: (instructions [(op, a, b, dst, level)], levels,
    elements, registrations); op is "combine" (x[dst] <- x[a] (.) x[b]), "move" (x[dst] <-
    x[a]) or "clear" (x[dst] <- the identity)."""
    lib = _lib()
    n, lv, ne, nr = (ctypes.c_int() for _ in range(4))
    lib.pprs_scan_program(SCAN_KINDS[kind], M, workers, None, 0, ctypes.byref(n),
                          ctypes.byref(lv), ctypes.byref(ne), ctypes.byref(nr))
    buf = (ctypes.c_int * max(5 * n.value, 1))()
    _check(lib.pprs_scan_program(SCAN_KINDS[kind], M, workers, buf, n.value, ctypes.byref(n),
                                 ctypes.byref(lv), ctypes.byref(ne), ctypes.byref(nr)))
    prog = [(SCAN_OPS[buf[5 * k]], buf[5 * k + 1], buf[5 * k + 2], buf[5 * k + 3],
             buf[5 * k + 4]) for k in range(n.value)]
    return prog, lv.value, ne.value, nr.value


class Context:
    """A libpprs context bound to one device and one HIP stream."""

    def __init__(self, device: int, stream_ptr: int):
        self.device = device
        self.stream_ptr = stream_ptr
        h = ctypes.c_void_p()
        _check(_lib().pprs_create(ctypes.byref(h), device, ctypes.c_void_p(stream_ptr)))
        self.handle = h

    def close(self):
        if self.handle:
            _lib().pprs_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_ctx_cache = {}


def _ctx(device) -> Context:
    import torch
    idx = device.index if device.index is not None else torch.cuda.current_device()
    stream = torch.cuda.current_stream(idx).cuda_stream
    key = (idx, stream)
    c = _ctx_cache.get(key)
    if c is None:
        c = Context(idx, stream)
        _ctx_cache[key] = c
    return c


def _dev_f32(t, name, shape=None, device=None):
    """Device pointer of a contiguous float32 tensor. shape (a tuple) and device, when given,
    must match: the library receives raw pointers and cannot check sizes itself, so a wrong
    shape is refused here, before any kernel could read or write past the tensor."""
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ValueError("%s must be a torch tensor on a HIP device" % name)
    if t.dtype != torch.float32 or not t.is_contiguous():
        raise ValueError("%s must be contiguous float32" % name)
    if shape is not None and tuple(t.shape) != tuple(int(x) for x in shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))
    if device is not None and t.device != device:
        raise ValueError("%s must be on %s, got %s" % (name, device, t.device))
    return ctypes.c_void_p(t.data_ptr())


def _frames3(frames, name="frames"):
    """(N, H, W) of a frame stack [N, H, W]."""
    if frames.dim() != 3:
        raise ValueError("%s must be [N, H, W], got %s" % (name, tuple(frames.shape)))
    return tuple(int(x) for x in frames.shape)


def _pair_stats(s: _CPairStats, levels: int) -> PairStats:
    return PairStats(list(s.iters[:levels]), list(s.passes[:levels]), s.energy, s.ncc, s.flags,
                     s.ms)


def register_pair(f_ref, f_tmpl, u_init=None, params: Params | None = None, out=None):
    """Function A: returns (u [2, H, W] pixels, PairStats)."""
    import torch
    params = params or Params()
    if f_ref.dim() != 2:
        raise ValueError("f_ref must be [H, W], got %s" % (tuple(f_ref.shape),))
    H, W = f_ref.shape
    dev = f_ref.device
    if out is None:
        out = torch.empty((2, H, W), device=dev, dtype=torch.float32)
    st = _CPairStats()
    cp = params.c()
    a_ref = _dev_f32(f_ref, "f_ref")
    a_tmpl = _dev_f32(f_tmpl, "f_tmpl", (H, W), dev)
    a_init = _dev_f32(u_init, "u_init", (2, H, W), dev) if u_init is not None else None
    a_out = _dev_f32(out, "out", (2, H, W), dev)
    c = _ctx(dev)
    _check(_lib().pprs_register_pair(c.handle, a_ref, a_tmpl, H, W, a_init, a_out,
                                     ctypes.byref(cp), ctypes.byref(st)))
    return out, _pair_stats(st, params.levels)


def register_pair_noalloc(f_ref, f_tmpl, out, u_init=None, params: Params | None = None):
    """Function A through pprs_register_pair_noalloc: the library allocates nothing (its
    buffers lie in a fixed per-device scratch array; frames up to 512 x 512). out [2, H, W] is
    the caller's. Returns (out, PairStats)."""
    params = params or Params()
    if f_ref.dim() != 2:
        raise ValueError("f_ref must be [H, W], got %s" % (tuple(f_ref.shape),))
    H, W = f_ref.shape
    dev = f_ref.device
    st = _CPairStats()
    cp = params.c()
    a_ref = _dev_f32(f_ref, "f_ref")
    a_tmpl = _dev_f32(f_tmpl, "f_tmpl", (H, W), dev)
    a_init = _dev_f32(u_init, "u_init", (2, H, W), dev) if u_init is not None else None
    a_out = _dev_f32(out, "out", (2, H, W), dev)
    c = _ctx(dev)
    _check(_lib().pprs_register_pair_noalloc(c.handle, a_ref, a_tmpl, H, W, a_init, a_out,
                                             ctypes.byref(cp), ctypes.byref(st)))
    return out, _pair_stats(st, params.levels)


def register_pairs(frames, ref, tmpl, params: Params | None = None, out=None):
    """Function A on pairs (frames[ref[p]], frames[tmpl[p]]) of frames [N, H, W]: returns
    (u [P, 2, H, W] pixels, [PairStats])."""
    import numpy as np
    import torch
    params = params or Params()
    ref = np.ascontiguousarray(ref, dtype=np.int32)
    tmpl = np.ascontiguousarray(tmpl, dtype=np.int32)
    if ref.shape != tmpl.shape or ref.ndim != 1:
        raise ValueError("ref and tmpl must be 1-D index arrays of one length")
    N, H, W = _frames3(frames)
    P = len(ref)
    if out is None:
        out = torch.empty((P, 2, H, W), device=frames.device, dtype=torch.float32)
    st = (_CPairStats * max(P, 1))()
    cp = params.c()
    a_fr = _dev_f32(frames, "frames")
    a_out = _dev_f32(out, "out", (P, 2, H, W), frames.device)
    c = _ctx(frames.device)
    _check(_lib().pprs_register_pairs(c.handle, a_fr, N, H, W, ref.ctypes.data,
                                      tmpl.ctypes.data, P, a_out, ctypes.byref(cp), st))
    return out, [_pair_stats(st[k], params.levels) for k in range(P)]


def compose_deformations(u_ij, u_jk, out=None):
    """(phi_jk o phi_ij) as a displacement [2, H, W] in pixels."""
    import torch
    if u_ij.dim() != 3 or u_ij.shape[0] != 2:
        raise ValueError("u_ij must be [2, H, W], got %s" % (tuple(u_ij.shape),))
    _, H, W = u_ij.shape
    if out is None:
        out = torch.empty_like(u_ij)
    dev = u_ij.device
    a_ij = _dev_f32(u_ij, "u_ij")
    a_jk = _dev_f32(u_jk, "u_jk", (2, H, W), dev)
    a_out = _dev_f32(out, "out", (2, H, W), dev)
    c = _ctx(dev)
    _check(_lib().pprs_compose_deformations(c.handle, a_ij, a_jk, a_out, H, W))
    return out


def register_pairs_rigid(frames, ref, tmpl, params: Params | None = None, p_init=None):
    """Rigid variant: pairs (ref[k], tmpl[k]) of frames [N, H, W]; phi_k(x) = R(alpha) x + t
    about pixel (0, 0). Returns (p [P, 3] float64: alpha (rad), t0, t1 (px), stats list)."""
    import numpy as np
    params = params or Params()
    N, H, W = _frames3(frames)
    ref = np.ascontiguousarray(ref, dtype=np.int32)
    tmpl = np.ascontiguousarray(tmpl, dtype=np.int32)
    if ref.ndim != 1 or ref.shape != tmpl.shape:
        raise ValueError("ref and tmpl must be 1-D index arrays of one length")
    P = ref.shape[0]
    out = np.zeros((max(P, 1), 3))
    pin = None
    if p_init is not None:
        pin = np.ascontiguousarray(p_init, dtype=np.float64)
        if pin.size != 3 * P:
            raise ValueError("p_init must hold 3 parameters per pair")
        pin = pin.reshape(P, 3)
    st = (_CPairStats * max(P, 1))()
    cp = params.c()
    c = _ctx(frames.device)
    _check(_lib().pprs_register_pairs_rigid(
        c.handle, _dev_f32(frames, "frames"), N, H, W, ref.ctypes.data, tmpl.ctypes.data, P,
        pin.ctypes.data if pin is not None else None, out.ctypes.data, ctypes.byref(cp), st))
    return out[:P], [_pair_stats(st[k], params.levels) for k in range(P)]


def prefix_register_series_rigid(frames, params: Params | None = None):
    """Rigid series: frames [N, H, W] -> (p [N, 3] float64: phi_0i as alpha (rad), t0, t1 (px),
    p[0] = 0; SeriesStats)."""
    import numpy as np
    params = params or Params()
    N, H, W = _frames3(frames)
    out = np.zeros((N, 3))
    ss = _CSeriesStats()
    cp = params.c()
    c = _ctx(frames.device)
    _check(_lib().pprs_prefix_register_series_rigid(
        c.handle, _dev_f32(frames, "frames"), N, H, W, out.ctypes.data, ctypes.byref(cp),
        ctypes.byref(ss)))
    stats = SeriesStats(ss.n_ops_a, ss.n_ops_b, ss.n_scan_levels, ss.flags_or, ss.ms_total,
                        ss.ms_prepare, ss.ms_preprocess, ss.ms_scan, ss.node_steps,
                        ss.node_passes)
    return out, stats


def series_average(frames, u, out=None):
    """Average of the aligned frames f_i o phi_{0,i}: [H, W] from frames [N, H, W] and the
    series result u [N, 2, H, W] (pixels)."""
    import torch
    N, H, W = _frames3(frames)
    if tuple(u.shape) != (N, 2, H, W):
        raise PprsError(-1, "u must be [N, 2, H, W] for frames [N, H, W]")
    if out is None:
        out = torch.empty((H, W), device=frames.device, dtype=torch.float32)
    dev = frames.device
    a_fr = _dev_f32(frames, "frames")
    a_u = _dev_f32(u, "u", (N, 2, H, W), dev)
    a_out = _dev_f32(out, "out", (H, W), dev)
    c = _ctx(dev)
    _check(_lib().pprs_series_average(c.handle, a_fr, a_u, N, H, W, a_out))
    return out


def series_average_refine(frames, u, passes: int = 1, params: Params | None = None, avg=None):
    """The series averaging procedure: `passes` rounds of averaging the aligned frames and
    re-registering each frame i >= 1 to the average from its current u_i. u [N, 2, H, W]
    (pixels, float32 on the frames' device) is refined in place. Returns (u, average of the
    final alignment [H, W], [[PairStats] * (N-1)] per pass)."""
    import torch
    params = params or Params()
    N, H, W = _frames3(frames)
    if int(passes) < 0:
        raise ValueError("passes must be >= 0")
    dev = frames.device
    if avg is None:
        avg = torch.empty((H, W), device=dev, dtype=torch.float32)
    n = int(passes) * (N - 1)
    st = (_CPairStats * max(n, 1))()
    cp = params.c()
    a_fr = _dev_f32(frames, "frames")
    a_u = _dev_f32(u, "u", (N, 2, H, W), dev)
    a_avg = _dev_f32(avg, "avg", (H, W), dev)
    c = _ctx(dev)
    _check(_lib().pprs_series_average_refine(c.handle, a_fr, N, H, W, a_u, int(passes),
                                             ctypes.byref(cp), a_avg, st))
    rows = [[_pair_stats(st[q * (N - 1) + r], params.levels) for r in range(N - 1)]
            for q in range(int(passes))]
    return u, avg, rows


def prefix_register_series(frames, params: Params | None = None, out=None,
                           want_op_stats: bool = False):
    """Series registration: returns (u [N, 2, H, W] pixels with u[0] = 0, SeriesStats,
    op stats list or None)."""
    import torch
    params = params or Params()
    N, H, W = _frames3(frames)
    if out is None:
        out = torch.empty((N, 2, H, W), device=frames.device, dtype=torch.float32)
    a_fr = _dev_f32(frames, "frames")
    a_out = _dev_f32(out, "out", (N, 2, H, W), frames.device)
    ss = _CSeriesStats()
    ops = None
    if want_op_stats:
        n_b = scan_program(params.scan, max(N - 1, 0), params.scan_workers)[3]
        ops = (_CPairStats * max(N - 1 + n_b, 1))()   # N-1 A entries, then the B entries
    cp = params.c()
    c = _ctx(frames.device)
    _check(_lib().pprs_prefix_register_series(c.handle, a_fr, N, H, W, a_out, ctypes.byref(cp),
                                              ctypes.byref(ss), ops))
    stats = SeriesStats(ss.n_ops_a, ss.n_ops_b, ss.n_scan_levels, ss.flags_or, ss.ms_total,
                        ss.ms_prepare, ss.ms_preprocess, ss.ms_scan, ss.node_steps,
                        ss.node_passes)
    op_list = None
    if want_op_stats:
        op_list = [_pair_stats(ops[k], params.levels) for k in range(ss.n_ops_a + ss.n_ops_b)]
    return out, stats, op_list


def workspace_query(N: int, H: int, W: int, params: Params | None = None) -> int:
    """Device bytes a series call of N frames of H x W keeps in its context (no HIP call)."""
    params = params or Params()
    b = ctypes.c_size_t()
    cp = params.c()
    _check(_lib().pprs_workspace_query(N, H, W, ctypes.byref(cp), ctypes.byref(b)))
    return b.value


def reserve_workspace(N: int, H: int, W: int, params: Params | None = None, device=None):
    """Allocates, on the current stream's context, what a series call of that size needs."""
    import torch
    params = params or Params()
    dev = device or torch.device("cuda", torch.cuda.current_device())
    cp = params.c()
    _check(_lib().pprs_reserve_workspace(_ctx(dev).handle, N, H, W, ctypes.byref(cp)))


def workspace_bytes(device=None) -> int:
    """Device bytes the current stream's context holds in its workspace."""
    import torch
    dev = device or torch.device("cuda", torch.cuda.current_device())
    b = ctypes.c_size_t()
    _check(_lib().pprs_workspace_bytes(_ctx(dev).handle, ctypes.byref(b)))
    return b.value


def set_pool(slots: int = 0, group_steps: int = 0, device=None):
    """Slot-pool shape of later series calls on the current stream's context (0 = default)."""
    import torch
    dev = device or torch.device("cuda", torch.cuda.current_device())
    _check(_lib().pprs_set_pool(_ctx(dev).handle, slots, group_steps))


class DecisionLog:
    """Records the line-search decision of every accepted step of the registrations of later
    calls on the current stream's context (pprs_set_decision_log): `rows` registrations of up
    to `cap` steps each, in a device buffer this object owns. Use as a context manager."""

    def __init__(self, rows: int, cap: int = 2048, device=None):
        import torch
        self.dev = device or torch.device("cuda", torch.cuda.current_device())
        self.buf = torch.zeros((max(rows, 1), cap), dtype=torch.uint8, device=self.dev)
        self.cap = cap

    def __enter__(self):
        _check(_lib().pprs_set_decision_log(_ctx(self.dev).handle,
                                            ctypes.c_void_p(self.buf.data_ptr()), self.cap))
        return self

    def __exit__(self, *exc):
        _check(_lib().pprs_set_decision_log(_ctx(self.dev).handle, None, 0))
        return False

    def rungs(self, row: int, steps: int):
        """Ladder positions of the first `steps` accepted steps of registration `row`."""
        if steps > self.cap:
            raise ValueError("the log holds %d steps per registration" % self.cap)
        return self.buf[row, :steps].cpu().numpy().astype(int).tolist()


def set_metric_solve(mode: str = "exact", device=None):
    """"exact": two passes of line solves (default); "window": one windowed pass where beta
    allows it."""
    import torch
    dev = device or torch.device("cuda", torch.cuda.current_device())
    _check(_lib().pprs_set_metric_solve(_ctx(dev).handle, {"exact": 0, "window": 1}[mode]))


def get_tuning(device=None) -> dict:
    """Launch shape of the current stream's context (see pprs_tuning)."""
    import torch
    dev = device or torch.device("cuda", torch.cuda.current_device())
    t = _CTuning()
    _check(_lib().pprs_get_tuning(_ctx(dev).handle, ctypes.byref(t)))
    return {k: getattr(t, k) for k in TUNING_KEYS}


def set_tuning(tuning: dict, device=None):
    """Sets the launch shape (missing keys keep their value; 0 means the default)."""
    import torch
    dev = device or torch.device("cuda", torch.cuda.current_device())
    cur = get_tuning(dev)
    cur.update({k: int(v) for k, v in tuning.items() if k in TUNING_KEYS})
    t = _CTuning(**cur)
    _check(_lib().pprs_set_tuning(_ctx(dev).handle, ctypes.byref(t)))


def register_series_batch(series, params: Params | None = None, levels=None, outs=None):
    """Several independent series (a list of device tensors [N_j, side_j, side_j]) in one run
    of the slot pool; `levels` optionally gives each series' level count. Returns (list of
    u [N_j, 2, side_j, side_j], list of SeriesStats, list of per-series latencies in ms)."""
    import torch
    params = params or Params()
    S = len(series)
    if S < 1:
        raise ValueError("at least one series")
    dev = series[0].device
    for j, f in enumerate(series):
        N, H, W = _frames3(f, "series[%d]" % j)
        if H != W:
            raise ValueError("series[%d] frames must be square, got %dx%d" % (j, H, W))
    if outs is None:
        outs = [torch.empty((f.shape[0], 2, f.shape[1], f.shape[2]), device=f.device,
                            dtype=torch.float32) for f in series]
    if len(outs) != S:
        raise ValueError("outs must hold one tensor per series")
    if levels is not None and len(levels) != S:
        raise ValueError("levels must hold one count per series")
    fr = (ctypes.c_void_p * S)(*[_dev_f32(f, "series[%d]" % j, None, dev).value
                                 for j, f in enumerate(series)])
    uo = (ctypes.c_void_p * S)(*[_dev_f32(u, "outs[%d]" % j,
                                          (f.shape[0], 2, f.shape[1], f.shape[2]), dev).value
                                 for j, (f, u) in enumerate(zip(series, outs))])
    ns = (ctypes.c_int * S)(*[int(f.shape[0]) for f in series])
    sd = (ctypes.c_int * S)(*[int(f.shape[1]) for f in series])
    st = (_CSeriesStats * S)()
    lat = (ctypes.c_double * S)()
    cp = params.c()
    c = _ctx(series[0].device)
    lv = (ctypes.c_int * S)(*[int(x) for x in levels]) if levels is not None else None
    _check(_lib().pprs_register_series_batch(c.handle, S, fr, ns, sd, lv, uo, ctypes.byref(cp),
                                             st, lat))
    stats = [SeriesStats(x.n_ops_a, x.n_ops_b, x.n_scan_levels, x.flags_or, x.ms_total,
                         x.ms_prepare, x.ms_preprocess, x.ms_scan, x.node_steps, x.node_passes)
             for x in st]
    return outs, stats, list(lat)


def prefix_register_series_batch(series, params: Params | None = None, outs=None):
    """pprs_prefix_register_series_batch: several series [N_j, H_j, W_j] (H_j == W_j), one
    level count for all. Returns (list of u [N_j, 2, H_j, W_j], list of SeriesStats)."""
    import torch
    params = params or Params()
    S = len(series)
    if S < 1:
        raise ValueError("at least one series")
    dev = series[0].device
    shapes = [_frames3(f, "series[%d]" % j) for j, f in enumerate(series)]
    if outs is None:
        outs = [torch.empty((N, 2, H, W), device=dev, dtype=torch.float32)
                for (N, H, W) in shapes]
    if len(outs) != S:
        raise ValueError("outs must hold one tensor per series")
    fr = (ctypes.c_void_p * S)(*[_dev_f32(f, "series[%d]" % j, None, dev).value
                                 for j, f in enumerate(series)])
    uo = (ctypes.c_void_p * S)(*[_dev_f32(u, "outs[%d]" % j, (N, 2, H, W), dev).value
                                 for j, (u, (N, H, W)) in enumerate(zip(outs, shapes))])
    ns = (ctypes.c_int * S)(*[x[0] for x in shapes])
    hs = (ctypes.c_int * S)(*[x[1] for x in shapes])
    ws = (ctypes.c_int * S)(*[x[2] for x in shapes])
    st = (_CSeriesStats * S)()
    cp = params.c()
    _check(_lib().pprs_prefix_register_series_batch(_ctx(dev).handle, S, fr, ns, hs, ws, uo,
                                                    ctypes.byref(cp), st))
    stats = [SeriesStats(x.n_ops_a, x.n_ops_b, x.n_scan_levels, x.flags_or, x.ms_total,
                         x.ms_prepare, x.ms_preprocess, x.ms_scan, x.node_steps, x.node_passes)
             for x in st]
    return outs, stats


def set_kernel_timing(enable: bool, device=None):
    import torch
    dev = device or torch.device("cuda", torch.cuda.current_device())
    _check(_lib().pprs_set_kernel_timing(_ctx(dev).handle, 1 if enable else 0))


def kernel_names():
    lib = _lib()
    names = []
    while True:
        nm = lib.pprs_kernel_name(len(names)).decode()
        if nm == "unknown":
            return names
        names.append(nm)


def kernel_timing(reset: bool = False, device=None):
    """{kernel kind: (total ms, launches, algorithmic bytes)} since the last reset."""
    import torch
    dev = device or torch.device("cuda", torch.cuda.current_device())
    cap = 16
    ms = (ctypes.c_double * cap)()
    la = (ctypes.c_longlong * cap)()
    by = (ctypes.c_double * cap)()
    nk = ctypes.c_int()
    _check(_lib().pprs_get_kernel_timing(_ctx(dev).handle, ms, la, by, cap, ctypes.byref(nk),
                                         1 if reset else 0))
    names = kernel_names()
    return {names[k]: (ms[k], la[k], by[k]) for k in range(nk.value)}


# ------------------------------------------------------------------------------------------ #
# Learned warm start

def _cnn_sigs(lib):
    vp = ctypes.c_void_p
    i = ctypes.c_int
    sigs = {
        "pprs_cnn_create": (i, [ctypes.POINTER(vp), i, vp, ctypes.c_ulonglong]),
        "pprs_cnn_destroy": (None, [vp]),
        "pprs_cnn_last_error": (ctypes.c_char_p, []),
        "pprs_cnn_param_count": (ctypes.c_size_t, [vp]),
        "pprs_cnn_set_params": (i, [vp, vp, ctypes.c_size_t]),
        "pprs_cnn_get_params": (i, [vp, vp, ctypes.c_size_t]),
        "pprs_cnn_load": (i, [vp, ctypes.c_char_p, ctypes.c_size_t]),
        "pprs_cnn_forward": (i, [vp, vp, i, vp]),
        "pprs_cnn_gradients": (i, [vp, vp, vp, i, i, ctypes.POINTER(ctypes.c_double), vp]),
        "pprs_cnn_train_step": (i, [vp, vp, vp, i, i, ctypes.c_float,
                                    ctypes.POINTER(ctypes.c_double)]),
        "pprs_pair_inputs": (i, [vp, vp, i, i, i, vp, vp, i, vp]),
        "pprs_level7_targets": (i, [vp, vp, i, i, i, vp]),
        "pprs_set_warm_start": (i, [vp, vp, ctypes.c_double, i]),
        "pprs_set_warm_sides": (i, [vp, ctypes.c_uint]),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


def _cnn_check(status: int):
    if status < 0:
        lib = _lib()
        msg = lib.pprs_cnn_last_error().decode() or lib.pprs_last_error().decode()
        raise PprsError(status, msg)
    return status


class WarmStartNet:
    """The BF16 encoder-decoder of the warm start (weights live on the device)."""

    def __init__(self, seed: int = 0, device=None):
        import torch
        dev = device or torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        lib = _cnn_sigs(_lib())
        h = ctypes.c_void_p()
        stream = torch.cuda.current_stream(dev).cuda_stream
        _cnn_check(lib.pprs_cnn_create(ctypes.byref(h), dev.index or 0, ctypes.c_void_p(stream),
                                       seed))
        self.handle = h
        self.n_params = lib.pprs_cnn_param_count(h)

    def close(self):
        if getattr(self, "handle", None):
            _lib().pprs_cnn_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self):
        import numpy as np
        out = np.empty(self.n_params, dtype=np.float32)
        _cnn_check(_lib().pprs_cnn_get_params(self.handle, out.ctypes.data, out.size))
        return out

    def set_params(self, params):
        import numpy as np
        p = np.ascontiguousarray(params, dtype=np.float32)
        _cnn_check(_lib().pprs_cnn_set_params(self.handle, p.ctypes.data, p.size))

    def forward(self, x):
        """x [B, 128, 128, 2] float32 on the device -> [B, 128, 128, 2]."""
        import torch
        B = _net_batch(x, "x")
        y = torch.empty_like(x)
        _cnn_check(_lib().pprs_cnn_forward(self.handle, _dev_f32(x, "x"), B, _dev_f32(y, "y")))
        return y

    def gradients(self, x, target, margin: int = 4):
        import numpy as np
        g = np.empty(self.n_params, dtype=np.float32)
        loss = ctypes.c_double()
        B = _net_batch(x, "x")
        a_t = _dev_f32(target, "target", tuple(x.shape), x.device)
        _cnn_check(_lib().pprs_cnn_gradients(self.handle, _dev_f32(x, "x"), a_t, B, margin,
                                             ctypes.byref(loss), g.ctypes.data))
        return loss.value, g

    def train_step(self, x, target, lr: float, margin: int = 4) -> float:
        loss = ctypes.c_double()
        B = _net_batch(x, "x")
        a_t = _dev_f32(target, "target", tuple(x.shape), x.device)
        _cnn_check(_lib().pprs_cnn_train_step(self.handle, _dev_f32(x, "x"), a_t, B, margin, lr,
                                              ctypes.byref(loss)))
        return loss.value

    def save(self, path: str):
        from safetensors.numpy import save_file
        save_file({"params": self.get_params()}, path)

    def load(self, path: str):
        """Reads a weights file (safetensors layout, one F32 tensor "params"); the library
        parses it (pprs_cnn_load)."""
        with open(path, "rb") as f:
            blob = f.read()
        self.load_bytes(blob)

    def load_bytes(self, blob: bytes):
        _cnn_check(_lib().pprs_cnn_load(self.handle, blob, len(blob)))


def _net_batch(x, name):
    """B of a network tensor [B, 128, 128, 2]."""
    if x.dim() != 4 or tuple(x.shape[1:]) != (128, 128, 2):
        raise ValueError("%s must be [B, 128, 128, 2], got %s" % (name, tuple(x.shape)))
    return int(x.shape[0])


def pair_inputs(frames, ref, tmpl):
    """Network inputs [P, 128, 128, 2] for frame pairs (ref[p], tmpl[p]) of frames [N, H, W]."""
    import numpy as np
    import torch
    _cnn_sigs(_lib())
    ref = np.ascontiguousarray(ref, dtype=np.int32)
    tmpl = np.ascontiguousarray(tmpl, dtype=np.int32)
    if ref.ndim != 1 or ref.shape != tmpl.shape:
        raise ValueError("ref and tmpl must be 1-D index arrays of one length")
    N, H, W = _frames3(frames)
    out = torch.empty((len(ref), 128, 128, 2), device=frames.device, dtype=torch.float32)
    c = _ctx(frames.device)
    _check(_lib().pprs_pair_inputs(c.handle, _dev_f32(frames, "frames"), N, H, W,
                                   ref.ctypes.data, tmpl.ctypes.data, len(ref),
                                   _dev_f32(out, "out")))
    return out


def level7_targets(u):
    """Displacements u [P, 2, H, W] (pixels) -> level-7 targets [P, 128, 128, 2] (cells)."""
    import torch
    _cnn_sigs(_lib())
    if u.dim() != 4 or u.shape[1] != 2:
        raise ValueError("u must be [P, 2, H, W], got %s" % (tuple(u.shape),))
    P, _, H, W = u.shape
    out = torch.empty((P, 128, 128, 2), device=u.device, dtype=torch.float32)
    c = _ctx(u.device)
    _check(_lib().pprs_level7_targets(c.handle, _dev_f32(u, "u"), P, H, W,
                                      _dev_f32(out, "out")))
    return out


WARM_MODES = {"refine": 0, "skip": 1}


def set_warm_start(net, max_cells: float = 8.0, mode: str = "refine", sides=None,
                   device=None):
    """Use `net` (or None) to warm-start later series and pair-batch calls on the current
    stream's context. mode "refine": the prediction becomes the coarsest-level initial guess;
    "skip": registrations start on level 7 from it and skip the coarser levels. `sides`
    (e.g. the sides the network was trained on) limits it to those frame sides."""
    import torch
    _cnn_sigs(_lib())
    dev = device or torch.device("cuda", torch.cuda.current_device())
    c = _ctx(dev)
    _check(_lib().pprs_set_warm_start(c.handle, net.handle if net else None, max_cells,
                                      WARM_MODES[mode]))
    mask = 0xFFFFFFFF
    if sides is not None:
        mask = 0
        for sd in sides:
            mask |= 1 << (int(sd).bit_length() - 1)  # side 2^L or 2^L + 1
    _check(_lib().pprs_set_warm_sides(c.handle, mask))
    c.warm_net = net  # the context refers to the network's device memory: keep it alive
