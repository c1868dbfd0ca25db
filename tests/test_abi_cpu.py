"""Host-side tests of libpprs (no GPU): the library loads and exports every symbol declared in
include/pprs.h, and the scan planner (pure host logic) produces correct schedules."""
import json
import math
import os
import re
import ctypes

import numpy as np
import pytest

import paper_1712_02533_amd as P
from paper_1712_02533_amd import api

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLD = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_values.json")))


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "pprs.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pprs_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(api.LIB_PATH)
    syms = declared_symbols()
    assert len(syms) >= 11
    for s in syms:
        assert hasattr(lib, s), s


def test_default_params_match_binding_defaults():
    assert P.default_params() == P.Params()


def _apply(plan, xs, op):
    xs = list(xs)
    for left, right, _ in plan:
        xs[right] = op(xs[left], xs[right])
    return xs


def _interval(a, b):
    assert a[1] == b[0], "operands do not share their middle index"
    return (a[0], b[1])


@pytest.mark.parametrize("kind", ["sequential", "brent_kung", "kogge_stone", "sklansky",
                                  "general", "general/1", "general/3", "general/M"])
@pytest.mark.parametrize("M", [0, 1, 2, 3, 7, 8, 9, 63, 64, 100, 511])
def test_plan_matches_sequential_scan_with_associative_ops(kind, M):
    workers = 0
    if "/" in kind:
        kind, w = kind.split("/")
        workers = M if w == "M" else int(w)
    plan, levels = P.scan_plan(kind, M, workers)
    # interval concatenation: exactly associative, non-commutative, checks index matching
    xs = [(m, m + 1) for m in range(M)]
    assert _apply(plan, xs, _interval) == [(0, m + 1) for m in range(M)]
    # 2x2 integer matrix products (exact, non-commutative)
    rng = np.random.default_rng(M)
    mats = [rng.integers(-2, 3, size=(2, 2)) for _ in range(M)]
    got = _apply(plan, mats, lambda a, b: a @ b)
    acc = None
    for m in range(M):
        acc = mats[m] if acc is None else acc @ mats[m]
        assert np.array_equal(got[m], acc)
    # ops of one level are independent: in list order no op reads an element that an earlier
    # op of its level wrote (Kogge-Stone relies on its right-to-left order for this), and no
    # element is written twice in a level
    by_level = {}
    for left, right, lv in plan:
        by_level.setdefault(lv, []).append((left, right))
    for ops in by_level.values():
        written = set()
        for left, right in ops:
            assert left not in written and right not in written
            written.add(right)
    assert len(by_level) == levels
    assert [lv for _, _, lv in plan] == sorted(lv for _, _, lv in plan)


def test_plan_counts_match_paper_figures_and_table():
    fig = GOLD["scan_figures_N8"]
    for kind in ("sequential", "brent_kung", "kogge_stone", "sklansky"):
        plan, levels = P.scan_plan(kind, 8)
        assert len(plan) == fig[kind]["ops"] and levels == fig[kind]["steps"]
    for k in range(1, 11):
        N = 2 ** k
        # work and span of the Kogge-Stone and Sklansky sections: N log2 N - N + 1 and
        # N/2 log2 N operator applications, log2 N steps each
        plan, levels = P.scan_plan("kogge_stone", N)
        assert len(plan) == N * k - N + 1 and levels == k
        plan, levels = P.scan_plan("sklansky", N)
        assert len(plan) == N // 2 * k and levels == k
        for kind in ("kogge_stone", "sklansky"):
            plan, levels = P.scan_plan(kind, N)
            assert len(plan) + levels >= 2 * N - 2    # Snir: size + depth >= 2N - 2
    for k in range(1, 11):
        N = 2 ** k
        plan, levels = P.scan_plan("brent_kung", N)
        assert len(plan) == 2 * N - k - 2                 # work, Brent-Kung row of the table
        assert levels == max(2 * k - 1, 1) if N > 1 else True  # span
        assert len(plan) + levels >= 2 * N - 2            # Snir: size + depth >= 2N - 2
        plan, levels = P.scan_plan("sequential", N)
        assert len(plan) == N - 1 and levels == N - 1


def _bk_work_span(n):
    plan, levels = P.scan_plan("brent_kung", n)
    return len(plan), levels


@pytest.mark.parametrize("M,workers", [(8, 2), (12, 3), (12, 4), (64, 8), (511, 7), (511, 73),
                                       (100, 10)])
def test_general_strategy_counts_match_the_chapter(M, workers):
    """General strategy, even division (M = P K): local stage one is P serial scans of K
    elements (M - P ops, K - 1 steps), the global stage a Brent-Kung scan of the P chunk ends,
    local stage two P - 1 workers each combining K - 1 elements (the chunk end is final after
    the inclusive global stage; the chapter's exclusive form touches all K): one step."""
    assert M % workers == 0
    K = M // workers
    plan, levels = P.scan_plan("general", M, workers)
    w_gs, s_gs = _bk_work_span(workers)
    assert len(plan) == (M - workers) + w_gs + (workers - 1) * (K - 1)
    assert levels == (K - 1) + s_gs + (1 if K > 1 and workers > 1 else 0)
    # one worker is the serial scan; one element per worker is Brent-Kung over all elements
    assert P.scan_plan("general", M, 1) == P.scan_plan("sequential", M)
    assert P.scan_plan("general", M, M) == P.scan_plan("brent_kung", M)
    # uneven division: the first M mod P workers hold one element more
    plan, _ = P.scan_plan("general", M + 1, workers)
    firsts = sorted({left + 1 for left, right, lv in plan if lv == 0})
    assert len(firsts) == workers and firsts[1] - firsts[0] == K + 1


def test_plan_rejects_bad_arguments():
    n = ctypes.c_int()
    lv = ctypes.c_int()
    lib = api._lib()
    assert lib.pprs_scan_plan(7, 8, None, 0, ctypes.byref(n), ctypes.byref(lv)) == -1
    assert lib.pprs_scan_plan(5, 8, None, 0, ctypes.byref(n), ctypes.byref(lv)) == -1
    assert lib.pprs_scan_plan_p(4, 8, -1, None, 0, ctypes.byref(n), ctypes.byref(lv)) == -1
    assert lib.pprs_scan_plan(-1, 8, None, 0, ctypes.byref(n), ctypes.byref(lv)) == -1
    assert lib.pprs_scan_plan(1, -1, None, 0, ctypes.byref(n), ctypes.byref(lv)) == -1
    buf = (ctypes.c_int * 3)()
    assert lib.pprs_scan_plan(1, 8, buf, 1, ctypes.byref(n), ctypes.byref(lv)) == -1
    assert n.value == 11


def test_workspace_query_host_only():
    """pprs_workspace_query makes no HIP call: the series workspace is planned on the host.
    It grows with the frame count and side, is 0 for a one-frame series (nothing to register)
    and refuses bad sizes."""
    p = P.Params()
    b512 = P.workspace_query(512, 512, 512, p)
    b64 = P.workspace_query(64, 512, 512, p)
    b256 = P.workspace_query(64, 256, 256, P.Params(levels=3))
    assert b512 > b64 > b256 > 0
    assert P.workspace_query(1, 512, 512, p) == 0
    # the version buffers alone: one [2][513][513] float field per A and B application
    assert b512 > (511 + 1004) * 2 * 513 * 513 * 4
    # and the whole stays far inside one MI355X's 288 GB
    assert b512 < 32 * 2 ** 30
    for bad in [(0, 512, 512), (8, 500, 500), (8, 512, 256)]:
        with pytest.raises(api.PprsError):
            P.workspace_query(*bad, p)
    with pytest.raises(api.PprsError):
        P.workspace_query(8, 64, 64, P.Params(levels=7))
    # the warm-start switches are 0 or 1 (defaults: warm start where a network is set, no forced
    # fallback)
    assert (p.warm_start, p.force_fallback) == (1, 0)
    for bad in [P.Params(warm_start=2), P.Params(force_fallback=-1)]:
        with pytest.raises(api.PprsError):
            P.workspace_query(8, 64, 64, bad)


def test_wrong_shapes_are_refused_before_the_library():
    """The binding checks every tensor's shape against the call's sizes before it passes raw
    pointers on (the library cannot check the extent of a device pointer). CPU tensors stand in
    for device tensors: each refusal happens before the device check would matter."""
    import torch
    with pytest.raises(ValueError):
        api._frames3(torch.zeros(4, 4))
    with pytest.raises(ValueError):
        api._net_batch(torch.zeros(2, 128, 128, 3), "x")
    assert api._net_batch(torch.zeros(3, 128, 128, 2), "x") == 3
    assert api._frames3(torch.zeros(5, 8, 8)) == (5, 8, 8)


def _run_program(prog, n_elems, xs, op):
    """Executes a scan program on host values xs (M of them) with the operator op; scratch
    elements start as the identity (None), a combination with it is the other operand.
    Returns (final elements, operator applications)."""
    v = list(xs) + [None] * (n_elems - len(xs))
    n = 0
    for code, a, b, dst, _ in prog:
        if code == "clear":
            v[dst] = None
        elif code == "move":
            v[dst] = v[a]
        elif v[a] is None or v[b] is None:
            v[dst] = v[b] if v[a] is None else v[a]
        else:
            v[dst] = op(v[a], v[b])
            n += 1
    return v, n


@pytest.mark.parametrize("kind", ["sequential", "brent_kung", "kogge_stone", "sklansky",
                                  "general", "blelloch", "reduce_then_scan",
                                  "reduce_then_scan/1", "reduce_then_scan/3",
                                  "reduce_then_scan/M"])
@pytest.mark.parametrize("M", [0, 1, 2, 3, 7, 8, 9, 63, 64, 100, 511])
def test_program_matches_sequential_scan_with_associative_ops(kind, M):
    """Every schedule as a program (pprs_scan_program) computes the inclusive scan with exactly
    associative, non-commutative operators (interval concatenation, which also checks that
    operands share their middle index, and 2x2 integer matrix products), reports its operator
    applications, and its combines of one level are independent."""
    workers = 0
    if "/" in kind:
        kind, w = kind.split("/")
        workers = M if w == "M" else int(w)
    prog, levels, n_elems, n_reg = P.scan_program(kind, M, workers)
    xs = [(m, m + 1) for m in range(M)]
    out, n = _run_program(prog, n_elems, xs, _interval)
    assert out[:M] == [(0, m + 1) for m in range(M)] and n == n_reg
    rng = np.random.default_rng(M + 7)
    mats = [rng.integers(-2, 3, size=(2, 2)) for _ in range(M)]
    out, _ = _run_program(prog, n_elems, mats, lambda a, b: a @ b)
    acc = None
    for m in range(M):
        acc = mats[m] if acc is None else acc @ mats[m]
        assert np.array_equal(out[m], acc)
    by_level = {}
    for code, a, b, dst, lv in prog:
        if code == "combine":
            by_level.setdefault(lv, []).append((a, b, dst))
    for ops in by_level.values():
        written = set()
        for a, b, dst in ops:
            assert a not in written and b not in written and dst not in written
            written.add(dst)
    if kind in ("sequential", "brent_kung", "kogge_stone", "sklansky", "general"):
        plan, lv = P.scan_plan(kind, M, workers)
        assert [(a, b, lvl) for c, a, b, d, lvl in prog] == plan and levels == lv


def test_blelloch_program_counts_match_the_chapter():
    """Blelloch (Prefix sum chapter): 2 log2 N steps and 2(N - 1) operator applications (figure:
    6 and 14 for 8 elements), of which log2 N combine with the identity element (the leftmost
    path of the down-sweep) and cost nothing; Snir's bound holds for the applications made."""
    fig = GOLD["scan_figures_N8"]["blelloch"]
    for k in range(1, 11):
        N = 2 ** k
        prog, levels, n_elems, n_reg = P.scan_program("blelloch", N)
        combines = sum(1 for x in prog if x[0] == "combine")
        assert levels == 2 * k and combines == 2 * (N - 1)          # span and work, table
        assert n_reg == combines - k
        assert n_reg + levels >= 2 * N - 2                          # Snir
        if N == 8:
            assert levels == fig["steps"] and combines == fig["ops"]


@pytest.mark.parametrize("M,workers", [(8, 2), (12, 3), (64, 8), (511, 7), (100, 10)])
def test_reduce_then_scan_program_counts(M, workers):
    """The alternative strategy: the reduction (M - P), the Brent-Kung scan of the P totals and
    the rescan of every chunk (M - 1 in all: worker 0's first element is already final)."""
    prog, levels, n_elems, n_reg = P.scan_program("reduce_then_scan", M, workers)
    w_gs, s_gs = _bk_work_span(workers)
    assert n_reg == (M - workers) + w_gs + (M - 1) and n_elems == M + workers
    K = -(-M // workers)
    assert levels == (K - 1) + s_gs + K
