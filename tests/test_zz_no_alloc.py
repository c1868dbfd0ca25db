"""The allocation-free entry point (pprs_register_pair_noalloc) against pprs_register_pair:
the same registrations bit for bit, two calls in a row with the second on smaller frames (the
scratch keeps the first call's contents), frames beyond the scratch refused on the host, and a
context that only makes allocation-free calls holds no workspace."""
import numpy as np
import pytest

from synth import SeriesSpec, make_series

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def say(*a):
    print("[noalloc]", *a, flush=True)


def _pair(spec, i=0, k=1):
    torch = _torch()
    s = make_series(spec)
    fr = torch.tensor(s.frames, device="cuda")
    return fr[i].contiguous(), fr[k].contiguous()


def test_noalloc_matches_register_pair_twice_then_smaller():
    torch = _torch()
    import paper_1712_02533_amd as P
    cases = [(SeriesSpec(2, 512, 8.0, 1.5, 5.0, 2), 4, False),
             (SeriesSpec(2, 128, 4.0, 1.0, 10.0, 1), 3, True)]
    stream = torch.cuda.Stream()    # a fresh context that only makes allocation-free calls
    for spec, levels, with_init in cases:
        f0, f1 = _pair(spec)
        side = spec.side
        params = P.Params(levels=levels)
        u_init = None
        if with_init:
            u_init = torch.full((2, side, side), 0.75, device="cuda")
        say("pair %dx%d, %d levels, initial guess %s" % (side, side, levels, with_init))
        ref, st_ref = P.register_pair(f0, f1, u_init=u_init, params=params)
        with torch.cuda.stream(stream):
            out = torch.full((2, side, side), float("nan"), device="cuda")
            got, st = P.register_pair_noalloc(f0, f1, out, u_init=u_init, params=params)
            held = P.workspace_bytes()
        stream.synchronize()
        say("  iters %s / %s, max |diff| %.3e px, context workspace %d bytes"
            % (st.iters, st_ref.iters, (got - ref).abs().max().item(), held))
        assert torch.equal(got, ref)
        assert st.iters == st_ref.iters and st.passes == st_ref.passes
        assert st.energy == st_ref.energy and st.flags == st_ref.flags
        assert held == 0


def test_noalloc_refuses_frames_beyond_its_scratch():
    torch = _torch()
    import paper_1712_02533_amd as P
    from paper_1712_02533_amd.api import PprsError
    f = torch.rand((1024, 1024), device="cuda")
    out = torch.empty((2, 1024, 1024), device="cuda")
    with pytest.raises(PprsError, match="scratch"):
        P.register_pair_noalloc(f, f, out, params=P.Params(levels=4))
