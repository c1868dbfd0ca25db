"""GPU parity of the warm-start network and its data plumbing against the FP64 CPU reference.

The network computes in BF16 (weights and activations) with FP32 accumulation; the reference
runs the same layers in FP64 with the BF16-rounded weights and input, so the remaining
difference is the rounding of the activations between layers (a few 2^-9 relative per layer).
"""
import numpy as np
import pytest

from oracle import cnn as C
import oracle as O
from synth import SeriesSpec, make_series

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def say(*a):
    print("[cnn]", *a, flush=True)


def _net_with_biases(seed):
    import paper_1712_02533_amd as P
    net = P.WarmStartNet(seed=seed)
    p = net.get_params()
    lay, total = C.layout()
    assert p.size == total
    rng = np.random.default_rng(seed)
    for l, (w, b) in enumerate(lay):
        p[b:b + C.COUT[l]] = rng.normal(0, 0.05, C.COUT[l]).astype(np.float32)
    # make the linear last layer as large as the others so its output is not tiny
    w6, b6 = lay[5]
    p[w6:b6] *= 10.0
    net.set_params(p)
    return net, p


def _bf16_params(p):
    lay, _ = C.layout()
    q = p.astype(np.float64).copy()
    for l, (w, b) in enumerate(lay):
        q[w:b] = C.bf16_round(p[w:b])
    return q


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def test_weights_blob_loaded_by_the_library():
    """pprs_cnn_load parses the shipped weights file itself (safetensors layout, one F32
    tensor): the parameters equal what a library reader of the same file returns, and
    malformed blobs are refused without touching the weights."""
    _torch()
    import os
    import struct
    import paper_1712_02533_amd as P
    from paper_1712_02533_amd.api import PprsError
    from safetensors.numpy import load_file
    path = os.path.join(os.path.dirname(P.__file__), "weights", "warmstart_512.safetensors")
    net = P.WarmStartNet(seed=1)
    before = net.get_params()
    net.load(path)
    want = load_file(path)["params"]
    got = net.get_params()
    say("loaded %d parameters from %s" % (got.size, os.path.basename(path)))
    assert np.array_equal(got, want)
    blob = open(path, "rb").read()
    hl = struct.unpack("<Q", blob[:8])[0]
    n = got.size
    hdr = lambda j: struct.pack("<Q", len(j)) + j
    data = np.arange(n, dtype=np.float32).tobytes()
    good = hdr(b'{"params":{"dtype":"F32","shape":[%d],"data_offsets":[0,%d]}}' % (n, 4 * n))
    net.load_bytes(good + data)
    assert np.array_equal(net.get_params(), np.arange(n, dtype=np.float32))
    bad = [blob[:7], blob[:8 + hl - 1], blob[:-4],
           struct.pack("<Q", 1 << 40) + blob[8:],
           hdr(b'{"params":{"dtype":"F16","shape":[%d],"data_offsets":[0,%d]}}' % (n, 4 * n))
           + data,
           hdr(b'{"params":{"dtype":"F32","shape":[%d],"data_offsets":[4,%d]}}' % (n, 4 * n + 4))
           + data,
           hdr(b'{"params":{"dtype":"F32","shape":[%d],"data_offsets":[0,%d]}' % (n, 4 * n))
           + data,
           hdr(b'{"other":{"dtype":"F32","shape":[1],"data_offsets":[0,4]},'
               b'"x":{"dtype":"F32","shape":[1],"data_offsets":[0,4]}}') + data[:4]]
    for blob_bad in bad:
        with pytest.raises(PprsError):
            net.load_bytes(blob_bad)
    assert np.array_equal(net.get_params(), np.arange(n, dtype=np.float32))
    assert not np.array_equal(before, want)


def test_params_roundtrip_and_layout():
    _torch()
    net, p = _net_with_biases(3)
    assert net.n_params == C.layout()[1]
    assert np.array_equal(net.get_params(), p)
    # padding columns of the K dimension stay zero after initialisation
    import paper_1712_02533_amd as P
    q = P.WarmStartNet(seed=5).get_params()
    lay, _ = C.layout()
    for l, (w, b) in enumerate(lay):
        m = q[w:b].reshape(C.COUT[l], C.kp(l))
        assert np.all(m[:, 9 * C.CIN[l]:] == 0)
        sd = m[:, :9 * C.CIN[l]].std()
        want = np.sqrt(2.0 / (9 * C.CIN[l])) * (0.1 if l == 5 else 1.0)
        assert 0.8 * want < sd < 1.2 * want, (l, sd, want)


@pytest.mark.parametrize("B", [1, 3])
def test_forward_matches_fp64_reference(B):
    torch = _torch()
    net, p = _net_with_biases(11)
    rng = np.random.default_rng(100 + B)
    x = C.bf16_round(rng.normal(size=(B, 128, 128, 2)).astype(np.float32))
    say("forward B=%d" % B)
    y = net.forward(torch.tensor(x, device="cuda")).cpu().numpy()
    ref = C.forward(_bf16_params(p), x)
    err = _rel(y, ref)
    say("rel L2 %.3e, max %.3e (scale %.3e)" % (err, np.abs(y - ref).max(), np.abs(ref).max()))
    assert np.all(np.isfinite(y))
    assert err < 2e-2
    assert np.abs(y - ref).max() < 0.05 * np.abs(ref).max()
    # samples are independent: the first sample does not depend on the batch size
    if B > 1:
        y1 = net.forward(torch.tensor(x[:1], device="cuda")).cpu().numpy()
        assert np.array_equal(y1[0], y[0])


def test_gradients_match_fp64_reference():
    torch = _torch()
    net, p = _net_with_biases(12)
    rng = np.random.default_rng(7)
    B = 2
    x = C.bf16_round(rng.normal(size=(B, 128, 128, 2)).astype(np.float32))
    t = rng.normal(0, 1.0, size=(B, 128, 128, 2)).astype(np.float32)
    say("gradients B=%d" % B)
    loss, g = net.gradients(torch.tensor(x, device="cuda"), torch.tensor(t, device="cuda"),
                            margin=4)
    rloss, rg = C.loss_and_grad(_bf16_params(p), x, t, margin=4)
    say("loss %.6e vs %.6e" % (loss, rloss))
    assert abs(loss - rloss) < 1e-2 * rloss
    lay, _ = C.layout()
    for l, (w, b) in enumerate(lay):
        k = 9 * C.CIN[l]
        gw = g[w:b].reshape(C.COUT[l], C.kp(l))
        rw = rg[w:b].reshape(C.COUT[l], C.kp(l))
        assert np.all(gw[:, k:] == 0)
        ew, eb = _rel(gw, rw), _rel(g[b:b + C.COUT[l]], rg[b:b + C.COUT[l]])
        cos = float(np.dot(gw.ravel(), rw.ravel()) /
                    (np.linalg.norm(gw) * np.linalg.norm(rw) + 1e-30))
        say("layer %d: weight rel %.3e cos %.6f, bias rel %.3e" % (l + 1, ew, cos, eb))
        assert ew < 5e-2 and eb < 5e-2 and cos > 0.998


def test_train_steps_reduce_loss():
    torch = _torch()
    import paper_1712_02533_amd as P
    net = P.WarmStartNet(seed=21)
    rng = np.random.default_rng(8)
    B = 4
    x = rng.normal(size=(B, 128, 128, 2)).astype(np.float32)
    # a learnable target: a smooth function of the input
    t = np.stack([0.5 + 0.3 * np.tanh(x[..., 0]), -0.25 + 0.2 * x[..., 1]], -1).astype(np.float32)
    xd, td = torch.tensor(x, device="cuda"), torch.tensor(t, device="cuda")
    losses = [net.train_step(xd, td, lr=1e-3) for _ in range(30)]
    say("losses", ["%.4f" % v for v in losses[::5]], "%.4f" % losses[-1])
    assert all(np.isfinite(losses))
    assert losses[-1] < 0.3 * losses[0]
    # the gradient entry point reports the loss of the current weights
    l2, _ = net.gradients(xd, td)
    assert l2 < losses[0]


def test_pair_inputs_match_reference():
    torch = _torch()
    import paper_1712_02533_amd as P
    spec = SeriesSpec(n_frames=3, side=256, drift=4.0, warp_amp=1.0, mean_counts=10.0, seed=41)
    s = make_series(spec)
    frames = torch.tensor(s.frames, device="cuda")
    ref, tmpl = [0, 1, 2, 0], [1, 2, 0, 0]
    say("pair_inputs 256")
    got = P.pair_inputs(frames, ref, tmpl).cpu().numpy()
    lv = []
    for k in range(3):
        f = O.frame_to_nodes(s.frames[k])
        f = O.restrict(f)
        fn, _, _ = O.normalize(f)
        lv.append(fn[:128, :128])
    want = np.stack([np.stack([lv[r], lv[t]], -1) for r, t in zip(ref, tmpl)])
    err = np.abs(got - want).max()
    say("max abs %.3e" % err)
    assert err < 1e-4


def test_level7_targets_match_reference():
    torch = _torch()
    import paper_1712_02533_amd as P
    rng = np.random.default_rng(9)
    side = 512
    y, x = np.mgrid[0:side, 0:side] / side
    u = np.stack([np.stack([3 * np.sin(2 * np.pi * (x + 0.3 * y) + k) + k,
                            2 * np.cos(2 * np.pi * (0.5 * x - y) + k) - k]) for k in range(2)])
    u += rng.normal(0, 0.05, size=u.shape)
    say("level7_targets 512")
    got = P.level7_targets(torch.tensor(u, dtype=torch.float32, device="cuda")).cpu().numpy()
    want = np.zeros((2, 128, 128, 2))
    for p in range(2):
        for c in range(2):
            f = O.frame_to_nodes(u[p, c]) / side
            f = O.restrict(O.restrict(f))
            want[p, :, :, c] = 128 * f[:128, :128]
    err = np.abs(got - want).max()
    say("max abs %.3e cells" % err)
    assert err < 1e-4


def test_bad_arguments_raise():
    torch = _torch()
    import paper_1712_02533_amd as P
    net = P.WarmStartNet(seed=1)
    with pytest.raises(P.PprsError):
        net.set_params(np.zeros(10, dtype=np.float32))
    with pytest.raises(P.PprsError):
        P.pair_inputs(torch.zeros((2, 64, 64), device="cuda"), [0], [1])
    with pytest.raises(P.PprsError):
        P.pair_inputs(torch.zeros((2, 128, 128), device="cuda"), [0], [2])
    with pytest.raises(P.PprsError):
        P.set_warm_start(net, max_cells=0.0)
