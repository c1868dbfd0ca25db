"""Pins of the FP64 reference network (CPU, no GPU)."""
import numpy as np
import pytest
import torch

from oracle import cnn as C


def _params(seed=0, scale=0.05):
    rng = np.random.default_rng(seed)
    lay, total = C.layout()
    p = np.zeros(total)
    for l, (w, b) in enumerate(lay):
        k = 9 * C.CIN[l]
        m = np.zeros((C.COUT[l], C.kp(l)))
        m[:, :k] = rng.normal(0, scale * np.sqrt(2.0 / k) / 0.05, size=(C.COUT[l], k))
        p[w:w + C.COUT[l] * C.kp(l)] = m.ravel()
        p[b:b + C.COUT[l]] = rng.normal(0, 0.1, size=C.COUT[l])
    return p


def test_layout_counts():
    lay, total = C.layout()
    # 0.92 M weights plus the zero padding of the K dimension
    real = sum(9 * ci * co + co for ci, co in zip(C.CIN, C.COUT))
    assert real == 924582
    assert total == real + sum(C.COUT[l] * (C.kp(l) - 9 * C.CIN[l]) for l in range(6))


def test_weight_layout_is_tap_major_then_channel():
    """A single 1 at (co=0, tap (dy=0, dx=2), ci=1) of a stride-1 layer gives
    out[y, x] = in_channel_1[y - 1, x + 1] (cross-correlation, padding 1)."""
    co, ci, dy, dx = 0, 1, 0, 2
    k = (dy * 3 + dx) * C.CIN[3] + ci
    flat = np.zeros(C.COUT[3] * C.kp(3))
    flat.reshape(C.COUT[3], C.kp(3))[co, k] = 1.0
    W = torch.as_tensor(flat).reshape(C.COUT[3], C.kp(3))[:, :9 * C.CIN[3]]
    W = W.reshape(C.COUT[3], 3, 3, C.CIN[3]).permute(0, 3, 1, 2)
    x = torch.randn(1, C.CIN[3], 8, 8, dtype=torch.float64)
    y = torch.nn.functional.conv2d(x, W, padding=1)[0, 0]
    ref = torch.zeros(8, 8, dtype=torch.float64)
    ref[1:, :7] = x[0, 1, :7, 1:]
    assert torch.equal(y, ref)


def test_upsample_concat_order():
    a = torch.arange(4, dtype=torch.float64).reshape(1, 1, 2, 2)
    u = C.up2(a)
    assert u.shape == (1, 1, 4, 4)
    assert u[0, 0].tolist() == [[0, 0, 1, 1], [0, 0, 1, 1], [2, 2, 3, 3], [2, 2, 3, 3]]


def test_gradient_matches_finite_differences():
    p = _params(1)
    rng = np.random.default_rng(2)
    x = rng.normal(size=(1, 128, 128, 2))
    t = rng.normal(size=(1, 128, 128, 2))
    loss, g = C.loss_and_grad(p, x, t, margin=4)
    lay, _ = C.layout()
    idx = []
    for l, (w, b) in enumerate(lay):
        for j in range(2):
            row = rng.integers(0, C.COUT[l])
            col = rng.integers(0, 9 * C.CIN[l])
            idx.append(w + row * C.kp(l) + col)
        idx.append(b + rng.integers(0, C.COUT[l]))
    h = 1e-6
    for i in idx:
        pp = p.copy()
        pp[i] += h
        pm = p.copy()
        pm[i] -= h
        fd = (C.loss_fn(torch.as_tensor(C.forward(pp, x)), t, 4) -
              C.loss_fn(torch.as_tensor(C.forward(pm, x)), t, 4)) / (2 * h)
        assert abs(float(fd) - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-9, (i, float(fd), g[i])


def test_padding_columns_get_no_gradient():
    p = _params(3)
    rng = np.random.default_rng(4)
    x = rng.normal(size=(1, 128, 128, 2))
    _, g = C.loss_and_grad(p, x, np.zeros_like(x), margin=4)
    lay, _ = C.layout()
    for l, (w, b) in enumerate(lay):
        m = g[w:w + C.COUT[l] * C.kp(l)].reshape(C.COUT[l], C.kp(l))
        assert np.all(m[:, 9 * C.CIN[l]:] == 0)


def test_bf16_rounding():
    v = np.array([1.0, 1.00390625, 1.005859375, -3.140625, 1e-30], dtype=np.float32)
    r = C.bf16_round(v)
    assert r[0] == 1.0 and r[1] == 1.0  # halfway to even
    assert r[2] == np.float32(1.0078125)
    assert r[3] == np.float32(-3.140625)


def test_upsampled_convolution_folds_onto_the_source_grid():
    """The reading the network kernels use for the layers after a 2x nearest upsampling (L4,
    L5, L6): output pixel (2Y + py, 2X + px) of a 3x3 convolution (padding 1) of the upsampled
    map sees only the source pixels (Y - 1 + py + i, X - 1 + px + j), i, j in {0, 1}, with the
    taps landing on one source pixel summed (tap rows {0}, {1, 2} for py = 0 and {0, 1}, {2}
    for py = 1; columns alike). Checked in FP64 against upsample-then-convolve with torch."""
    rng = np.random.default_rng(7)
    B, C_in, C_out, S = 2, 5, 3, 6
    src = torch.tensor(rng.standard_normal((B, C_in, S, S)), dtype=torch.float64)
    w = torch.tensor(rng.standard_normal((C_out, C_in, 3, 3)), dtype=torch.float64)
    ref = torch.nn.functional.conv2d(torch.nn.functional.interpolate(src, scale_factor=2,
                                                                     mode="nearest"),
                                     w, padding=1)
    groups = {0: ([0], [1, 2]), 1: ([0, 1], [2])}   # tap rows (columns) per offset i (j)
    out = torch.zeros_like(ref)
    pad = torch.nn.functional.pad(src, (1, 1, 1, 1))   # source offsets -1 .. +1
    for py in (0, 1):
        for px in (0, 1):
            wf = torch.zeros((C_out, C_in, 2, 2), dtype=torch.float64)
            for i in (0, 1):
                for j in (0, 1):
                    for ty in groups[py][i]:
                        for tx in groups[px][j]:
                            wf[:, :, i, j] += w[:, :, ty, tx]
            # source pixel (Y - 1 + py + i) sits at row Y + py + i of the padded map
            part = torch.nn.functional.conv2d(pad[:, :, py:py + S + 1, px:px + S + 1], wf)
            out[:, :, py::2, px::2] = part
    # everywhere, the border rows and columns included: the taps that leave the upsampled map
    # (its zero padding) are exactly the source pixels outside the source map
    assert (out - ref).abs().max().item() < 1e-12
