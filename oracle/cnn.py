"""FP64 CPU reference of the warm-start network (test infrastructure only).

Plain torch CPU operations in float64: conv2d, ReLU, nearest upsampling, concatenation, mean
squared error and autograd. The flat parameter vector follows the layout of the library's
network: for each layer, weights [Cout][Kp] with k = (dy * 3 + dx) * Cin + ci (columns beyond
9 Cin are zero padding), then the bias [Cout]. Inputs and outputs are [B, 128, 128, 2].

Architecture (3x3, padding 1, ReLU except the last layer):
  L1 2->64 s2, L2 64->128 s2, L3 128->256 s2, L4 [up2(L3), L2] 384->128,
  L5 [up2(L4), L1] 192->64, L6 [up2(L5), input] 66->2 (linear).
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as F

CIN = [2, 64, 128, 384, 192, 66]
COUT = [64, 128, 256, 128, 64, 2]
STRIDE = [2, 2, 2, 1, 1, 1]


def kp(layer: int) -> int:
    k = 9 * CIN[layer]
    if layer == 0:
        return 64
    if layer == 5:
        return k
    return (k + 31) // 32 * 32


def layout():
    """[(w_offset, b_offset)] per layer and the total parameter count."""
    off = 0
    out = []
    for l in range(6):
        w = off
        off += COUT[l] * kp(l)
        b = off
        off += COUT[l]
        out.append((w, b))
    return out, off


def unpack(params) -> list:
    """Flat vector -> [(weight [Cout, Cin, 3, 3], bias [Cout])] as float64 tensors."""
    lay, total = layout()
    p = torch.as_tensor(np.asarray(params, dtype=np.float64))
    assert p.numel() == total
    layers = []
    for l, (w, b) in enumerate(lay):
        k = 9 * CIN[l]
        W = p[w:w + COUT[l] * kp(l)].reshape(COUT[l], kp(l))[:, :k]
        W = W.reshape(COUT[l], 3, 3, CIN[l]).permute(0, 3, 1, 2).contiguous()
        layers.append((W, p[b:b + COUT[l]].clone()))
    return layers


def pack(grads) -> np.ndarray:
    """[(dW [Cout, Cin, 3, 3], db)] -> flat vector in the library layout (zeros in padding)."""
    lay, total = layout()
    out = np.zeros(total)
    for l, ((w, b), (dW, db)) in enumerate(zip(lay, grads)):
        k = 9 * CIN[l]
        m = np.zeros((COUT[l], kp(l)))
        m[:, :k] = dW.detach().permute(0, 2, 3, 1).reshape(COUT[l], k).numpy()
        out[w:w + COUT[l] * kp(l)] = m.ravel()
        out[b:b + COUT[l]] = db.detach().numpy()
    return out


def up2(x):
    return x.repeat_interleave(2, dim=2).repeat_interleave(2, dim=3)


def forward_layers(layers, x_nhwc):
    """Forward pass in float64; x [B, 128, 128, 2] -> y [B, 128, 128, 2]."""
    x = torch.as_tensor(np.asarray(x_nhwc, dtype=np.float64)).permute(0, 3, 1, 2)
    (W1, b1), (W2, b2), (W3, b3), (W4, b4), (W5, b5), (W6, b6) = layers
    a1 = F.relu(F.conv2d(x, W1, b1, stride=2, padding=1))
    a2 = F.relu(F.conv2d(a1, W2, b2, stride=2, padding=1))
    a3 = F.relu(F.conv2d(a2, W3, b3, stride=2, padding=1))
    a4 = F.relu(F.conv2d(torch.cat([up2(a3), a2], 1), W4, b4, padding=1))
    a5 = F.relu(F.conv2d(torch.cat([up2(a4), a1], 1), W5, b5, padding=1))
    y = F.conv2d(torch.cat([up2(a5), x], 1), W6, b6, padding=1)
    return y.permute(0, 2, 3, 1)


def forward(params, x_nhwc) -> np.ndarray:
    with torch.no_grad():
        return forward_layers(unpack(params), x_nhwc).numpy()


def loss_fn(y, target, margin: int):
    t = torch.as_tensor(np.asarray(target, dtype=np.float64))
    d = (y - t)[:, margin:128 - margin, margin:128 - margin, :]
    return (d * d).mean()


def loss_and_grad(params, x_nhwc, target, margin: int = 4):
    """Mean squared error over the interior and its gradient (flat, library layout)."""
    layers = unpack(params)
    for W, b in layers:
        W.requires_grad_(True)
        b.requires_grad_(True)
    loss = loss_fn(forward_layers(layers, x_nhwc), target, margin)
    loss.backward()
    return float(loss.detach()), pack([(W.grad, b.grad) for W, b in layers])


def bf16_round(a) -> np.ndarray:
    """Round float32 values to bfloat16 (round to nearest even), returned as float32."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)
