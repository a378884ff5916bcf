"""CPU reference of the warm-start network — TEST INFRASTRUCTURE ONLY.

Forward and backward pass of x -> relu(x W1 + b1) -> relu(h1 W2 + b2) ->
sigmoid(h2 . w3 + b3) with the mean squared error, in float64.  With
``bf16=True`` the operands that the GPU feeds to its BF16 matrix products
(inputs, W1, W2, hidden activations, hidden gradients) are rounded to
bfloat16 at the same points, so the comparison isolates the kernels.  The
backward formulas are pinned by central finite differences of the float64
loss (tests/test_mlp_cpu.py).
"""
from __future__ import annotations

import numpy as np

IN, HID = 32, 256
OFF_W1 = 0
OFF_B1 = OFF_W1 + IN * HID
OFF_W2 = OFF_B1 + HID
OFF_B2 = OFF_W2 + HID * HID
OFF_W3 = OFF_B2 + HID
OFF_B3 = OFF_W3 + HID
NPARAM = OFF_B3 + 1


def bf16(a):
    """Round-to-nearest-even to bfloat16, returned as float64."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    return (p[OFF_W1:OFF_B1].reshape(IN, HID), p[OFF_B1:OFF_W2], p[OFF_W2:OFF_B2].reshape(HID, HID),
            p[OFF_B2:OFF_W3], p[OFF_W3:OFF_B3], p[OFF_B3])


def forward(p, X, bf=True):
    W1, b1, W2, b2, w3, b3 = unpack(p)
    r = bf16 if bf else (lambda a: np.asarray(a, dtype=np.float64))
    Xb = r(X)
    z1 = Xb @ r(W1) + b1
    h1 = r(np.maximum(z1, 0.0))
    z2 = h1 @ r(W2) + b2
    h2 = r(np.maximum(z2, 0.0))
    z = h2 @ w3 + b3
    y = 1.0 / (1.0 + np.exp(-z))
    return y, (Xb, z1, h1, z2, h2)


def loss_and_grad(p, X, t, bf=True):
    W1, b1, W2, b2, w3, b3 = unpack(p)
    r = bf16 if bf else (lambda a: np.asarray(a, dtype=np.float64))
    y, (Xb, z1, h1, z2, h2) = forward(p, X, bf)
    t = np.asarray(t, dtype=np.float64)
    R = len(t)
    d = y - t
    loss = float(np.mean(d * d))
    dz = 2.0 * d / R * y * (1.0 - y)
    g = np.zeros(NPARAM)
    g[OFF_W3:OFF_B3] = h2.T @ dz
    g[OFF_B3] = dz.sum()
    dh2 = np.outer(dz, w3) * (z2 > 0)
    g[OFF_W2:OFF_B2] = (h1.T @ r(dh2)).ravel()
    g[OFF_B2:OFF_W3] = dh2.sum(axis=0)
    dh1 = (r(dh2) @ r(W2).T) * (z1 > 0)
    g[OFF_W1:OFF_B1] = (Xb.T @ r(dh1)).ravel()
    g[OFF_B1:OFF_W2] = dh1.sum(axis=0)
    return loss, g
