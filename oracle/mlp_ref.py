"""Test infrastructure only: FP64 reference of the distance-predictor MLP.

Network 7 -> 64 -> 64 -> 1 with ReLU, output d = base * (1 + softplus(y)),
loss mean(((d - target) / scale)^2). Parameters are one flat vector in the
order W1[7][64], b1[64], W2[64][64], b2[64], W3[64], b3 (as the GPU library).

With ``bf16=True`` the inputs, the weights W1, W2, W3 and the hidden
activations are rounded to BF16 (round to nearest even, via float32) before
they enter a product, as on the GPU; the backward pass treats the rounding as
the identity (straight-through). With ``bf16=False`` the network is plain
FP64, which central finite differences pin.
"""
from __future__ import annotations

import numpy as np

NIN, H = 7, 64
OW1 = 0
OB1 = OW1 + NIN * H
OW2 = OB1 + H
OB2 = OW2 + H * H
OW3 = OB2 + H
OB3 = OW3 + H
NP = OB3 + 1


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round to the nearest BF16 value (ties to even), through float32."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    special = (u & 0x7F800000) == 0x7F800000
    r = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    r = np.where(special, u, r).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    return (p[OW1:OB1].reshape(NIN, H), p[OB1:OW2], p[OW2:OB2].reshape(H, H), p[OB2:OW3], p[OW3:OB3], p[OB3])


def _softplus(y):
    return np.where(y > 20.0, y, np.log1p(np.exp(np.minimum(y, 20.0))))


def _sigmoid(y):
    return 1.0 / (1.0 + np.exp(-y))


def forward(p, X, base, bf16=True):
    W1, b1, W2, b2, W3, b3 = unpack(p)
    rnd = bf16_round if bf16 else (lambda a: np.asarray(a, np.float64))
    x = rnd(X)
    z1 = x @ rnd(W1) + b1
    a1 = rnd(np.maximum(z1, 0.0))
    z2 = a1 @ rnd(W2) + b2
    a2 = rnd(np.maximum(z2, 0.0))
    y = a2 @ rnd(W3) + b3
    d = base * (1.0 + _softplus(y))
    return d, (x, z1, a1, z2, a2, y)


def loss_and_grad(p, X, base, target, scale, bf16=True):
    W1, b1, W2, b2, W3, b3 = unpack(p)
    rnd = bf16_round if bf16 else (lambda a: np.asarray(a, np.float64))
    n = X.shape[0]
    d, (x, z1, a1, z2, a2, y) = forward(p, X, base, bf16)
    r = (d - target) / scale
    loss = float(np.sum(r * r) / n)
    dd = 2.0 * r / scale / n
    dy = dd * base * _sigmoid(y)
    gW3 = a2.T @ dy
    gb3 = dy.sum()
    dz2 = np.where(z2 > 0.0, dy[:, None] * rnd(W3)[None, :], 0.0)
    gW2 = a1.T @ dz2
    gb2 = dz2.sum(axis=0)
    da1 = dz2 @ rnd(W2).T
    dz1 = np.where(z1 > 0.0, da1, 0.0)
    gW1 = x.T @ dz1
    gb1 = dz1.sum(axis=0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3, [gb3]])
    return loss, g


def features(xyz, s, center, radius):
    v = np.asarray(xyz, np.float64)
    sv = v[s]
    ch = np.linalg.norm(v - sv, axis=1)
    X = np.concatenate([(v - center) / radius, np.broadcast_to((sv - center) / radius, v.shape),
                        (ch / radius)[:, None]], axis=1)
    return X.astype(np.float32), ch.astype(np.float32)
