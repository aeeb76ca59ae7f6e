"""Plain numpy oracle of the surrogate MLP (forward, backward, Adam) and of
BF16 round-to-nearest-even.

TEST INFRASTRUCTURE ONLY (used by the tests and nothing in the library).

The network advances one cell by a macro step of four time steps: input
x in R^16 (the 14 normalised state variables, the normalised gap current and
the normalised evoked input), two hidden layers of width 128 with SiLU, and a
linear output in R^16 whose first 14 entries are the normalised state
increments (the last two are padding and carry no loss).

    z1 = W1 x + b1,  h1 = silu(z1)
    z2 = W2 h1 + b2, h2 = silu(z2)
    y  = W3 h2 + b3
    loss = mean over the batch and the 14 outputs of (y - t)^2

In ``bf16`` mode every matrix-product operand is rounded to BF16 (round to
nearest even) exactly where the GPU kernels round it: the weights, the
input, h1, h2 and the back-propagated dy, dz2, dz1; sums are exact (fp64
here, fp32 on the GPU); element-wise work is unrounded.
"""
from __future__ import annotations

import numpy as np

K_IN = 16
HID = 128
K_OUT = 16
N_TARGET = 14

SHAPES = (("W1", (HID, K_IN)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)),
          ("W3", (K_OUT, HID)), ("b3", (K_OUT,)))
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def bf16_round(a) -> np.ndarray:
    """Round float32 values to the nearest BF16 (ties to even), returned as
    float32. Integer definition on the fp32 bit pattern: add 0x7FFF plus the
    lowest kept bit, drop the low 16 bits; NaN stays a (quiet) NaN."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    r = (r & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    nan = np.isnan(f)
    r[nan] = (f.view(np.uint32)[nan] & np.uint32(0xFFFF0000)) | np.uint32(0x00400000)
    return r.view(np.float32).reshape(np.shape(a))


def unpack(flat):
    out, k = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = np.asarray(flat[k:k + n], dtype=np.float64).reshape(shp)
        k += n
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def _sig(z):
    return 1.0 / (1.0 + np.exp(-z))


def silu(z):
    return z * _sig(z)


def silu_grad(z):
    s = _sig(z)
    return s * (1.0 + z * (1.0 - s))


def _q(a, bf16):
    return bf16_round(a).astype(np.float64) if bf16 else np.asarray(a, dtype=np.float64)


def forward(flat, x, bf16=False):
    """x: [B, 16]. Returns y [B, 16] and the cache for backward."""
    p = unpack(flat)
    W1, W2, W3 = (_q(p[k], bf16) for k in ("W1", "W2", "W3"))
    xq = _q(x, bf16)
    z1 = xq @ W1.T + p["b1"]
    h1 = _q(silu(z1), bf16)
    z2 = h1 @ W2.T + p["b2"]
    h2 = _q(silu(z2), bf16)
    y = h2 @ W3.T + p["b3"]
    return y, dict(W1=W1, W2=W2, W3=W3, x=xq, z1=z1, h1=h1, z2=z2, h2=h2)


def loss_and_grad(flat, x, t, bf16=False):
    """Mean-squared error over the batch and the first 14 outputs, and its
    gradient with respect to every parameter (flat, same order as pack)."""
    y, c = forward(flat, x, bf16)
    B = x.shape[0]
    diff = np.zeros_like(y)
    diff[:, :N_TARGET] = y[:, :N_TARGET] - np.asarray(t, np.float64)[:, :N_TARGET]
    loss = float(np.sum(diff ** 2) / (B * N_TARGET))
    dy = _q(2.0 * diff / (B * N_TARGET), bf16)
    g = {}
    g["W3"] = dy.T @ c["h2"]
    g["b3"] = dy.sum(axis=0)
    dz2 = _q((dy @ c["W3"]) * silu_grad(c["z2"]), bf16)
    g["W2"] = dz2.T @ c["h1"]
    g["b2"] = dz2.sum(axis=0)
    dz1 = _q((dz2 @ c["W2"]) * silu_grad(c["z1"]), bf16)
    g["W1"] = dz1.T @ c["x"]
    g["b1"] = dz1.sum(axis=0)
    return loss, pack(g)


def adam_step(w, m, v, g, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba, 2015) with bias correction; t >= 1."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    w = w - lr * mh / (np.sqrt(vh) + eps)
    return w, m, v

