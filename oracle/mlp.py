"""Reference for the small ell/k predictor network (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Not in the paper.  MLP 16 -> 64 -> 64 -> 2 with SiLU activations
(5,378 parameters): y = W3^T s(W2^T s(W1^T x + b1) + b2) + b3, loss
0.5 * mean over the batch of ||y - t||^2 (both outputs).

Numerics of the GPU kernels, emulated here when ``bf16=True``: the weights
and every matrix-product operand (layer inputs, backpropagated errors) are
rounded to bfloat16 (round to nearest, ties to even, from float32); products
accumulate in float32 on the GPU (float64 here); bias, activation and loss
are float32.  Master weights and Adam state are float32.
With ``bf16=False`` everything is float64 (for finite-difference checks).
"""
from __future__ import annotations

import numpy as np

SIZES = (16, 64, 64, 2)


def bf16_round(x):
    """Round float32 values to the nearest bfloat16 (ties to even)."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    bits = a.view(np.uint32).astype(np.uint64)
    bits = bits + 0x7FFF + ((bits >> 16) & 1)
    out = (bits & 0xFFFF0000).astype(np.uint32).view(np.float32)
    return out.reshape(np.shape(x))


def init_params(seed: int = 0):
    rng = np.random.default_rng(seed)
    p = {}
    for i, (a, b) in enumerate(zip(SIZES[:-1], SIZES[1:]), start=1):
        p[f"W{i}"] = (rng.standard_normal((a, b)) * np.sqrt(2.0 / (a + b))).astype(np.float32)
        p[f"b{i}"] = np.zeros(b, dtype=np.float32)
    return p


def n_params() -> int:
    return sum(a * b + b for a, b in zip(SIZES[:-1], SIZES[1:]))


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def _q(x, bf16):
    return bf16_round(x).astype(np.float64) if bf16 else np.asarray(x, dtype=np.float64)


def forward(p, X, bf16: bool = True):
    """Returns (Y, cache).  X: (B, 16)."""
    W = [_q(p[f"W{i}"], bf16) for i in (1, 2, 3)]
    b = [np.asarray(p[f"b{i}"], np.float64) for i in (1, 2, 3)]
    h0 = _q(X, bf16)
    z1 = h0 @ W[0] + b[0]
    h1 = _q(silu(z1), bf16)
    z2 = h1 @ W[1] + b[1]
    h2 = _q(silu(z2), bf16)
    y = h2 @ W[2] + b[2]
    return y, dict(h0=h0, z1=z1, h1=h1, z2=z2, h2=h2, W=W)


def loss_and_grad(p, X, T, bf16: bool = True):
    """0.5 * mean_b ||y_b - t_b||^2 and its gradient for every parameter."""
    B = X.shape[0]
    y, c = forward(p, X, bf16)
    e = y - T
    loss = 0.5 * float(np.sum(e * e)) / B
    g = {}
    d3 = e / B                                   # dL/dy
    g["W3"] = c["h2"].T @ _q(d3, bf16)
    g["b3"] = d3.sum(axis=0)
    dh2 = _q(d3, bf16) @ c["W"][2].T
    d2 = dh2 * dsilu(c["z2"])
    g["W2"] = c["h1"].T @ _q(d2, bf16)
    g["b2"] = d2.sum(axis=0)
    dh1 = _q(d2, bf16) @ c["W"][1].T
    d1 = dh1 * dsilu(c["z1"])
    g["W1"] = c["h0"].T @ _q(d1, bf16)
    g["b1"] = d1.sum(axis=0)
    return loss, g


ADAM_B1, ADAM_B2, ADAM_EPS = 0.9, 0.999, 1e-8


def adam_init(p):
    return {k: (np.zeros_like(v), np.zeros_like(v)) for k, v in p.items()}


def adam_step(p, g, state, lr: float, t: int):
    """One Adam update of the float32 master weights (t counts from 1)."""
    out = {}
    for k in p:
        m, v = state[k]
        gk = np.asarray(g[k], np.float32)
        m = (ADAM_B1 * m + (1 - ADAM_B1) * gk).astype(np.float32)
        v = (ADAM_B2 * v + (1 - ADAM_B2) * gk * gk).astype(np.float32)
        mh = m / (1 - ADAM_B1 ** t)
        vh = v / (1 - ADAM_B2 ** t)
        out[k] = (p[k] - lr * mh / (np.sqrt(vh) + ADAM_EPS)).astype(np.float32)
        state[k] = (m, v)
    return out
