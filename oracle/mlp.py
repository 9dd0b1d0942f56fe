"""FP64 numpy reference of the learned alpha starter (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use it.
The network and its loss are plain definitions, written out here in FP64:

  a1 = W1 z + b1,  h1 = silu(a1),  a2 = W2 h1 + b2,  h2 = silu(a2),
  y  = w3 . h2 + b3,               L = (1 / 2M) sum_i (y_i - t_i)^2,

with silu(a) = a / (1 + exp(-a)), and the hand-derived gradient of L by the
chain rule.  The gradient is pinned by central finite differences of L, not
by itself.  Parameter vector (1761 values): W1 [32][20], b1 [32], W2 [32][32],
b2 [32], w3 [32], b3.

The starter's input for one node and component (Eq. entropic alpha is what
it approximates): the 19 ratios r_p = f_p / f_eq_p as z_p = (r_p - 1)/s and
s = max_p |r_p - 1| (20 values); target (alpha* - 2)/s, alpha* the root of
the H balance.

``bf16=True`` rounds to bfloat16 (round to nearest even) where a matrix-core
implementation stores its operands: the input z, W1, W2 and h1.  Everything
else stays FP64.
"""
from __future__ import annotations

import numpy as np

N_IN, N_H = 20, 32
OFF_W1, OFF_B1, OFF_W2, OFF_B2, OFF_W3, OFF_B3, NPARAM = 0, 640, 672, 1696, 1728, 1760, 1761


def unpack(w):
    w = np.asarray(w, dtype=np.float64)
    assert w.shape == (NPARAM,)
    return (w[OFF_W1:OFF_B1].reshape(N_H, N_IN), w[OFF_B1:OFF_W2], w[OFF_W2:OFF_B2].reshape(N_H, N_H),
            w[OFF_B2:OFF_W3], w[OFF_W3:OFF_B3], w[OFF_B3])


def pack(W1, b1, W2, b2, w3, b3):
    return np.concatenate([np.ravel(W1), b1, np.ravel(W2), b2, w3, [b3]]).astype(np.float64)


def round_bf16(x):
    """Nearest bfloat16 (ties to even) of each FP32 value of x, returned in FP64."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def silu(a):
    return a / (1.0 + np.exp(-a))


def silu_grad(a):
    s = 1.0 / (1.0 + np.exp(-a))
    return s * (1.0 + a * (1.0 - s))


def forward(w, Z, bf16: bool = False, keep: bool = False):
    """Outputs y [M] for inputs Z [M][20]."""
    W1, b1, W2, b2, w3, b3 = unpack(w)
    Z = np.asarray(Z, dtype=np.float64)
    if bf16:
        Z, W1, W2 = round_bf16(Z), round_bf16(W1), round_bf16(W2)
    a1 = Z @ W1.T + b1
    h1 = silu(a1)
    if bf16:
        h1 = round_bf16(h1)
    a2 = h1 @ W2.T + b2
    h2 = silu(a2)
    y = h2 @ w3 + b3
    if keep:
        return y, (Z, a1, h1, a2, h2)
    return y


def loss_and_grad(w, Z, T):
    """L = (1/2M) sum (y - T)^2 and dL/dw (FP64, parameter order)."""
    W1, b1, W2, b2, w3, b3 = unpack(w)
    T = np.asarray(T, dtype=np.float64)
    M = T.shape[0]
    y, (Z, a1, h1, a2, h2) = forward(w, Z, keep=True)
    e = y - T
    L = 0.5 * float(e @ e) / M
    dy = e / M
    dw3 = h2.T @ dy
    db3 = dy.sum()
    da2 = np.outer(dy, w3) * silu_grad(a2)
    dW2 = da2.T @ h1
    db2 = da2.sum(axis=0)
    da1 = (da2 @ W2) * silu_grad(a1)
    dW1 = da1.T @ Z
    db1 = da1.sum(axis=0)
    return L, pack(dW1, db1, dW2, db2, dw3, db3)


def loss(w, Z, T):
    e = forward(w, Z) - np.asarray(T, dtype=np.float64)
    return 0.5 * float(e @ e) / e.shape[0]


def init_weights(seed: int, scale_out: float = 0.1):
    """Seeded Glorot-uniform matrices, zero biases (the starting point of training)."""
    rng = np.random.default_rng(seed)
    lim1 = np.sqrt(6.0 / (N_IN + N_H))
    lim2 = np.sqrt(6.0 / (2 * N_H))
    W1 = rng.uniform(-lim1, lim1, (N_H, N_IN))
    W2 = rng.uniform(-lim2, lim2, (N_H, N_H))
    w3 = rng.uniform(-scale_out, scale_out, N_H)
    return pack(W1, np.zeros(N_H), W2, np.zeros(N_H), w3, 0.0)


def starter_features(f, fe):
    """Scaled ratios of one node-component: (z [19], s, valid)."""
    f = np.asarray(f, dtype=np.float64)
    fe = np.asarray(fe, dtype=np.float64)
    if np.any(fe <= 0.0) or np.any(f <= 0.0):
        return np.zeros(19), 0.0, False
    r = f / fe - 1.0
    s = float(np.max(np.abs(r)))
    if not (0.0 < s <= 1.0):
        return np.zeros(19), s, False
    return r / s, s, True


def starter_input(f, fe):
    """The network input [20] = (z, s) of one node-component, and validity."""
    z, s, ok = starter_features(f, fe)
    return np.concatenate([z, [s if ok else 0.0]]), ok
