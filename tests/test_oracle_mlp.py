"""Pins of the FP64 reference of the learned alpha starter (CPU only)."""
import numpy as np
import pytest

import oracle
from oracle import mlp


def _data(seed, M=40):
    rng = np.random.default_rng(seed)
    Z = rng.uniform(-1, 1, (M, mlp.N_IN))
    T = rng.normal(size=M)
    w = mlp.init_weights(seed, scale_out=0.5)
    w[mlp.OFF_B1:mlp.OFF_W2] = rng.normal(scale=0.3, size=32)
    w[mlp.OFF_B2:mlp.OFF_W3] = rng.normal(scale=0.3, size=32)
    w[mlp.OFF_B3] = 0.2
    return w, Z, T


def test_gradient_matches_central_differences():
    """Every one of the 1761 partial derivatives against a central difference of L."""
    w, Z, T = _data(1)
    L, g = mlp.loss_and_grad(w, Z, T)
    assert L == pytest.approx(mlp.loss(w, Z, T), rel=1e-14)
    h = 1e-5
    fd = np.empty(mlp.NPARAM)
    for j in range(mlp.NPARAM):
        wp, wm = w.copy(), w.copy()
        wp[j] += h
        wm[j] -= h
        fd[j] = (mlp.loss(wp, Z, T) - mlp.loss(wm, Z, T)) / (2 * h)
    err = np.abs(fd - g)
    assert np.max(err) <= 1e-8 * max(1.0, np.max(np.abs(g))), np.argmax(err)
    # every block of the parameter vector carries a non-zero gradient
    for a, b in [(0, 640), (640, 672), (672, 1696), (1696, 1728), (1728, 1760), (1760, 1761)]:
        assert np.max(np.abs(g[a:b])) > 1e-6


def test_silu_and_its_derivative():
    a = np.linspace(-8, 8, 101)
    assert np.allclose(mlp.silu(a), a * 0.5 * (1 + np.tanh(a / 2)), rtol=1e-14, atol=1e-15)
    h = 1e-6
    assert np.allclose(mlp.silu_grad(a), (mlp.silu(a + h) - mlp.silu(a - h)) / (2 * h), atol=1e-9)
    assert mlp.silu(0.0) == 0.0 and mlp.silu_grad(0.0) == 0.5


def test_forward_closed_forms():
    """Zero hidden matrices: y = w3 . silu(b2) + b3 for every input; zero input
    gives the same through the first layer's bias alone."""
    w, Z, _ = _data(2)
    W1, b1, W2, b2, w3, b3 = mlp.unpack(w)
    w0 = mlp.pack(W1, b1, np.zeros((32, 32)), b2, w3, b3)
    y = mlp.forward(w0, Z)
    assert np.allclose(y, float(w3 @ mlp.silu(b2) + b3), rtol=1e-14)
    y0 = mlp.forward(w, np.zeros((3, mlp.N_IN)))
    expect = w3 @ mlp.silu(W2 @ mlp.silu(b1) + b2) + b3
    assert np.allclose(y0, expect, rtol=1e-14)
    # one unit, one input: scalar composition written out by hand
    W1 = np.zeros((32, 20)); W1[3, 7] = 1.5
    W2 = np.zeros((32, 32)); W2[5, 3] = -2.0
    w3 = np.zeros(32); w3[5] = 0.75
    ws = mlp.pack(W1, np.zeros(32), W2, np.zeros(32), w3, 0.1)
    z = np.zeros((1, 20)); z[0, 7] = 0.4
    s1 = 0.6 / (1 + np.exp(-0.6))
    s2 = -2.0 * s1 / (1 + np.exp(2.0 * s1))
    assert mlp.forward(ws, z)[0] == pytest.approx(0.75 * s2 + 0.1, rel=1e-15)


def test_round_bf16_against_definition():
    """bfloat16 is the top half of an FP32 word; round to nearest, ties to even."""
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, 1.0 + 2 ** -9, 1.0 + 2 ** -7 + 2 ** -9, -3.0e-5, 0.0],
                 dtype=np.float32)
    r = mlp.round_bf16(x)
    assert r[0] == 1.0
    assert r[1] == 1.0            # exactly half an ulp (2^-8) above 1: tie, even is 1.0
    assert r[2] == 1.0 + 2 ** -7  # 0.75 ulp rounds up
    assert r[3] == 1.0            # 0.25 ulp rounds down
    assert r[4] == 1.0 + 2 ** -7  # 1.25 ulp rounds to 1 ulp
    assert r[6] == 0.0
    assert abs(r[5] + 3.0e-5) <= 3.0e-5 * 2 ** -8
    rng = np.random.default_rng(0)
    v = rng.normal(size=10000).astype(np.float32)
    rv = mlp.round_bf16(v)
    assert np.all(np.abs(rv - v) <= np.abs(v) * 2 ** -8 * (1 + 1e-7))
    assert np.all((rv.astype(np.float32).view(np.uint32) & 0xFFFF) == 0)


def test_starter_features_properties():
    c, wts = oracle.lattice()
    rng = np.random.default_rng(3)
    u = np.array([0.02, -0.01, 0.03])
    fe = oracle.feq(1.3, u)
    f = fe * (1 + 1e-3 * rng.uniform(-1, 1, 19))
    z, s, ok = mlp.starter_features(f, fe)
    assert ok and np.max(np.abs(z)) == pytest.approx(1.0, abs=1e-15)
    assert np.allclose(z * s, f / fe - 1, rtol=1e-13)
    # invariant under a common scale of f and f_eq
    z2, s2, ok2 = mlp.starter_features(7 * f, 7 * fe)
    assert ok2 and np.allclose(z2, z, atol=1e-13) and s2 == pytest.approx(s, rel=1e-13)
    # equilibrium (s = 0), a non-positive population and s > 1 are rejected
    assert not mlp.starter_features(fe, fe)[2]
    fbad = f.copy(); fbad[4] = -1e-6
    assert not mlp.starter_features(fbad, fe)[2]
    assert not mlp.starter_features(f * np.r_[3.5, np.ones(18)], fe)[2]
