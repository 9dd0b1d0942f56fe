"""Node-level pins of the CPU oracle: lattice tables, equilibrium, alpha,
matrix norm, Carreau law and shear-rate root, each checked against closed
forms, library routines or 50-digit brute force, never against itself."""
import math
from decimal import Decimal, getcontext

import numpy as np
import pytest
from scipy.optimize import brentq

CS2 = 1.0 / 3.0


def test_lattice_isotropy(ora):
    # D3Q19 (the paper's D2Q9 lifted to 3-D, Sec. II): weights sum to one,
    # odd moments vanish, second moment c_s^2 I, fourth moment c_s^4 (dd+dd+dd).
    c, w = ora.lattice()
    assert c.shape == (19, 3)
    assert math.isclose(w.sum(), 1.0, rel_tol=0, abs_tol=1e-15)
    d = np.eye(3)
    for a in range(3):
        assert abs(np.sum(w * c[:, a])) < 1e-16
        for b in range(3):
            assert abs(np.sum(w * c[:, a] * c[:, b]) - CS2 * d[a, b]) < 1e-15
            for g in range(3):
                assert abs(np.sum(w * c[:, a] * c[:, b] * c[:, g])) < 1e-16
                for e in range(3):
                    ref = CS2 ** 2 * (d[a, b] * d[g, e] + d[a, g] * d[b, e] + d[a, e] * d[b, g])
                    assert abs(np.sum(w * c[:, a] * c[:, b] * c[:, g] * c[:, e]) - ref) < 1e-15
    # rest, 6 faces (w 1/18), 12 edges (w 1/36); opposite pairs at (odd, even)
    n2 = np.sum(c * c, axis=1)
    assert list(n2) == [0] + [1] * 6 + [2] * 12
    assert np.allclose(w[n2 == 1], 1 / 18) and np.allclose(w[n2 == 2], 1 / 36)
    for p in range(1, 19, 2):
        assert np.all(c[p] == -c[p + 1])


@pytest.mark.parametrize("seed", range(5))
def test_feq_moments(ora, seed):
    # Second-order equilibrium: sum f = rho, sum c f = rho u, sum cc f = rho c_s^2 I + rho u u.
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.01, 2.0)
    u = rng.uniform(-0.1, 0.1, 3)
    c, w = ora.lattice()
    fe = ora.feq(rho, u)
    assert math.isclose(fe.sum(), rho, rel_tol=1e-15)
    assert np.allclose(c.T @ fe, rho * u, rtol=0, atol=1e-16)
    P = np.einsum("pa,pb,p->ab", c, c, fe)
    assert np.allclose(P, rho * CS2 * np.eye(3) + rho * np.outer(u, u), rtol=0, atol=1e-15)


def _H_dec(f, w):
    return sum(fi * (fi / wi).ln() for fi, wi in zip(f, w))


def _alpha_decimal(f, fe, w, lo, hi, iters=200):
    """Root of H(f + a (fe - f)) - H(f) by bisection in 60-digit decimal,
    with H evaluated literally as sum f ln(f / w)."""
    getcontext().prec = 60
    F = [Decimal(float(x)) for x in f]
    E = [Decimal(float(x)) for x in fe]
    # the lattice weights as exact decimals (given as Decimals, else D3Q19)
    if isinstance(w, (list, tuple)) and isinstance(w[0], Decimal):
        W = list(w)
    else:
        W = [Decimal(1) / Decimal(3)] + [Decimal(1) / Decimal(18)] * 6 + [Decimal(1) / Decimal(36)] * 12
    H0 = _H_dec(F, W)

    def g(a):
        a = Decimal(a)
        return _H_dec([fi + a * (ei - fi) for fi, ei in zip(F, E)], W) - H0

    a, b = Decimal(lo), Decimal(hi)
    ga = g(a)
    for _ in range(iters):
        m = (a + b) / 2
        gm = g(m)
        if (gm > 0) == (ga > 0):
            a, ga = m, gm
        else:
            b = m
    return float((a + b) / 2)


@pytest.mark.parametrize("seed,jit,umax", [(0, 1e-2, 0.05), (1, 3e-2, 0.1), (2, 1e-1, 0.02), (3, 5e-3, 0.0)])
def test_alpha_vs_decimal_bisection(ora, seed, jit, umax):
    # Eq. entropic / Eq. H: the oracle's cancellation-free Newton must land on
    # the literal root of H(f + alpha Delta) = H(f).
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.5, 1.5)
    u0 = rng.uniform(-umax, umax, 3)
    f = ora.feq(rho, u0) * (1 + jit * rng.uniform(-1, 1, 19))
    c, w = ora.lattice()
    r = f.sum()
    u = (c.T @ f) / r
    fe = ora.feq(r, u)
    a, it = ora.alpha(f, fe, u, r)
    assert it >= 0
    x = (fe - f) / f
    amax = np.min(-1 / x[x < 0])
    ref = _alpha_decimal(f, fe, w, 1.0 if a > 1.0 else 0.05, min(amax, 2.0 * a) * (1 - 1e-12))
    assert abs(a - ref) <= 1e-11 * ref, (a, ref)


def test_alpha_where_polynomial_equilibrium_is_negative(ora):
    # A fast node: some f_eq_p < 0 while every f_p > 0.  H(f + alpha Delta) is
    # still defined on the positivity interval and the root must be the literal one.
    c, w = ora.lattice()
    rng = np.random.default_rng(6)
    fac = rng.uniform(5, 40)
    d = rng.normal(size=3)
    d /= np.linalg.norm(d)
    f = w * (1.0 + 0.5 * rng.uniform(-1, 1, 19)) * np.exp(fac / 10 * (c @ d))  # strong drift along d
    r = f.sum()
    u = (c.T @ f) / r
    fe = ora.feq(r, u)
    assert fe.min() < 0 < f.min()
    a, it = ora.alpha(f, fe, u, r)
    assert it >= 0
    x = (fe - f) / f
    amax = np.min(-1 / x[x < 0])
    # bracket the non-trivial root on a grid of the positivity interval, then bisect
    grid = np.linspace(1e-3, amax * (1 - 1e-9), 400)
    getcontext().prec = 60
    F = [Decimal(float(v)) for v in f]
    E = [Decimal(float(v)) for v in fe]
    W = [Decimal(1) / Decimal(3)] + [Decimal(1) / Decimal(18)] * 6 + [Decimal(1) / Decimal(36)] * 12
    H0 = _H_dec(F, W)
    g = [float(_H_dec([fi + Decimal(float(t)) * (ei - fi) for fi, ei in zip(F, E)], W) - H0) for t in grid]
    k = next(i for i in range(len(g) - 1) if g[i] < 0 <= g[i + 1])
    ref = _alpha_decimal(f, fe, w, grid[k], grid[k + 1])
    assert abs(a - ref) <= 1e-11 * ref, (a, ref)


def test_alpha_nonpositive_population_falls_back(ora):
    # H(f) needs f > 0: a non-positive population gives the fallback value.
    c, w = ora.lattice()
    u = np.zeros(3)
    fe = ora.feq(1.0, u)
    f = fe.copy()
    f[3] = -1e-3
    f[4] += 1e-3
    a, it = ora.alpha(f, fe, u, 1.0)
    assert it == -1


def test_alpha_equilibrium_is_bgk(ora):
    # f = f_eq: Delta = 0, the collision vanishes and alpha takes the BGK value 2.
    u = np.array([0.03, -0.02, 0.01])
    fe = ora.feq(0.8, u)
    a, it = ora.alpha(fe.copy(), fe, u, 0.8)
    assert a == 2.0 and it == 0


def test_alpha_small_jitter_at_rest_tends_to_two(ora):
    # At u = 0 the equilibrium w rho is the H minimiser, so alpha -> 2 linearly
    # in the deviation (the paper's BGK limit of the entropic step).
    c, w = ora.lattice()
    rng = np.random.default_rng(7)
    devs = []
    for jit in [1e-2, 1e-3, 1e-4]:
        f = w * 1.0 * (1 + jit * rng.uniform(-1, 1, 19))
        r = f.sum()
        u = (c.T @ f) / r
        a, it = ora.alpha(f, ora.feq(r, u), u, r)
        devs.append(abs(a - 2.0))
    assert devs[2] < 3e-4 and devs[1] < 3e-3
    assert devs[2] < devs[1] < devs[0]


def test_alpha_no_root_falls_back(ora):
    # L >= 0 means g(alpha) > 0 for every alpha > 0 (no entropy-preserving
    # mirror state): the fallback value min(2, 0.99 alpha_max) is returned.
    c, w = ora.lattice()
    u = np.array([0.3, 0.0, 0.0])
    rho = 1.0
    fe = ora.feq(rho, u)
    # a tiny deviation along a direction where the polynomial equilibrium is
    # far from the H minimiser: L is dominated by sum Delta ln(f_eq/(w rho))
    d = np.zeros(19)
    d[1], d[2] = 1e-9, -1e-9
    f = fe - d
    x = d / f
    L = np.sum(d * np.log(f / (w * rho)))
    assert L >= 0
    a, it = ora.alpha(f, fe, u, rho)
    amax = np.min(-1 / x[x < 0])
    assert it == -1 and a == min(2.0, 0.99 * amax)


def _minority_node(ora, seed):
    """A dilute, fast, strongly distorted node, as the minority component of
    a two-component interface: rho ~ 0.01-0.05, |u| up to 0.25."""
    c, w = ora.lattice()
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.01, 0.05)
    u0 = rng.normal(size=3)
    u0 *= rng.uniform(0.05, 0.25) / np.linalg.norm(u0)
    f = rho * ora.feq(1.0, u0) * (1 + rng.uniform(-0.5, 1.5, 19))
    r = f.sum()
    u = (c.T @ f) / r
    fe = ora.feq(r, u)
    x = (fe - f) / f
    return f, fe, u, r, w, np.min(-1 / x[x < 0])


def _g_dec(f, fe, w, a):
    """H(f + a (fe - f)) - H(f) in 60-digit decimal; a vanishing population
    contributes 0 ln 0 = 0 (the limit at the top of the positivity interval)."""
    getcontext().prec = 60
    F = [Decimal(float(v)) for v in f]
    E = [Decimal(float(v)) for v in fe]
    W = [Decimal(1) / Decimal(3)] + [Decimal(1) / Decimal(18)] * 6 + [Decimal(1) / Decimal(36)] * 12
    A = Decimal(float(a))
    P = [fi + A * (ei - fi) for fi, ei in zip(F, E)]
    return float(sum(pi * (pi / wi).ln() for pi, wi in zip(P, W) if pi > 0) - _H_dec(F, W))


@pytest.mark.parametrize("seed", [16, 20, 29])
def test_alpha_no_root_in_positivity_interval(ora, seed):
    # L < 0, yet H(f + alpha Delta) stays below H(f) up to the top of the
    # positivity interval, where one population vanishes: no entropy-preserving
    # mirror state exists, and the fallback min(2, 0.99 alpha_max) is returned.
    f, fe, u, r, w, amax = _minority_node(ora, seed)
    assert np.sum((fe - f) * np.log(f / (w * r))) < 0
    xs = np.concatenate([np.linspace(1e-3, amax * (1 - 1e-9), 60), [amax]])
    assert max(_g_dec(f, fe, w, t) for t in xs) < 0
    a, it = ora.alpha(f, fe, u, r)
    assert it == -1 and a == min(2.0, 0.99 * amax)


@pytest.mark.parametrize("seed", [5, 12])
def test_alpha_root_near_top_of_positivity_interval(ora, seed):
    # The root lies within a few per cent of alpha_max, where Newton steps from
    # 2 leave the interval: it must still be found, and be the literal one.
    f, fe, u, r, w, amax = _minority_node(ora, seed)
    a, it = ora.alpha(f, fe, u, r)
    assert it >= 0 and a > 0.97 * amax
    grid = np.linspace(0.5 * amax, amax * (1 - 1e-12), 200)
    g = [_g_dec(f, fe, w, t) for t in grid]
    k = next(i for i in range(len(g) - 1) if g[i] < 0 <= g[i + 1])
    ref = _alpha_decimal(f, fe, w, grid[k], grid[k + 1])
    assert abs(a - ref) <= 1e-11 * ref, (a, ref)


@pytest.mark.parametrize("seed", range(10))
def test_sym3_norm_vs_eigvalsh(ora, seed):
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(3, 3)) * 10.0 ** rng.uniform(-8, 0)
    A = A + A.T
    if seed == 9:  # repeated eigenvalues
        A = np.diag([1.0, -1.0, 1.0])
    ref = np.max(np.abs(np.linalg.eigvalsh(A)))
    got = ora.sym3_norm2([A[0, 0], A[1, 1], A[2, 2], A[0, 1], A[0, 2], A[1, 2]])
    assert abs(got - ref) <= 1e-14 * ref


def test_carreau_limits(ora):
    # Eq. carreau: nu(0) = nu0; n = 1 is Newtonian; nu -> nu_inf for shear-thinning at large rate.
    nu0, ninf = 0.5, 0.05
    assert ora.carreau_nu(0.0, nu0, ninf, 10.0, 0.5) == nu0
    for gd in [1e-3, 0.1, 10.0]:
        assert math.isclose(ora.carreau_nu(gd, nu0, ninf, 10.0, 1.0), nu0, rel_tol=1e-15)
    assert abs(ora.carreau_nu(1e9, nu0, ninf, 10.0, 0.5) - ninf) < 1e-4
    vals = [ora.carreau_nu(g, nu0, ninf, 10.0, 0.4) for g in np.logspace(-4, 3, 30)]
    assert all(a > b for a, b in zip(vals, vals[1:]))
    # closed form at lambda*gamma = 1: nu_inf + (nu0 - nu_inf) 2^((n-1)/2)
    assert math.isclose(ora.carreau_nu(0.1, nu0, ninf, 10.0, 0.5), ninf + (nu0 - ninf) * 2 ** -0.25,
                        rel_tol=1e-15)


@pytest.mark.parametrize("Pn,rho,alpha,n,lam", [(1e-3, 1.0, 2.0, 0.5, 10.0), (5e-2, 0.01, 1.7, 0.4, 20.0),
                                                 (1e-6, 1.2, 2.3, 0.3, 10.0), (2e-2, 0.5, 2.0, 0.9, 1000.0)])
def test_shear_rate_vs_brentq(ora, Pn, rho, alpha, n, lam):
    # Eq. strain2 solved literally: gamma = Pi / (rho tau(gamma) c_s^2),
    # tau = 1/(alpha beta), beta = c_s^2/(2 nu(gamma) + c_s^2).
    nu0, ninf = 0.5, 0.05

    def resid(g):
        nu = ninf + (nu0 - ninf) * (1 + (lam * g) ** 2) ** ((n - 1) / 2)
        beta = CS2 / (2 * nu + CS2)
        tau = 1.0 / (alpha * beta)
        return g - Pn / (rho * tau * CS2)

    ref = brentq(resid, 0.0, 10.0 * alpha * Pn / (rho * CS2), xtol=1e-300, rtol=1e-15, maxiter=500)
    got = ora.shear_rate(Pn, rho, alpha, nu0, ninf, lam, n)
    assert abs(got - ref) <= 1e-13 * ref


def test_shear_rate_newtonian_closed_form(ora):
    # n = 1: nu = nu0, so gamma = alpha Pi / (rho (2 nu0 + c_s^2)).
    Pn, rho, alpha, nu0 = 3e-3, 0.9, 1.95, 1.0 / 6.0
    got = ora.shear_rate(Pn, rho, alpha, nu0, 0.05, 10.0, 1.0)
    assert math.isclose(got, alpha * Pn / (rho * (2 * nu0 + CS2)), rel_tol=1e-14)
    assert ora.shear_rate(0.0, rho, alpha, nu0, 0.05, 10.0, 0.5) == 0.0


def test_shear_rate_degenerate_inputs(ora):
    # No stress, or a non-positive density (only after negative populations):
    # Eq. strain2 has no positive root and the shear rate is taken as zero.
    assert ora.shear_rate(0.0, 1.0, 2.0, 0.5, 0.05, 10.0, 0.5) == 0.0
    assert ora.shear_rate(1e-3, 0.0, 2.0, 0.5, 0.05, 10.0, 0.5) == 0.0
    assert ora.shear_rate(1e-3, -1e-3, 2.0, 0.5, 0.05, 10.0, 0.5) == 0.0
