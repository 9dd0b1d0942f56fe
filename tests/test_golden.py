"""The oracle against the numbers the paper prints for its charged drop
(fixture tests/golden/paper_charged_drop.txt, with its citation)."""
import math
import os

import numpy as np
import pytest

from paper_1612_05404_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden():
    vals = {}
    for line in open(os.path.join(HERE, "golden", "paper_charged_drop.txt")):
        line = line.split("#", 1)[0].strip()
        if line:
            k, v = line.split()
            vals[k] = float(v)
    return vals


def test_critical_point_of_the_equation_of_state():
    # With psi = 1 - exp(-rho) and p = c_s^2 (rho + G psi^2 / 2), the printed
    # critical coupling and density make dp/drho and d2p/drho2 vanish, and the
    # printed ratio G / G_crit follows.
    g = _golden()
    G, r = g["G_crit"], g["rho_crit"]
    assert r == pytest.approx(math.log(2.0), rel=1e-15)
    psi, d1, d2 = 1 - math.exp(-r), math.exp(-r), -math.exp(-r)
    assert abs(1 + G * psi * d1) < 1e-15
    assert abs(G * (d1 * d1 + psi * d2)) < 1e-15
    assert g["G"] / g["G_crit"] == pytest.approx(g["G_over_Gcrit"], rel=1e-15)


def test_flat_interface_reaches_the_printed_densities(ora):
    # The oracle's flat liquid/gas interface at the printed G relaxes to the
    # densities the paper starts its drop from, to the two digits printed.
    g = _golden()
    nz = 64
    z = np.arange(nz)
    rA = np.where((z >= 16) & (z < 48), g["rho_liquid"], g["rho_gas"])[:, None, None] * np.ones((nz, 2, 2))
    t = np.zeros((nz, 2, 2), np.uint8)
    b = inputs.Box(2, 2, nz, [1, 1, 1], t, rA[None], np.zeros((3, nz, 2, 2)), np.zeros((nz, 2, 2)),
                   np.zeros((3, nz, 2, 2)), np.zeros((1, 19, nz, 2, 2)), 0.0, {})
    p = inputs.Params(ncomp=1, G=[[g["G"], 0.0], [0.0, 0.0]], Q_b=0.0, Q_s=0.0, sor_sweeps=0, nu0=g["nu"])
    o = ora.Oracle(p, b, nthreads=1)
    o.step(3000)
    r = o.field(ora.F_RHO)[0, :, 0, 0]
    assert abs(r[32] - g["rho_liquid"]) < 0.1, r[32]
    assert abs(r[0] - g["rho_gas"]) < 0.01, r[0]


def test_bgk_limit_of_eq_beta(ora):
    # Eq. beta with the printed nu = 1/6 gives beta = 1/2, so alpha beta = 1 at
    # the BGK value alpha = 2: a resting fluid with a tiny non-equilibrium
    # part collides onto its own equilibrium up to |1 - alpha/2| ~ the jitter.
    g = _golden()
    cs2 = 1.0 / 3.0
    assert cs2 / (2 * g["nu"] + cs2) == pytest.approx(0.5, rel=1e-15)
    n = 4
    t = np.zeros((n, n, n), np.uint8)
    rho0 = np.ones((1, n, n, n))
    xi = inputs.jitter_draws(11, 1, n ** 3).reshape(1, 19, n, n, n)
    b = inputs.Box(n, n, n, [1, 1, 1], t, rho0, np.zeros((3, n, n, n)), np.zeros((n, n, n)),
                   np.zeros((3, n, n, n)), xi, 1e-6, {})
    p = inputs.Params(ncomp=1, G=[[0.0, 0.0], [0.0, 0.0]], Q_b=0.0, Q_s=0.0, sor_sweeps=0, nu0=g["nu"],
                      electrostriction=0)
    o = ora.Oracle(p, b, nthreads=1)
    o.step(1)
    fin = o.field(ora.F_PULLED)[0].reshape(19, -1)
    fout = o.field(ora.F_POP)[0].reshape(19, -1)
    c, _ = ora.lattice()
    rho = fin.sum(0)
    u = (c.T.astype(np.float64) @ fin) / rho
    feq = np.stack([ora.feq(rho[i], u[:, i]) for i in range(rho.size)], axis=1)
    ratio = np.abs(fout - feq).max() / np.abs(fin - feq).max()
    assert ratio < 1e-5, ratio


def test_printed_charge_split(ora):
    # Q = Q_s + Q_b = 2.13 with Q_s / Q_b = 10 (Eq. surface-q2 with K_d = 1):
    # the oracle's bulk and surface charges integrate to the two parts.
    g = _golden()
    Qb = g["Q_total"] / (1.0 + g["Qs_over_Qb"])
    Qs = g["Q_total"] - Qb
    b = inputs.droplet_box(24, 24, 24, 7.0, seed=3, ncomp=1, rho_in=g["rho_liquid"], rho_out=g["rho_gas"])
    p = inputs.Params(ncomp=1, G=[[g["G"], 0.0], [0.0, 0.0]], Q_b=Qb, Q_s=Qs, K_d=g["K_d"], sor_sweeps=2,
                      sor_omega=1.5, nu0=g["nu"], rho_th=0.5 * (g["rho_liquid"] + g["rho_gas"]))
    o = ora.Oracle(p, b, nthreads=1)
    o.step(1)
    q = o.field(ora.F_Q)
    bulk, surf = o.field(ora.F_BULK), o.field(ora.F_SURF)
    qb = Qb * bulk / bulk.sum()
    qs = Qs * surf / surf.sum()
    assert np.allclose(q, qb + qs, rtol=1e-12, atol=1e-15)
    assert q.sum() == pytest.approx(g["Q_total"], rel=1e-12)
    assert qs.sum() / qb.sum() == pytest.approx(g["Qs_over_Qb"], rel=1e-12)
