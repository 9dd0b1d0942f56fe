"""The 2-D jet's printed set-up against its own definitions and the oracle
(fixture tests/golden/paper_jet_2d.txt, with its section).

Oh = nu0 sqrt(rho / (sigma a0)) and De = lambda sqrt(sigma / (rho a0^3))
(Eq. oh) with the drop section's printed sigma give the printed Oh and De;
with the oracle's own surface tension of the same fluid they stay within the
printed two digits' tolerance.  The charge model of Eq. surface-q3 with the
printed constants gives the printed surface-to-bulk ratio on the initial
state of the set-up, and the potentials make the printed uniform field."""
import math
import os

import numpy as np

from paper_1612_05404_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden(name):
    vals = {}
    for line in open(os.path.join(HERE, "golden", name)):
        line = line.split("#", 1)[0].strip()
        if line:
            k, v = line.split()
            vals[k] = float(v)
    return vals


def test_ohnesorge_and_deborah_numbers():
    g, d = _golden("paper_jet_2d.txt"), _golden("paper_charged_drop.txt")
    rho, a0, sigma = g["rho_liquid"], g["a0"], d["sigma"]
    oh = g["nu0"] * math.sqrt(rho / (sigma * a0))
    de = g["lambda"] * math.sqrt(sigma / (rho * a0 ** 3))
    assert abs(oh - g["Oh"]) <= 0.005 and abs(de - g["De"]) <= 0.05, (oh, de)
    # with the surface tension the oracle measures for this fluid (0.0554 to
    # 0.0558 by the Laplace law, tests/test_oracle_d2q9.py)
    for s in (0.0554, 0.0558):
        assert abs(g["nu0"] * math.sqrt(rho / (s * a0)) - g["Oh"]) <= 0.01
        assert abs(g["lambda"] * math.sqrt(s / (rho * a0 ** 3)) - g["De"]) <= 0.1


def test_set_up_matches_the_printed_parameters(ora):
    g = _golden("paper_jet_2d.txt")
    wl = inputs.paper_jet_2d(case="b")
    p, b = wl.params, wl.boxes[0]
    assert b.nx == b.ny == g["mesh"] and p.G[0][0] == g["G"] and p.Gw[0][0] == g["G_wall"]
    assert (p.xi_b, p.xi_s, p.rho_in[0], p.rho_out[0]) == (g["xi_b"], g["xi_s"], g["rho_liquid"], g["rho_gas"])
    assert (p.nu0, p.nu_inf, p.lam, p.n_flow) == (g["nu0"], g["nu_inf"], g["lambda"], g["n_b"])
    # the edge potentials are those of a uniform field of the printed strength,
    # zero one node left of the box and the printed right potential at the
    # printed spacing (to its 321 / 322 spread)
    phi = b.phi0[0]
    assert np.allclose(np.diff(phi[0, :]), -g["E_back"], rtol=0, atol=1e-12)
    assert abs(phi[0, 0] + g["E_back"]) < 1e-12
    assert abs(phi[0, -1] * 322.0 / 320.0 - g["phi_right"]) < 0.2
    # Eq. surface-q3 with the printed constants on the initial state: the
    # surface-to-bulk charge ratio the constants were tuned to
    o = ora.Oracle(p, b, nthreads=4)
    o.step(1)
    qb = p.xi_b * o.field(ora.F_BULK).sum()
    qs = p.xi_s * o.field(ora.F_SURF).sum()
    assert abs(qs / qb - g["Qs_over_Qb"]) <= 0.5, qs / qb
