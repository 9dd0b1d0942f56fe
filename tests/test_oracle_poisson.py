"""Pins of the oracle's Poisson problem (Sec. II, Gauss law div(eps E) = q with
E = E_ext - grad phi and eps = 1 + rho_A), through the functions the oracle's
step calls: the right-hand side sum_f eps_f E_ext . e_f - (q - qbar), the
red-black SOR with its stop rule, and the residual.  Expected values come
from closed forms of electrostatics (a layered dielectric, a dielectric
sphere in a uniform field), the solvability condition of the periodic
problem, and the step's own fields."""
import math

import numpy as np
import pytest

from paper_1612_05404_amd import inputs


def _box(nx, ny, nz, rhoA, periodic=(1, 1, 1), node_type=None, ncomp=2):
    """A box with a given liquid density field (no jitter) and node types."""
    b = inputs.droplet_box(nx, ny, nz, 1.0, seed=5, periodic=periodic, jitter=0.0, ncomp=ncomp)
    if node_type is not None:
        b.node_type = np.asarray(node_type, dtype=np.uint8)
        b.periodic = list(periodic)
    rA = np.asarray(rhoA, dtype=np.float64) * np.ones((nz, ny, nx))
    b.rho0 = np.stack([rA, 1.01 - rA]) if ncomp == 2 else rA[None].copy()
    return b


def _params(**kw):
    kw.setdefault("sor_sweeps", 0)
    return inputs.base_params(Q_b=0.0, Q_s=0.0, **kw)


def test_layered_dielectric_constant_flux(ora):
    # Gauss law with no free charge in a periodic stack of layers eps(z) and an
    # external field along the stack: div D = 0 makes the displacement
    # D_z = eps_f (E_z - dphi/dz) the same on every face, and the periodic phi
    # fixes it to the harmonic mean, D_z = E_z N / sum_f (1 / eps_f).  A field
    # along the layers (E_x) leaves phi flat.
    nz = 32
    rng = np.random.default_rng(7)
    eps_z = 1.0 + rng.uniform(0.05, 1.5, nz)
    E = [2e-3, 0.0, 3e-3]
    b = _box(2, 2, nz, 0.5)
    o = ora.Oracle(_params(E_ext=E), b, nthreads=4)
    eps = np.broadcast_to(eps_z[:, None, None], (nz, 2, 2)).copy()
    q = np.zeros_like(eps)
    rhs, qbar = o.poisson_rhs(eps, q)
    assert qbar == 0.0
    phi = np.zeros_like(eps)
    done, res, sc = o.poisson_solve(eps, rhs, phi, 20000, 1.8, tol=1e-13, check_every=50)
    assert res <= 1e-13 * sc, (done, res, sc)
    # phi is flat across the layers (E_x along them adds no flux)
    assert np.abs(phi - phi[:, :1, :1]).max() <= 1e-14
    pz = phi[:, 0, 0]
    ef = 0.5 * (eps_z + np.roll(eps_z, -1))            # face between z and z + 1
    D = ef * (E[2] - (np.roll(pz, -1) - pz))
    closed = E[2] * nz / np.sum(1.0 / ef)
    assert np.abs(D - closed).max() <= 1e-12 * closed, (D.min(), D.max(), closed)


def test_layered_dielectric_through_the_step(ora):
    # The same stack set up through the step itself: a periodic box whose liquid
    # density varies only with z and carries no charge.  The step's right-hand
    # side equals the stand-alone one for eps = 1 + rho_A, and after a converged
    # solve the step's E gives the constant displacement of the closed form.
    nz = 24
    z = np.arange(nz)
    rA = 0.3 + 0.6 * (0.5 + 0.5 * np.cos(2 * math.pi * z / nz))
    Ez = 2e-3
    b = _box(2, 2, nz, rA[:, None, None])
    p = _params(E_ext=[0.0, 0.0, Ez], sor_sweeps=6000, sor_omega=1.8, sor_tol=1e-13, sor_check_every=100)
    o = ora.Oracle(p, b, nthreads=4)
    o.step(1)
    rho = o.field(ora.F_RHO)[0]
    eps = 1.0 + rho
    rhs_step = o.field(ora.F_RHS)
    rhs, qbar = o.poisson_rhs(eps, np.zeros_like(eps))
    assert np.array_equal(rhs, rhs_step)
    st = o.poisson_stats()
    assert st["residual"] <= 1e-13 * st["scale"], st
    phi = o.field(ora.F_PHI)[:, 0, 0]
    ez = eps[:, 0, 0]
    ef = 0.5 * (ez + np.roll(ez, -1))
    D = ef * (Ez - (np.roll(phi, -1) - phi))
    closed = Ez * nz / np.sum(1.0 / ef)
    assert np.abs(D - closed).max() <= 1e-11 * closed


def test_dielectric_sphere_in_uniform_field(ora):
    # A dielectric sphere (eps_in) in a medium (eps_out) under a uniform field
    # E0: the field inside is uniform, E_in = 3 eps_out / (eps_in + 2 eps_out) E0
    # (textbook electrostatics).  Periodic box, the sphere's volume fraction below
    # 1 %, a diffuse tanh interface: lattice accuracy, a few per cent.
    n, R = 40, 6.0
    c = (n - 1) / 2.0
    zz, yy, xx = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    d = np.sqrt((xx - c) ** 2 + (yy - c) ** 2 + (zz - c) ** 2)
    rA = 0.01 + 0.99 * 0.5 * (1.0 - np.tanh(2.0 * (d - R) / 1.0))
    E0 = 1e-3
    b = _box(n, n, n, rA)
    o = ora.Oracle(_params(E_ext=[0.0, 0.0, E0]), b, nthreads=8)
    eps = 1.0 + rA
    rhs, qbar = o.poisson_rhs(eps, np.zeros_like(eps))
    phi = np.zeros_like(eps)
    omega = 2.0 / (1.0 + math.sin(2.0 * math.pi / n))
    done, res, sc = o.poisson_solve(eps, rhs, phi, 4000, omega, tol=1e-11, check_every=50)
    assert res <= 1e-11 * sc, (done, res, sc)
    Ez = E0 - 0.5 * (np.roll(phi, -1, axis=0) - np.roll(phi, 1, axis=0))
    Ex = -0.5 * (np.roll(phi, -1, axis=2) - np.roll(phi, 1, axis=2))
    core = d < R / 2
    e_in, e_out = 2.0, 1.01
    expect = 3.0 * e_out / (e_in + 2.0 * e_out) * E0
    assert abs(Ez[core].mean() / expect - 1.0) < 0.03, (Ez[core].mean(), expect)
    assert (Ez[core].max() - Ez[core].min()) < 0.02 * expect          # uniform inside
    assert np.abs(Ex[core]).max() < 0.01 * expect                     # along E0
    # far from the sphere the field returns to E0 (within the periodic images)
    far = d > 0.45 * n
    assert abs(Ez[far].mean() / E0 - 1.0) < 0.02


def test_periodic_rhs_is_solvable(ora):
    # The periodic Poisson problem is solvable only when its right-hand side sums
    # to zero: the external-field fluxes cancel face by face and the neutralising
    # charge qbar = sum q / N removes the net charge.  A converged solve then
    # reaches a residual at rounding level.
    rng = np.random.default_rng(3)
    nx, ny, nz = 8, 6, 10
    b = _box(nx, ny, nz, 0.5)
    E = [1e-3, -2e-3, 3e-3]
    o = ora.Oracle(_params(E_ext=E), b, nthreads=4)
    eps = 1.0 + rng.uniform(0.0, 1.0, (nz, ny, nx))
    q = rng.uniform(0.0, 1e-3, (nz, ny, nx))
    rhs, qbar = o.poisson_rhs(eps, q)
    assert abs(qbar - q.mean()) <= 1e-15 * q.mean()
    assert abs(rhs.sum()) <= 1e-15 * np.abs(rhs).sum()
    phi = np.zeros_like(eps)
    done, res, sc = o.poisson_solve(eps, rhs, phi, 5000, 1.7, tol=1e-13, check_every=25)
    assert res <= 1e-13 * sc and done < 5000
    assert abs(phi.mean()) <= 1e-15 * np.abs(phi).max()               # the zero-mean gauge


def test_dirichlet_box_neutralises_unknown_nodes(ora):
    # With fixed-potential nodes the neutralising charge is the mean over the
    # Poisson-unknown nodes only (the walls hold no charge of their own), and the
    # solve converges to the discrete solution for any right-hand side.
    rng = np.random.default_rng(4)
    nx, ny, nz = 6, 6, 12
    b = inputs.droplet_box(nx, ny, nz, 2.0, seed=9, walls_z=True, phi_bottom=0.0, phi_top=-0.011, jitter=0.0)
    o = ora.Oracle(_params(), b, nthreads=4)
    eps = 1.0 + rng.uniform(0.0, 1.0, (nz, ny, nx))
    q = rng.uniform(0.0, 1e-3, (nz, ny, nx))
    unknown = (b.node_type & inputs.DIRICHLET) == 0
    rhs, qbar = o.poisson_rhs(eps, q)
    assert abs(qbar - q[unknown].mean()) <= 1e-15 * qbar
    assert abs(rhs[unknown].sum()) <= 1e-14 * np.abs(rhs[unknown]).sum()
    phi = b.phi0.copy()
    done, res, sc = o.poisson_solve(eps, rhs, phi, 4000, 1.7, tol=1e-13, check_every=25)
    assert res <= 1e-13 * sc
    assert np.array_equal(phi[~unknown], b.phi0[~unknown])


def test_stop_rule_counts_and_checks(ora):
    # The stop rule: sweeps end at the first check (every m sweeps) whose residual
    # is within tol * max|rhs|; tol = 0 runs exactly the given sweeps; the
    # residual reported is the one after the last sweep done.
    rng = np.random.default_rng(5)
    b = _box(8, 8, 8, 0.5)
    o = ora.Oracle(_params(E_ext=[0.0, 0.0, 1e-3]), b, nthreads=4)
    eps = 1.0 + rng.uniform(0.0, 1.0, (8, 8, 8))
    q = rng.uniform(0.0, 1e-3, (8, 8, 8))
    rhs, _ = o.poisson_rhs(eps, q)
    phi = np.zeros_like(eps)
    n, r, sc = o.poisson_solve(eps, rhs, phi, 7, 1.5)
    assert n == 7
    r2, sc2 = o.poisson_residual(eps, rhs, phi + 0.5)                 # gauge-free
    assert abs(r2 - r) <= 1e-9 * r and sc2 == sc
    phi = np.zeros_like(eps)
    n, r, sc = o.poisson_solve(eps, rhs, phi, 400, 1.5, tol=1e-6, check_every=4)
    assert n % 4 == 0 and r <= 1e-6 * sc
    phi2 = np.zeros_like(eps)
    n2, r2, _ = o.poisson_solve(eps, rhs, phi2, n - 4, 1.5)
    assert r2 > 1e-6 * sc                                             # the check before did not pass


def test_generator_charge_sharp_theta_and_flat_interface(ora):
    # Eq. surface-q3: q = xi_b rho_A theta + xi_s |grad rho_A|^2 w_K.  In the sharp
    # limit of theta the bulk part sums to xi_b times the liquid mass (nodes above
    # the threshold); on a flat interface the curvature vanishes (w_K = 1) and the
    # surface part sums to xi_s times the integral of (d rho/dz)^2 across the
    # profile, 2 b^2 / (3 W) per interface for a tanh step of height b, width W.
    n, W, b_ = 64, 12.0, 0.9
    z = np.arange(n)
    prof = 0.05 + b_ * 0.5 * (np.tanh(2.0 * (z - 16.0) / W) - np.tanh(2.0 * (z - 48.0) / W))
    box = _box(4, 4, n, prof[:, None, None])
    p = inputs.base_params(charge_model=1, xi_b=1.0, xi_s=0.0, sor_sweeps=0, w_theta=1e-9)
    o = ora.Oracle(p, box, nthreads=4)
    o.step(1)
    rho = o.field(ora.F_RHO)[0]
    q = o.field(ora.F_Q)
    assert abs(q.sum() - rho[rho > p.rho_th].sum()) <= 1e-12 * q.sum()
    p2 = inputs.base_params(charge_model=1, xi_b=0.0, xi_s=1.0, sor_sweeps=0)
    o2 = ora.Oracle(p2, box, nthreads=4)
    o2.step(1)
    K = o2.field(ora.F_K)
    g = o2.field(ora.F_GRAD)
    g2 = (g ** 2).sum(axis=0)
    q2 = o2.field(ora.F_Q)
    band = g2 > 1e-3 * g2.max()
    assert np.abs(K[band]).max() == 0.0
    assert np.array_equal(q2[band], g2[band])
    per_interface = q2.sum() / (2 * 4 * 4)
    assert abs(per_interface / (2.0 * b_ ** 2 / (3.0 * W)) - 1.0) < 0.02, per_interface


def test_point_charge_field_is_coulomb(ora):
    # Gauss law in a uniform dielectric: a positive point charge Q drives an
    # outward field of magnitude Q_enc / (4 pi eps r^2), Q_enc = Q minus the
    # neutralising background inside radius r, sampled by central differences
    # of phi along the axes (the difference of 1/r gives 1/(r^2 - 1)); periodic
    # box, lattice accuracy a few per cent at 7 to 9 spacings.
    n, Q, eps0 = 40, 1e-2, 1.5
    c = n // 2
    b = _box(n, n, n, 0.5)
    o = ora.Oracle(_params(), b, nthreads=8)
    eps = np.full((n, n, n), eps0)
    q = np.zeros((n, n, n))
    q[c, c, c] = Q
    rhs, qbar = o.poisson_rhs(eps, q)
    phi = np.zeros_like(eps)
    omega = 2.0 / (1.0 + math.sin(2.0 * math.pi / n))
    done, res, sc = o.poisson_solve(eps, rhs, phi, 4000, omega, tol=1e-12, check_every=50)
    assert res <= 1e-12 * sc
    for r in (7, 8, 9):
        expect = Q / (4.0 * math.pi * eps0 * (r * r - 1)) - Q * r / (3.0 * eps0 * n ** 3)
        # outward components along the six axis directions, central differences
        ex_p = -0.5 * (phi[c, c, c + r + 1] - phi[c, c, c + r - 1])
        ex_m = +0.5 * (phi[c, c, c - r + 1] - phi[c, c, c - r - 1])
        ey_p = -0.5 * (phi[c, c + r + 1, c] - phi[c, c + r - 1, c])
        ez_p = -0.5 * (phi[c + r + 1, c, c] - phi[c + r - 1, c, c])
        for e in (ex_p, ex_m, ey_p, ez_p):
            assert abs(e / expect - 1.0) < 0.03, (r, e, expect)
