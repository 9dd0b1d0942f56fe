"""Seeded synthetic workloads for the charged two-phase entropic LB update.

This module is shared by the HIP path and by the CPU oracle.  It holds the
workload definitions only -- box sizes, node types, initial density fields,
boundary values, parameter sets and the random numbers a run draws -- and
none of the method's arithmetic (no equilibria, forces, charges or solves).

Random numbers come from SplitMix64 (Steele, Lea & Flood, OOPSLA 2014),
evaluated counter-based: draw ``i`` of stream ``seed`` is
``mix(seed + (i + 1) * 0x9E3779B97F4A7C15)``.

Node-type byte (x fastest, then y, then z):
  bits 0-1: 0 fluid, 1 solid wall, 2 inlet, 3 outlet;
  bit 2   : potential fixed (Dirichlet node of the Poisson problem).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Dict, List, Optional

import numpy as np

FLUID, SOLID, INLET, OUTLET = 0, 1, 2, 3
DIRICHLET = 4
NOZZLE = 8      # fluid node inside the nozzle: enters the adaptive inlet's mean velocity

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, counters: np.ndarray) -> np.ndarray:
    """SplitMix64 outputs for the given counters of stream ``seed`` (uint64)."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (counters.astype(np.uint64) + np.uint64(1)) * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def uniform01(seed: int, n: int, offset: int = 0) -> np.ndarray:
    """n doubles in [0, 1) from the top 53 bits of SplitMix64."""
    c = np.arange(offset, offset + n, dtype=np.uint64)
    return (splitmix64(seed, c) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def uniform(seed: int, n: int, lo: float, hi: float, offset: int = 0) -> np.ndarray:
    return lo + (hi - lo) * uniform01(seed, n, offset)


# --------------------------------------------------------------------------
# Parameter set of one run (the model constants of one box family)
# --------------------------------------------------------------------------
@dataclass
class Params:
    # lattice: 0 = D3Q19; 1 = D2Q9 (the paper's 2-D lattice; boxes with nz = 1,
    # bounded in z)
    lattice: int = 0
    ncomp: int = 2
    # Shan-Chen couplings G[s][t] and the fluid-wall couplings Gw[s][t]
    # (None: Gw = G, a neutral wall)
    G: List[List[float]] = field(default_factory=lambda: [[0.0, 3.0], [3.0, 0.0]])
    Gw: Optional[List[List[float]]] = None
    # rheology: Newtonian nu0 unless carreau
    carreau: int = 0
    nu0: float = 1.0 / 6.0
    nu_inf: float = 0.05
    lam: float = 10.0
    n_flow: float = 0.5
    # charge model: 0 conserving totals (Q_b, Q_s); 1 generator-connected (xi_b, xi_s)
    charge_model: int = 0
    Q_b: float = 1.0
    Q_s: float = 0.0
    xi_b: float = 1e-4
    xi_s: float = 6e-2
    K_d: float = 1.0
    curvature: int = 1
    electrostriction: int = 1
    rho_th: float = 0.5
    w_theta: float = 0.05
    E_ext: List[float] = field(default_factory=lambda: [0.0, 0.0, 0.0])
    # Poisson: red-black SOR, at most sor_sweeps sweeps per step; sor_tol > 0
    # stops them once the residual is at most sor_tol * max|rhs| (checked after
    # every sor_check_every sweeps, 0 = after the last only)
    sor_omega: float = 1.6
    sor_sweeps: int = 8
    sor_tol: float = 0.0
    sor_check_every: int = 0
    # entropic alpha Newton
    newton_rtol: float = 1e-12
    newton_max: int = 30
    # boundary densities (per component) of inlet and outlet nodes
    rho_in: List[float] = field(default_factory=lambda: [1.0, 0.01])
    rho_out: List[float] = field(default_factory=lambda: [0.01, 1.0])
    # inlet: 0 velocity u_bc at the neighbours' density; 1 + a: density rho_in
    # and velocity ubar * u_bc, ubar the mean velocity along axis a of the
    # fluid in the nozzle (NOZZLE nodes), measured every step
    inlet_mode: int = 0

    def with_(self, **kw) -> "Params":
        return replace(self, **kw)


@dataclass
class Box:
    """One lattice box: geometry, initial fields and the random draws."""
    nx: int
    ny: int
    nz: int
    periodic: List[int]
    node_type: np.ndarray          # uint8 [nz][ny][nx]
    rho0: np.ndarray               # float64 [C][nz][ny][nx]  initial component densities
    u0: np.ndarray                 # float64 [3][nz][ny][nx]  initial velocity
    phi0: np.ndarray               # float64 [nz][ny][nx]     initial / Dirichlet potential
    u_bc: np.ndarray               # float64 [3][nz][ny][nx]  inlet velocity (inlet nodes only)
    xi: np.ndarray                 # float64 [C][19][nz][ny][nx] jitter draws in [-1, 1)
    jitter: float                  # relative jitter amplitude
    info: Dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz


@dataclass
class Workload:
    name: str
    params: Params
    boxes: List[Box]
    dtype: str                     # "f64" or "f32" population storage
    steps: int                     # steps of the full run the workload describes
    info: Dict = field(default_factory=dict)

    @property
    def nodes(self) -> int:
        return sum(b.n for b in self.boxes)


def _min_image(coord: np.ndarray, centre: float, size: int, periodic: bool) -> np.ndarray:
    d = coord - centre
    if periodic:
        d = d - size * np.round(d / size)
    return d


def drop_profile(nx, ny, nz, centre, radius, width, rho_in, rho_out, periodic) -> np.ndarray:
    """Liquid density of a spherical drop with a tanh interface of the given width."""
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    dx = _min_image(x, centre[0], nx, periodic[0])
    dy = _min_image(y, centre[1], ny, periodic[1])
    dz = _min_image(z, centre[2], nz, periodic[2])
    d = np.sqrt(dx * dx + dy * dy + dz * dz)
    return rho_out + (rho_in - rho_out) * 0.5 * (1.0 - np.tanh(2.0 * (d - radius) / width))


def jitter_draws(seed: int, ncomp: int, n: int, q: int = 19) -> np.ndarray:
    """Jitter draws xi in [-1, 1): index (s * q + p) * n + node, q directions."""
    return uniform(seed, ncomp * q * n, -1.0, 1.0).reshape(ncomp, q, n)


def droplet_box(edge_x, edge_y, edge_z, radius, *, seed, periodic=(1, 1, 1), walls_z=False,
                phi_bottom=0.0, phi_top=0.0, rho_in=1.0, rho_out=0.01, width=2.0,
                jitter=1e-4, ncomp=2, q=19) -> Box:
    nx, ny, nz = edge_x, edge_y, edge_z
    n = nx * ny * nz
    t = np.zeros((nz, ny, nx), dtype=np.uint8)
    phi0 = np.zeros((nz, ny, nx))
    per = list(periodic)
    if walls_z:
        per[2] = 0
        t[0] = SOLID | DIRICHLET
        t[nz - 1] = SOLID | DIRICHLET
        # uniform-field start: linear potential between the two electrodes
        zz = np.arange(nz, dtype=np.float64)
        phi0[:] = (phi_bottom + (phi_top - phi_bottom) * zz / (nz - 1))[:, None, None]
    centre = ((nx - 1) / 2.0, (ny - 1) / 2.0, (nz - 1) / 2.0)
    rA = drop_profile(nx, ny, nz, centre, radius, width, rho_in, rho_out, per)
    if ncomp == 2:
        rho0 = np.stack([rA, rho_in + rho_out - rA])
    else:
        rho0 = rA[None]
    solid = (t & 3) == SOLID
    rho0[:, solid] = 0.0
    xi = jitter_draws(seed, ncomp, n, q).reshape(ncomp, q, nz, ny, nx)
    return Box(nx, ny, nz, per, t, rho0, np.zeros((3, nz, ny, nx)), phi0,
               np.zeros((3, nz, ny, nx)), xi, jitter,
               info=dict(radius=radius, centre=centre))


# --------------------------------------------------------------------------
# The five workloads of the study
# --------------------------------------------------------------------------
# Two-component Shan-Chen cross coupling.  Chosen so that a flat interface
# between the two components holds a minority density close to 0.01 on
# either side (calibrated with the oracle on a flat slab).
G_CROSS = 8.26


def base_params(**kw) -> Params:
    p = Params(G=[[0.0, G_CROSS], [G_CROSS, 0.0]])
    return p.with_(**kw)


def drop32(seed: int = 1234, n: int = 32, steps: int = 100) -> Workload:
    """Plain method, FP64: periodic cube, one charged drop at rest, no field."""
    box = droplet_box(n, n, n, 8.0 * n / 32.0, seed=seed)
    p = base_params(Q_b=1.0, Q_s=0.0, carreau=0, nu0=1.0 / 6.0,
                    sor_omega=sor_omega_opt(n, n, n, True), sor_sweeps=8)
    return Workload("drop32", p, [box], "f64", steps, info=dict(seed=seed))


def sor_omega_opt(nx, ny, nz, periodic: bool) -> float:
    nmax = max(nx, ny, nz)
    k = 2.0 if periodic else 1.0
    return 2.0 / (1.0 + math.sin(k * math.pi / nmax))


def efield_drop(seed: int = 1235, nx: int = 64, ny: int = 64, nz: int = 128,
                steps: int = 2000) -> Workload:
    """Drop between two fixed-potential electrodes (uniform E_z = 1e-3), Carreau fluid, FP32."""
    radius = 16.0 * nz / 128.0
    ez = 1e-3
    box = droplet_box(nx, ny, nz, radius, seed=seed, walls_z=True,
                      phi_bottom=0.0, phi_top=-ez * (nz - 1))
    rho_q = float(uniform(seed ^ 0x5A5A, 1, 1e-4, 1e-3)[0])
    Q = rho_q * 4.0 / 3.0 * math.pi * radius ** 3
    p = base_params(Q_b=Q, Q_s=0.0, carreau=1, nu0=0.5, nu_inf=0.05, lam=10.0, n_flow=0.5,
                    sor_omega=sor_omega_opt(nx, ny, nz, False), sor_sweeps=8)
    box.info.update(rho_q=rho_q, E_z=ez)
    return Workload("efield_drop", p, [box], "f32", steps, info=dict(seed=seed, rho_q=rho_q))


def jet(seed: int = 1236, nx: int = 128, ny: int = 128, nz: int = 512, steps: int = 10000,
        r_noz: float = 8.0, u_mean: float = 0.02, ez: float = 2e-3) -> Workload:
    """Electrified jet: nozzle in a plate at z=0, collector/outlet plane at z=nz-1."""
    n = nx * ny * nz
    t = np.zeros((nz, ny, nx), dtype=np.uint8)
    phi0 = np.zeros((nz, ny, nx))
    u_bc = np.zeros((3, nz, ny, nx))
    cx, cy = (nx - 1) / 2.0, (ny - 1) / 2.0
    # 1% azimuthal perturbation of the nozzle radius, 8 seeded Fourier modes
    a = uniform(seed, 8, -1.0, 1.0)
    a = a / np.sum(np.abs(a))
    ph = uniform(seed, 8, 0.0, 2.0 * math.pi, offset=8)
    yy, xx = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64), indexing="ij")
    dx, dy = xx - cx, yy - cy
    r = np.sqrt(dx * dx + dy * dy)
    th = np.arctan2(dy, dx)
    rth = r_noz * (1.0 + 0.01 * sum(a[k] * np.cos((k + 1) * th + ph[k]) for k in range(8)))
    inside = r < rth
    t[0] = np.where(inside, INLET, SOLID) | DIRICHLET
    t[nz - 1] = OUTLET | DIRICHLET
    zz = np.arange(nz, dtype=np.float64)
    phi0[:] = (-ez * zz)[:, None, None]
    u_bc[2, 0] = np.where(inside, 2.0 * u_mean * (1.0 - (r / rth) ** 2), 0.0)
    # ambient everywhere, a drop of liquid sitting on the nozzle
    rA = drop_profile(nx, ny, nz, (cx, cy, r_noz), r_noz, 2.0, 1.0, 0.01, (1, 1, 0))
    rA[0] = np.where(inside, 1.0, 0.0)
    rho0 = np.stack([rA, 1.01 - rA])
    rho0[1, 0] = np.where(inside, 0.01, 0.0)
    rho0[:, nz - 1] = np.array([0.01, 1.0])[:, None, None]
    xi = jitter_draws(seed, 2, n).reshape(2, 19, nz, ny, nx)
    box = Box(nx, ny, nz, [1, 1, 0], t, rho0, np.zeros((3, nz, ny, nx)), phi0, u_bc, xi, 1e-4,
              info=dict(r_noz=r_noz, u_mean=u_mean, E_z=ez))
    p = base_params(charge_model=1, xi_b=1e-4, xi_s=6e-2, carreau=1, nu0=0.8, nu_inf=0.05,
                    lam=20.0, n_flow=0.4, sor_omega=sor_omega_opt(nx, ny, nz, False), sor_sweeps=8,
                    rho_in=[1.0, 0.01], rho_out=[0.01, 1.0])
    return Workload("jet", p, [box], "f32", steps, info=dict(seed=seed))


def ensemble(seed: int = 1238, nboxes: int = 256, edges=(24, 32, 48, 64), steps: int = 1000) -> Workload:
    """Independent periodic drop boxes of uneven size, each with its own parameters."""
    e = np.array(edges)[np.floor(uniform(seed, nboxes, 0, len(edges))).astype(int)]
    radius = np.minimum(uniform(seed, nboxes, 6.0, 20.0, offset=nboxes), e / 3.0)
    rho_q = uniform(seed, nboxes, 1e-4, 1e-3, offset=2 * nboxes)
    ez = uniform(seed, nboxes, 0.0, 2e-3, offset=3 * nboxes)
    nfl = uniform(seed, nboxes, 0.3, 1.0, offset=4 * nboxes)
    boxes = []
    for b in range(nboxes):
        edge = int(e[b])
        box = droplet_box(edge, edge, edge, float(radius[b]), seed=seed * 1000003 + b)
        box.info.update(E_ext=[0.0, 0.0, float(ez[b])], Q_b=float(rho_q[b] * 4.0 / 3.0 * math.pi * radius[b] ** 3),
                        n_flow=float(nfl[b]), sor_omega=sor_omega_opt(edge, edge, edge, True))
        boxes.append(box)
    p = base_params(carreau=1, nu0=0.5, nu_inf=0.05, lam=10.0, sor_sweeps=8)
    return Workload("ensemble", p, boxes, "f32", steps, info=dict(seed=seed))


def paper_drop_2d(n: int = 320, radius: float = 40.0, Q: float = 2.13, surface_ratio: float = 10.0,
                  E_ext: float = 0.0, steps: int = 1000, width: float = 2.0, seed: int = 1240) -> Workload:
    """The paper's charged drop (Sec. III.A) on its own lattice: a periodic
    n x n D2Q9 mesh, one Shan-Chen fluid with G = -5 (psi = 1 - exp(-rho)), a
    circular drop of density 2.0 and radius 40 in vapour of density 0.16, total
    charge Q = Q_s + Q_b = 2.13 with Q_s / Q_b = 10 (Eq. surface-q2, K_d = 1),
    a uniform neutralising charge, F_el = q E (the force the section uses),
    Newtonian with nu = 1/6; E_ext along x for the drop in a field."""
    box = droplet_box(n, n, 1, radius, seed=seed, periodic=(1, 1, 0), rho_in=2.0, rho_out=0.16, width=width,
                      jitter=0.0, ncomp=1, q=9)
    Q_b = Q / (1.0 + surface_ratio)
    p = Params(lattice=1, ncomp=1, G=[[-5.0, 0.0], [0.0, 0.0]], carreau=0, nu0=1.0 / 6.0, Q_b=Q_b,
               Q_s=Q - Q_b, K_d=1.0, curvature=1, electrostriction=0, rho_th=1.0, w_theta=0.05,
               E_ext=[E_ext, 0.0, 0.0], sor_omega=sor_omega_opt(n, n, 1, True), sor_sweeps=400, sor_tol=1e-5,
               sor_check_every=4, rho_in=[2.0, 0.0], rho_out=[0.16, 0.0])
    return Workload("paper_drop_2d", p, [box], "f64", steps, info=dict(seed=seed, radius=radius, Q=Q))


PAPER_JET_CASES = {
    # Sec. III.B: case a Newtonian; b and c Carreau with nu_inf = 0.001,
    # lambda = 1000 and flow index 0.75 / 0.5
    "a": dict(carreau=0, n_flow=1.0),
    "b": dict(carreau=1, n_flow=0.75),
    "c": dict(carreau=1, n_flow=0.5),
}


def paper_jet_2d(case: str = "b", n: int = 320, diameter: int = 40, nozzle_len: int = 40, wall: int = 4,
                 E0: float = 0.1, steps: int = 25000, width: float = 2.0, seed: int = 1241) -> Workload:
    """The paper's electrospinning set-up (Sec. III.B) on its own lattice: an
    n x n D2Q9 mesh, one Shan-Chen fluid (G = G_w = -5), bounce-back walls on
    the bottom and top rows, a nozzle of inner diameter 40 on the left (a tube
    of `wall`-node walls reaching `nozzle_len` nodes into the box from a solid
    left column that holds the inlet nodes), outlet nodes on the right column
    in contact with a gas reservoir (density 0.16), the generator charge model
    (Eq. surface-q3, xi_b = 1e-4, xi_s = 6e-2, K_d = 1) and Dirichlet
    potentials on every edge, phi = -E0 (x + 1) (phi = 0 one node left of the
    box, a uniform field E0 = 0.1 along x).  The inlet holds the liquid
    density 2.0 and a Poiseuille profile 1.5 (1 - (y - y_c)^2 / a0^2) (unit
    mean) scaled every step by the mean velocity inside the nozzle.  Liquid
    (2.0) fills the nozzle with a drop of radius a0 = diameter/2 just outside
    it; gas (0.16) elsewhere.  `case`: "a" Newtonian nu = 1/6, "b" / "c"
    Carreau (nu0 = 1/6, nu_inf = 0.001, lambda = 1000, n = 0.75 / 0.5)."""
    a0 = diameter / 2.0
    yc = (n - 1) / 2.0
    xx = np.arange(n, dtype=np.float64)[None, :]
    yy = np.arange(n, dtype=np.float64)[:, None]
    dy = np.abs(yy - yc) + 0.0 * xx
    chan = dy < a0
    tube = (dy > a0) & (dy < a0 + wall) & (xx < nozzle_len)
    t = np.full((n, n), FLUID, dtype=np.uint8)
    t[tube] = SOLID
    t[:, -1] = OUTLET
    t[:, 0] = np.where(chan[:, 0], INLET, SOLID)
    t[0, :] = SOLID
    t[-1, :] = SOLID
    edge = np.zeros((n, n), dtype=bool)
    edge[:, 0] = edge[:, -1] = edge[0, :] = edge[-1, :] = True
    t[edge] |= DIRICHLET
    t[chan & (xx >= 1) & (xx < nozzle_len) & ((t & 3) == FLUID)] |= NOZZLE
    phi0 = -E0 * (xx + 1.0) + 0.0 * yy
    u_bc = np.zeros((3, 1, n, n))
    u_bc[0, 0] = np.where(t == (INLET | DIRICHLET), 1.5 * (1.0 - ((yy - yc) / a0) ** 2), 0.0)
    drop = drop_profile(n, n, 1, (float(nozzle_len), yc, 0.0), a0, width, 2.0, 0.16, (0, 0, 0))[0]
    rho = np.where(chan & (xx < nozzle_len), 2.0, drop)
    rho = np.where((t & 3) == SOLID, 0.0, rho)
    rho = np.where((t & 3) == INLET, 2.0, rho)
    rho = np.where((t & 3) == OUTLET, 0.16, rho)
    xi = jitter_draws(seed, 1, n * n, q=9).reshape(1, 9, 1, n, n)
    box = Box(n, n, 1, [0, 0, 0], t[None].copy(), rho[None, None].copy(), np.zeros((3, 1, n, n)), phi0[None].copy(),
              u_bc, xi, 0.0, info=dict(case=case, a0=a0, nozzle_len=nozzle_len, wall=wall, E0=E0))
    p = Params(lattice=1, ncomp=1, G=[[-5.0, 0.0], [0.0, 0.0]], Gw=[[-5.0, 0.0], [0.0, 0.0]], nu0=1.0 / 6.0,
               nu_inf=0.001, lam=1000.0, charge_model=1, xi_b=1e-4, xi_s=6e-2, K_d=1.0, curvature=1,
               electrostriction=0, rho_th=1.0, w_theta=0.05, E_ext=[0.0, 0.0, 0.0],
               sor_omega=sor_omega_opt(n, n, 1, False), sor_sweeps=400, sor_tol=1e-5, sor_check_every=4,
               rho_in=[2.0, 0.0], rho_out=[0.16, 0.0], inlet_mode=1, **PAPER_JET_CASES[case])
    return Workload("paper_jet_2d", p, [box], "f64", steps, info=dict(seed=seed, case=case))


WORKLOADS = {"drop32": drop32, "efield_drop": efield_drop, "jet": jet, "ensemble": ensemble,
             "paper_drop_2d": paper_drop_2d, "paper_jet_2d": paper_jet_2d}
