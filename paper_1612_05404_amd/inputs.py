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


WORKLOADS = {"drop32": drop32, "efield_drop": efield_drop, "jet": jet, "ensemble": ensemble,
             "paper_drop_2d": paper_drop_2d}
