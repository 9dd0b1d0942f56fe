"""CPU oracle of the charged two-phase entropic LB update (test infrastructure).

Plain FP64 C (``elbm_oracle.c``, scalar loops, OpenMP over z) behind ctypes.
Only the tests, the smoke check and the benchmark's CPU-baseline leg use it;
the product path never imports it.  It shares no code with the HIP library.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "elbm_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

Q = 19
F_RHO, F_J, F_PSI, F_GRAD, F_NHAT, F_K, F_BULK, F_SURF, F_Q, F_PHI, F_RHS, F_E, F_E2, \
    F_FEL, F_F, F_ALPHA, F_NU, F_UPH, F_POP, F_PULLED = range(20)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain IEEE double: no fast-math, no FMA contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-o", LIB + ".tmp", SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


class OraParams(ct.Structure):
    _fields_ = [
        ("nx", ct.c_int32), ("ny", ct.c_int32), ("nz", ct.c_int32), ("ncomp", ct.c_int32),
        ("periodic", ct.c_int32 * 3),
        ("carreau", ct.c_int32), ("curvature", ct.c_int32), ("electrostriction", ct.c_int32),
        ("charge_model", ct.c_int32),
        ("sor_sweeps", ct.c_int32), ("newton_max", ct.c_int32), ("nthreads", ct.c_int32),
        ("pad_", ct.c_int32),
        ("G", (ct.c_double * 2) * 2), ("Gw", (ct.c_double * 2) * 2),
        ("nu0", ct.c_double), ("nu_inf", ct.c_double), ("lam", ct.c_double), ("n_flow", ct.c_double),
        ("Q_b", ct.c_double), ("Q_s", ct.c_double), ("xi_b", ct.c_double), ("xi_s", ct.c_double),
        ("K_d", ct.c_double), ("rho_th", ct.c_double), ("w_theta", ct.c_double),
        ("E_ext", ct.c_double * 3),
        ("sor_omega", ct.c_double), ("newton_rtol", ct.c_double),
        ("rho_in", ct.c_double * 2), ("rho_out", ct.c_double * 2),
        ("sor_tol", ct.c_double), ("sor_check_every", ct.c_int32), ("lattice", ct.c_int32),
        ("inlet_mode", ct.c_int32), ("pad2_", ct.c_int32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=True)
        L = ct.CDLL(LIB)
        dp = ct.POINTER(ct.c_double)
        L.ora_create.restype = ct.c_void_p
        L.ora_create.argtypes = [ct.POINTER(OraParams), ct.c_void_p, ct.c_void_p, ct.c_void_p]
        L.ora_destroy.argtypes = [ct.c_void_p]
        L.ora_init.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_double]
        L.ora_step.argtypes = [ct.c_void_p, ct.c_int]
        L.ora_field.restype = ct.c_int64
        L.ora_field.argtypes = [ct.c_void_p, ct.c_int, ct.c_void_p]
        L.ora_iters.argtypes = [ct.c_void_p, ct.c_void_p]
        L.ora_set_populations.argtypes = [ct.c_void_p, ct.c_void_p]
        L.ora_set_phi.argtypes = [ct.c_void_p, ct.c_void_p]
        L.ora_counters.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_void_p]
        L.ora_feq.argtypes = [ct.c_double, dp, dp]
        L.ora_alpha.restype = ct.c_double
        L.ora_alpha.argtypes = [dp, dp, dp, ct.c_double, ct.c_double, ct.c_double, ct.c_int,
                                ct.POINTER(ct.c_int)]
        L.ora_sym3_norm2.restype = ct.c_double
        L.ora_sym3_norm2.argtypes = [dp]
        L.ora_carreau_nu.restype = ct.c_double
        L.ora_carreau_nu.argtypes = [ct.c_double] * 5
        L.ora_shear_rate.restype = ct.c_double
        L.ora_shear_rate.argtypes = [ct.c_double] * 7
        L.ora_lattice.argtypes = [ct.c_void_p, ct.c_void_p]
        L.ora_inlet_ubar.restype = ct.c_double
        L.ora_inlet_ubar.argtypes = [ct.c_void_p]
        L.ora_lattice_q.restype = ct.c_int
        L.ora_lattice_q.argtypes = [ct.c_int, ct.c_void_p, ct.c_void_p]
        L.ora_feq_lat.argtypes = [ct.c_int, ct.c_double, dp, dp]
        L.ora_alpha_lat.restype = ct.c_double
        L.ora_alpha_lat.argtypes = [ct.c_int, dp, dp, ct.c_double, ct.c_double, ct.c_double, ct.c_int,
                                    ct.POINTER(ct.c_int)]
        L.ora_threads.restype = ct.c_int
        L.ora_poisson.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int,
                                  ct.c_double]
        L.ora_poisson_rhs.restype = ct.c_double
        L.ora_poisson_rhs.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p]
        L.ora_poisson_residual.restype = ct.c_double
        L.ora_poisson_residual.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                                           ct.POINTER(ct.c_double)]
        L.ora_poisson_solve.restype = ct.c_int
        L.ora_poisson_solve.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int,
                                        ct.c_double, ct.c_double, ct.c_int, ct.POINTER(ct.c_double),
                                        ct.POINTER(ct.c_double)]
        L.ora_poisson_stats.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_void_p]
        _lib = L
    return _lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ct.POINTER(ct.c_double))


def nq(lattice: int = 0) -> int:
    """Number of lattice directions: 19 (D3Q19, lattice 0) or 9 (D2Q9, lattice 1)."""
    return 9 if lattice == 1 else 19


def lattice(lat: int = 0):
    q = nq(lat)
    c = np.zeros((q, 3), dtype=np.int32)
    w = np.zeros(q)
    assert lib().ora_lattice_q(int(lat), c.ctypes.data, w.ctypes.data) == q
    return c, w


def feq(rho: float, u, lat: int = 0) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros(nq(lat))
    lib().ora_feq_lat(int(lat), rho, _dptr(u), _dptr(out))
    return out


def alpha(f, fe, u, rho, alpha0=2.0, rtol=1e-12, maxit=30, lat: int = 0):
    f = np.ascontiguousarray(f, dtype=np.float64)
    fe = np.ascontiguousarray(fe, dtype=np.float64)
    it = ct.c_int(0)
    a = lib().ora_alpha_lat(int(lat), _dptr(f), _dptr(fe), rho, alpha0, rtol, maxit, ct.byref(it))
    return a, it.value


def sym3_norm2(m6) -> float:
    m6 = np.ascontiguousarray(m6, dtype=np.float64)
    return lib().ora_sym3_norm2(_dptr(m6))


def carreau_nu(gd, nu0, nu_inf, lam, n):
    return lib().ora_carreau_nu(gd, nu0, nu_inf, lam, n)


def shear_rate(Pn, rho, alpha, nu0, nu_inf, lam, n):
    return lib().ora_shear_rate(Pn, rho, alpha, nu0, nu_inf, lam, n)


def make_params(p, box, nthreads: int = 0) -> OraParams:
    """Oracle parameter struct from an inputs.Params and an inputs.Box (plus box overrides)."""
    P = OraParams()
    P.nx, P.ny, P.nz, P.ncomp = box.nx, box.ny, box.nz, p.ncomp
    for a in range(3):
        P.periodic[a] = int(box.periodic[a])
    P.carreau, P.curvature, P.electrostriction = int(p.carreau), int(p.curvature), int(p.electrostriction)
    P.charge_model = int(p.charge_model)
    P.sor_sweeps, P.newton_max, P.nthreads = int(p.sor_sweeps), int(p.newton_max), int(nthreads)
    gw = p.G if p.Gw is None else p.Gw  # None: a neutral wall, G_w = G
    for s in range(2):
        for t in range(2):
            P.G[s][t] = float(p.G[s][t]) if s < len(p.G) and t < len(p.G[s]) else 0.0
            P.Gw[s][t] = float(gw[s][t]) if s < len(gw) and t < len(gw[s]) else 0.0
    info = box.info
    P.nu0, P.nu_inf, P.lam = p.nu0, p.nu_inf, p.lam
    P.n_flow = float(info.get("n_flow", p.n_flow))
    P.Q_b = float(info.get("Q_b", p.Q_b))
    P.Q_s = float(info.get("Q_s", p.Q_s))
    P.xi_b, P.xi_s, P.K_d, P.rho_th, P.w_theta = p.xi_b, p.xi_s, p.K_d, p.rho_th, p.w_theta
    E = info.get("E_ext", p.E_ext)
    for a in range(3):
        P.E_ext[a] = float(E[a])
    P.sor_omega = float(info.get("sor_omega", p.sor_omega))
    P.newton_rtol = p.newton_rtol
    P.sor_tol = float(getattr(p, "sor_tol", 0.0))
    P.sor_check_every = int(getattr(p, "sor_check_every", 0))
    P.lattice = int(getattr(p, "lattice", 0))
    P.inlet_mode = int(getattr(p, "inlet_mode", 0))
    for s in range(2):
        P.rho_in[s] = p.rho_in[s]
        P.rho_out[s] = p.rho_out[s]
    return P


class Oracle:
    """One box advanced by the oracle."""

    def __init__(self, params, box, nthreads: int = 0):
        self.p, self.box = params, box
        self.C = params.ncomp
        self.Q = nq(int(getattr(params, "lattice", 0)))
        self.N = box.n
        self.shape = (box.nz, box.ny, box.nx)
        self._P = make_params(params, box, nthreads)
        L = lib()
        self._t = np.ascontiguousarray(box.node_type.reshape(-1), dtype=np.uint8)
        self._phi0 = np.ascontiguousarray(box.phi0.reshape(-1), dtype=np.float64)
        self._ubc = np.ascontiguousarray(box.u_bc.reshape(3, -1), dtype=np.float64)
        self.h = L.ora_create(ct.byref(self._P), self._t.ctypes.data, self._phi0.ctypes.data,
                              self._ubc.ctypes.data)
        rho0 = np.ascontiguousarray(box.rho0.reshape(self.C, -1), dtype=np.float64)
        u0 = np.ascontiguousarray(box.u0.reshape(3, -1), dtype=np.float64)
        xi = np.ascontiguousarray(box.xi.reshape(self.C, self.Q, -1), dtype=np.float64)
        L.ora_init(self.h, rho0.ctypes.data, u0.ctypes.data, xi.ctypes.data, float(box.jitter))

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().ora_destroy(h)
            self.h = None

    def step(self, n: int = 1):
        lib().ora_step(self.h, int(n))

    _COUNTS = {F_RHO: "C", F_J: "C3", F_PSI: "C", F_GRAD: "3", F_NHAT: "3", F_K: "1", F_BULK: "1",
               F_SURF: "1", F_Q: "1", F_PHI: "1", F_RHS: "1", F_E: "3", F_E2: "1", F_FEL: "3",
               F_F: "C3", F_ALPHA: "C", F_NU: "C", F_UPH: "3", F_POP: "CQ", F_PULLED: "CQ"}

    def field(self, which: int) -> np.ndarray:
        kind = self._COUNTS[which]
        lead = {"C": (self.C,), "C3": (self.C, 3), "3": (3,), "1": (), "CQ": (self.C, self.Q)}[kind]
        out = np.zeros(lead + self.shape)
        lib().ora_field(self.h, which, out.ctypes.data)
        return out

    def iters(self) -> np.ndarray:
        out = np.zeros((self.C,) + self.shape, dtype=np.int32)
        lib().ora_iters(self.h, out.ctypes.data)
        return out

    def counters(self):
        i = np.zeros(3, dtype=np.int64)
        d = np.zeros(3)
        lib().ora_counters(self.h, i.ctypes.data, d.ctypes.data)
        return dict(fallbacks=int(i[0]), nonfinite=int(i[1]), negative=int(i[2]),
                    S_b=float(d[0]), S_s=float(d[1]), qbar=float(d[2]))

    def set_populations(self, f: np.ndarray):
        f = np.ascontiguousarray(f, dtype=np.float64)
        lib().ora_set_populations(self.h, f.ctypes.data)

    def set_phi(self, phi: np.ndarray):
        phi = np.ascontiguousarray(phi, dtype=np.float64)
        lib().ora_set_phi(self.h, phi.ctypes.data)

    def inlet_ubar(self) -> float:
        """Mean velocity inside the nozzle measured in the last step (the
        adaptive inlet, Sec. III.B); 0 without it."""
        return float(lib().ora_inlet_ubar(self.h))

    def poisson_stats(self):
        """Residual, its scale max|rhs|, sweeps done of the last step's Poisson
        solve, and the number of steps whose solve missed the tolerance."""
        d = np.zeros(2)
        i = np.zeros(2, dtype=np.int64)
        lib().ora_poisson_stats(self.h, d.ctypes.data, i.ctypes.data)
        return dict(residual=float(d[0]), scale=float(d[1]), sweeps=int(i[0]), noconv=int(i[1]))

    def poisson_rhs(self, eps, q):
        """The step's Poisson right-hand side for given eps and q: (rhs, qbar)."""
        eps = np.ascontiguousarray(eps, dtype=np.float64)
        q = np.ascontiguousarray(q, dtype=np.float64)
        rhs = np.zeros(self.shape)
        qbar = lib().ora_poisson_rhs(self.h, eps.ctypes.data, q.ctypes.data, rhs.ctypes.data)
        return rhs, qbar

    def poisson_residual(self, eps, rhs, phi):
        """(max residual over unknown nodes, max|rhs| over the same nodes)."""
        eps = np.ascontiguousarray(eps, dtype=np.float64)
        rhs = np.ascontiguousarray(rhs, dtype=np.float64)
        phi = np.ascontiguousarray(phi, dtype=np.float64)
        sc = ct.c_double()
        r = lib().ora_poisson_residual(self.h, eps.ctypes.data, rhs.ctypes.data, phi.ctypes.data, ct.byref(sc))
        return r, sc.value

    def poisson_solve(self, eps, rhs, phi, sweeps, omega, tol=0.0, check_every=0):
        """The step's stopping SOR on given eps/rhs, phi updated in place:
        (sweeps done, residual, scale)."""
        eps = np.ascontiguousarray(eps, dtype=np.float64)
        rhs = np.ascontiguousarray(rhs, dtype=np.float64)
        assert phi.flags.c_contiguous and phi.dtype == np.float64
        r, sc = ct.c_double(), ct.c_double()
        n = lib().ora_poisson_solve(self.h, eps.ctypes.data, rhs.ctypes.data, phi.ctypes.data, int(sweeps),
                                    float(omega), float(tol), int(check_every), ct.byref(r), ct.byref(sc))
        return n, r.value, sc.value

    def poisson(self, eps, rhs, phi, sweeps, omega):
        """Run the oracle's red-black SOR on given eps/rhs, updating phi in place."""
        eps = np.ascontiguousarray(eps, dtype=np.float64)
        rhs = np.ascontiguousarray(rhs, dtype=np.float64)
        assert phi.flags.c_contiguous and phi.dtype == np.float64
        lib().ora_poisson(self.h, eps.ctypes.data, rhs.ctypes.data, phi.ctypes.data, int(sweeps),
                          float(omega))
