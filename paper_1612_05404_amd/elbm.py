"""Thin ctypes binding of libelbm.so (declared in include/elbm.h).

Argument marshalling only: every step of the update runs in the HIP
kernels of the library.  PyTorch supplies the device arena and the stream.
The binding refuses to run without the built library -- there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as ct
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libelbm.so")

ELBM_OK, ELBM_EINVAL, ELBM_ENOMEM, ELBM_EHIP, ELBM_ENONFINITE, ELBM_ESTATE = 0, -1, -2, -3, -4, -7
ELBM_ENEGPOP, ELBM_ENOCONV = -5, -6
STRICT_NEGPOP, STRICT_ALPHA = 1, 2
STORAGE_F64, STORAGE_F32, STORAGE_F32_ALL = 0, 1, 2
# dtype names: "f64" all FP64; "f32" FP32 populations + FP64 fields; "f32all" all FP32
STORAGE = {"f64": STORAGE_F64, "f32": STORAGE_F32, "f32all": STORAGE_F32_ALL}
# initial guess of the alpha Newton iteration (every guess is polished to the same rule)
GUESS = {"standard": 0, "mlp": 1, "series": 2}
# the alpha iteration (same stopping rule): Newton, or Halley with g''
ITER = {"newton": 0, "halley": 1}
# inlet nodes: neighbour-density velocity inlet, or the adaptive jet inlet along x / y / z
INLET_NEIGHBOUR, INLET_ADAPTIVE_X, INLET_ADAPTIVE_Y, INLET_ADAPTIVE_Z = 0, 1, 2, 3
Q = 19


class ElbmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"elbm status {status}: {msg}")
        self.status = status


class elbm_params(ct.Structure):
    _fields_ = [
        ("ncomp", ct.c_int32), ("storage", ct.c_int32), ("carreau", ct.c_int32), ("curvature", ct.c_int32),
        ("electrostriction", ct.c_int32), ("charge_model", ct.c_int32), ("sor_sweeps", ct.c_int32),
        ("newton_max", ct.c_int32), ("alpha_guess", ct.c_int32), ("strict", ct.c_int32),
        ("G", (ct.c_double * 2) * 2), ("Gw", (ct.c_double * 2) * 2),
        ("nu0", ct.c_double), ("nu_inf", ct.c_double), ("lam", ct.c_double), ("K_d", ct.c_double),
        ("rho_th", ct.c_double), ("w_theta", ct.c_double), ("xi_b", ct.c_double), ("xi_s", ct.c_double),
        ("newton_rtol", ct.c_double), ("rho_in", ct.c_double * 2), ("rho_out", ct.c_double * 2),
        ("sor_tol", ct.c_double), ("sor_check_every", ct.c_int32), ("alpha_iter", ct.c_int32),
        ("lattice", ct.c_int32), ("inlet_mode", ct.c_int32),
    ]


class elbm_box(ct.Structure):
    _fields_ = [
        ("nx", ct.c_int32), ("ny", ct.c_int32), ("nz", ct.c_int32), ("periodic", ct.c_int32 * 3),
        ("E_ext", ct.c_double * 3), ("Q_b", ct.c_double), ("Q_s", ct.c_double),
        ("n_flow", ct.c_double), ("sor_omega", ct.c_double),
    ]


class elbm_launch(ct.Structure):
    _fields_ = [("xcd_remap", ct.c_int32), ("graph_steps", ct.c_int32), ("tile", ct.c_int32),
                ("sweep_priority", ct.c_int32), ("stencil_lds", ct.c_int32)]


class elbm_diag(ct.Structure):
    _fields_ = [
        ("mass", ct.c_double * 2), ("momentum", ct.c_double * 3),
        ("alpha_min", ct.c_double), ("alpha_max", ct.c_double), ("alpha_mean", ct.c_double),
        ("mean_newton_iters", ct.c_double), ("n_fallback", ct.c_int64), ("n_negative", ct.c_int64),
        ("n_collisions", ct.c_int64), ("sum_Fel", ct.c_double * 3), ("sor_residual", ct.c_double),
        ("sor_scale", ct.c_double), ("sor_sweeps", ct.c_int32), ("pad_", ct.c_int32),
        ("n_sor_noconv", ct.c_int64), ("inlet_ubar", ct.c_double),
    ]


# every symbol include/elbm.h declares
SYMBOLS = [
    "elbm_abi_version", "elbm_create", "elbm_required_bytes", "elbm_bind", "elbm_set_box", "elbm_step",
    "elbm_sync", "elbm_read_moments", "elbm_read_potential", "elbm_read_charge", "elbm_read_alpha",
    "elbm_get_populations", "elbm_set_populations", "elbm_set_potential", "elbm_diagnostics",
    "elbm_set_graphs", "elbm_set_timing", "elbm_timing", "elbm_mlp_set_weights", "elbm_mlp_get_weights",
    "elbm_mlp_forward", "elbm_mlp_grad", "elbm_mlp_grad_noalloc", "elbm_mlp_train", "elbm_alpha_samples", "elbm_set_launch",
    "elbm_get_launch", "elbm_autotune", "elbm_last_error", "elbm_destroy",
]
TUNE_CANDIDATES = 11
TILES = {0: "linear", 1: "8x8x4", 2: "8x4x8", 3: "4x4x16"}
PHASES = ["density", "charge", "poisson", "efield", "alpha", "collide"]

_lib = None
ABI_VERSION = 7  # include/elbm.h ELBM_ABI_VERSION


def load(path: str = LIB_PATH):
    """Loads libelbm.so and declares its signatures; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    # the HIP runtime comes up through torch first: the library's calls then
    # share the process's device view (loading the library first left its
    # runtime without a device on the MI355X machine)
    import torch  # noqa: F401
    if not os.path.exists(path):
        raise ImportError(f"libelbm.so not built at {path}; run __graft_entry__.build()")
    L = ct.CDLL(path)
    vp, i32, dp = ct.c_void_p, ct.c_int32, ct.POINTER(ct.c_double)
    L.elbm_abi_version.restype = ct.c_uint32
    L.elbm_abi_version.argtypes = []
    if L.elbm_abi_version() != ABI_VERSION:
        raise ImportError(f"{path} has ABI version {L.elbm_abi_version()}, this binding needs {ABI_VERSION}; "
                          "rebuild with __graft_entry__.build()")
    L.elbm_create.argtypes = [ct.POINTER(elbm_params), ct.POINTER(elbm_box), i32, ct.POINTER(vp)]
    L.elbm_required_bytes.argtypes = [vp, ct.POINTER(ct.c_size_t)]
    L.elbm_bind.argtypes = [vp, vp, ct.c_size_t, vp]
    L.elbm_set_box.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, ct.c_double]
    L.elbm_step.argtypes = [vp, i32, i32]
    L.elbm_sync.argtypes = [vp]
    L.elbm_read_moments.argtypes = [vp, i32, vp, vp]
    L.elbm_read_potential.argtypes = [vp, i32, vp]
    L.elbm_read_charge.argtypes = [vp, i32, vp]
    L.elbm_read_alpha.argtypes = [vp, i32, vp, vp]
    L.elbm_get_populations.argtypes = [vp, i32, vp]
    L.elbm_set_populations.argtypes = [vp, i32, vp]
    L.elbm_set_potential.argtypes = [vp, i32, vp]
    L.elbm_diagnostics.argtypes = [vp, i32, ct.POINTER(elbm_diag)]
    L.elbm_set_graphs.argtypes = [vp, i32]
    i64, fp = ct.c_int64, ct.POINTER(ct.c_float)
    L.elbm_mlp_set_weights.argtypes = [vp, vp, i64]
    L.elbm_mlp_get_weights.argtypes = [vp, vp, i64]
    L.elbm_mlp_forward.argtypes = [vp, vp, vp, i64]
    L.elbm_mlp_grad.argtypes = [vp, vp, vp, i64, vp, vp]
    L.elbm_mlp_grad_noalloc.argtypes = [vp, vp, vp, i64, vp]
    L.elbm_mlp_train.argtypes = [vp, vp, vp, i64, i32, i32, ct.c_float, vp]
    L.elbm_alpha_samples.argtypes = [vp, i32, vp, vp, vp, vp]
    L.elbm_set_launch.argtypes = [vp, ct.POINTER(elbm_launch)]
    L.elbm_get_launch.argtypes = [vp, ct.POINTER(elbm_launch)]
    L.elbm_autotune.argtypes = [vp, i32, ct.POINTER(elbm_launch), vp]
    L.elbm_set_timing.argtypes = [vp, i32]
    L.elbm_timing.argtypes = [vp, vp, vp]
    L.elbm_last_error.restype = ct.c_char_p
    L.elbm_last_error.argtypes = [vp]
    L.elbm_destroy.restype = None
    L.elbm_destroy.argtypes = [vp]
    for name in SYMBOLS:
        fn = getattr(L, name)
        if name not in ("elbm_abi_version", "elbm_last_error", "elbm_destroy"):
            fn.restype = ct.c_int
    _lib = L
    return L


def make_params(p, storage: int, guess: int = 0, alpha_iter: int = 0, strict: int = 0) -> elbm_params:
    P = elbm_params()
    P.ncomp, P.storage = int(p.ncomp), int(storage)
    P.carreau, P.curvature, P.electrostriction = int(p.carreau), int(p.curvature), int(p.electrostriction)
    P.charge_model, P.sor_sweeps, P.newton_max = int(p.charge_model), int(p.sor_sweeps), int(p.newton_max)
    P.alpha_guess = int(guess)
    P.alpha_iter = int(alpha_iter)
    P.strict = int(strict)
    P.sor_tol = float(getattr(p, "sor_tol", 0.0))
    P.sor_check_every = int(getattr(p, "sor_check_every", 0))
    P.lattice = int(getattr(p, "lattice", 0))
    P.inlet_mode = int(getattr(p, "inlet_mode", 0))
    gw = p.G if p.Gw is None else p.Gw
    for s in range(2):
        for t in range(2):
            P.G[s][t] = float(p.G[s][t]) if s < len(p.G) and t < len(p.G[s]) else 0.0
            P.Gw[s][t] = float(gw[s][t]) if s < len(gw) and t < len(gw[s]) else 0.0
    P.nu0, P.nu_inf, P.lam, P.K_d = p.nu0, p.nu_inf, p.lam, p.K_d
    P.rho_th, P.w_theta, P.xi_b, P.xi_s, P.newton_rtol = p.rho_th, p.w_theta, p.xi_b, p.xi_s, p.newton_rtol
    for s in range(2):
        P.rho_in[s], P.rho_out[s] = p.rho_in[s], p.rho_out[s]
    return P


def make_box(p, box) -> elbm_box:
    B = elbm_box()
    B.nx, B.ny, B.nz = box.nx, box.ny, box.nz
    for a in range(3):
        B.periodic[a] = int(box.periodic[a])
    info = box.info
    E = info.get("E_ext", p.E_ext)
    for a in range(3):
        B.E_ext[a] = float(E[a])
    B.Q_b = float(info.get("Q_b", p.Q_b))
    B.Q_s = float(info.get("Q_s", p.Q_s))
    B.n_flow = float(info.get("n_flow", p.n_flow))
    B.sor_omega = float(info.get("sor_omega", p.sor_omega))
    return B


def _c(a, dtype=np.float64):
    return None if a is None else np.ascontiguousarray(a, dtype=dtype)


class Lattice:
    """Boxes of one parameter set advanced by the HIP library on one GPU.

    ``params`` is an inputs.Params, ``boxes`` a list of inputs.Box,
    ``dtype`` "f64" (FP64 populations and fields), "f32" (FP32 populations,
    FP64 fields) or "f32all" (FP32 populations and fields); the entropic
    alpha is FP64 in every mode."""

    def __init__(self, params, boxes: Sequence, dtype: str = "f64", device: str = "cuda:0",
                 stream=None, alpha_guess: str = "standard", alpha_iter: str = "newton", strict: int = 0):
        import torch
        self.L = load()
        self.params = params
        self.boxes = list(boxes)
        self.C = params.ncomp
        self.Q = 9 if int(getattr(params, "lattice", 0)) == 1 else 19
        if dtype not in STORAGE:
            raise ValueError(f"dtype must be one of {sorted(STORAGE)}")
        storage = STORAGE[dtype]
        if alpha_guess not in GUESS:
            raise ValueError(f"alpha_guess must be one of {sorted(GUESS)}")
        if alpha_iter not in ITER:
            raise ValueError(f"alpha_iter must be one of {sorted(ITER)}")
        self._P = make_params(params, storage, GUESS[alpha_guess], ITER[alpha_iter], strict)
        self._B = (elbm_box * len(self.boxes))(*[make_box(params, b) for b in self.boxes])
        h = ct.c_void_p()
        self._check(self.L.elbm_create(ct.byref(self._P), self._B, len(self.boxes), ct.byref(h)), None)
        self.h = h
        nbytes = ct.c_size_t()
        self._check(self.L.elbm_required_bytes(self.h, ct.byref(nbytes)))
        self.nbytes = nbytes.value
        self.device = torch.device(device)
        self.arena = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=self.device)
        ptr = self.arena.data_ptr()
        aligned = (ptr + 255) & ~255
        # a stream of its own (default priority): the step graphs cannot be
        # captured on the null stream
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        self.arena.record_stream(self.stream)
        self._check(self.L.elbm_bind(self.h, ct.c_void_p(aligned), self.nbytes, ct.c_void_p(self.stream.cuda_stream)))
        for i, b in enumerate(self.boxes):
            self.set_box(i, b)

    # ------------------------------------------------------------------
    def _check(self, status: int, h=-1):
        if status != ELBM_OK:
            hh = self.h if h == -1 else h
            msg = self.L.elbm_last_error(hh).decode() if hh else ""
            raise ElbmError(status, msg)

    def close(self):
        if getattr(self, "h", None):
            self.L.elbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_box(self, i: int, box):
        t = _c(box.node_type.reshape(-1), np.uint8)
        rho = _c(box.rho0.reshape(self.C, -1))
        u = _c(box.u0.reshape(3, -1))
        phi = _c(box.phi0.reshape(-1))
        ubc = _c(box.u_bc.reshape(3, -1))
        xi = _c(box.xi.reshape(self.C, self.Q, -1)) if box.xi is not None else None
        self._keep = (t, rho, u, phi, ubc, xi)
        self._check(self.L.elbm_set_box(self.h, i, t.ctypes.data, rho.ctypes.data, u.ctypes.data,
                                        phi.ctypes.data, ubc.ctypes.data,
                                        xi.ctypes.data if xi is not None else None, float(box.jitter)))

    def step(self, n: int = 1, record: bool = True):
        self._check(self.L.elbm_step(self.h, int(n), int(bool(record))))

    def sync(self):
        self._check(self.L.elbm_sync(self.h))

    def _shape(self, i):
        b = self.boxes[i]
        return (b.nz, b.ny, b.nx)

    def read_moments(self, i: int = 0):
        sh = self._shape(i)
        rho = np.zeros((self.C,) + sh)
        u = np.zeros((3,) + sh)
        self._check(self.L.elbm_read_moments(self.h, i, rho.ctypes.data, u.ctypes.data))
        return rho, u

    def read_potential(self, i: int = 0):
        phi = np.zeros(self._shape(i))
        self._check(self.L.elbm_read_potential(self.h, i, phi.ctypes.data))
        return phi

    def read_charge(self, i: int = 0):
        q = np.zeros(self._shape(i))
        self._check(self.L.elbm_read_charge(self.h, i, q.ctypes.data))
        return q

    def read_alpha(self, i: int = 0):
        sh = (self.C,) + self._shape(i)
        al = np.zeros(sh)
        it = np.zeros(sh, dtype=np.int32)
        self._check(self.L.elbm_read_alpha(self.h, i, al.ctypes.data, it.ctypes.data))
        return al, it

    def get_populations(self, i: int = 0):
        f = np.zeros((self.C, self.Q) + self._shape(i))
        self._check(self.L.elbm_get_populations(self.h, i, f.ctypes.data))
        return f

    def set_populations(self, i: int, f):
        f = _c(f)
        self._check(self.L.elbm_set_populations(self.h, i, f.ctypes.data))

    def set_potential(self, i: int, phi):
        phi = _c(phi)
        self._check(self.L.elbm_set_potential(self.h, i, phi.ctypes.data))

    def diagnostics(self, i: int = 0) -> dict:
        d = elbm_diag()
        self._check(self.L.elbm_diagnostics(self.h, i, ct.byref(d)))
        return dict(mass=list(d.mass), momentum=list(d.momentum), alpha_min=d.alpha_min,
                    alpha_max=d.alpha_max, alpha_mean=d.alpha_mean, mean_newton_iters=d.mean_newton_iters,
                    n_fallback=d.n_fallback, n_negative=d.n_negative, n_collisions=d.n_collisions,
                    sum_Fel=list(d.sum_Fel), sor_residual=d.sor_residual, sor_scale=d.sor_scale,
                    sor_sweeps=d.sor_sweeps, n_sor_noconv=d.n_sor_noconv, inlet_ubar=d.inlet_ubar)

    def set_graphs(self, enable: bool = True):
        self._check(self.L.elbm_set_graphs(self.h, int(bool(enable))))

    def set_timing(self, enable: bool = True):
        self._check(self.L.elbm_set_timing(self.h, int(bool(enable))))

    def timing(self) -> dict:
        """Accumulated device ms per phase and the timed step count (then reset)."""
        ms = np.zeros(len(PHASES))
        n = ct.c_int64()
        self._check(self.L.elbm_timing(self.h, ms.ctypes.data, ct.byref(n)))
        return dict(steps=n.value, **{k: float(v) for k, v in zip(PHASES, ms)})

    # ---------------------------------------------------- learned starter
    MLP_NPARAM = 1761
    MLP_IN = 20

    def mlp_set_weights(self, w):
        w = np.ascontiguousarray(w, dtype=np.float32)
        self._check(self.L.elbm_mlp_set_weights(self.h, w.ctypes.data, w.size))

    def mlp_get_weights(self):
        w = np.zeros(self.MLP_NPARAM, dtype=np.float32)
        self._check(self.L.elbm_mlp_get_weights(self.h, w.ctypes.data, w.size))
        return w

    def mlp_forward(self, X):
        """X: float32 device tensor [M, 20] -> float32 device tensor [M]."""
        import torch
        X = X.contiguous()
        Y = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
        self.stream.wait_stream(torch.cuda.current_stream(X.device))
        self._check(self.L.elbm_mlp_forward(self.h, ct.c_void_p(X.data_ptr()), ct.c_void_p(Y.data_ptr()),
                                            X.shape[0]))
        self.sync()
        return Y

    def mlp_grad(self, X, T):
        """Gradient (FP32, parameter order) and loss of 1/(2M) sum (y - T)^2."""
        import torch
        X, T = X.contiguous(), T.contiguous()
        g = np.zeros(self.MLP_NPARAM, dtype=np.float32)
        loss = ct.c_float()
        self.stream.wait_stream(torch.cuda.current_stream(X.device))
        self._check(self.L.elbm_mlp_grad(self.h, ct.c_void_p(X.data_ptr()), ct.c_void_p(T.data_ptr()), X.shape[0],
                                         g.ctypes.data, ct.byref(loss)))
        return g, loss.value

    def mlp_grad_noalloc(self, X, T, G):
        """The gradient and loss into the device tensor G (float32 [1762]),
        enqueued on the library's stream with no allocation and no
        synchronisation (the library's allocation-free entry point)."""
        import torch
        X, T = X.contiguous(), T.contiguous()
        assert G.dtype == torch.float32 and G.numel() == self.MLP_NPARAM + 1 and G.is_contiguous()
        self.stream.wait_stream(torch.cuda.current_stream(X.device))
        self._check(self.L.elbm_mlp_grad_noalloc(self.h, ct.c_void_p(X.data_ptr()), ct.c_void_p(T.data_ptr()),
                                                 X.shape[0], ct.c_void_p(G.data_ptr())))

    def mlp_train(self, X, T, batch: int, steps: int, lr: float):
        """Adam steps over consecutive batches of (X, T); returns the batch losses."""
        import torch
        X, T = X.contiguous(), T.contiguous()
        self.stream.wait_stream(torch.cuda.current_stream(X.device))
        losses = np.zeros(max(steps, 1), dtype=np.float32)
        done = 0
        while done < steps:
            n = min(4096, steps - done)
            buf = np.zeros(n, dtype=np.float32)
            self._check(self.L.elbm_mlp_train(self.h, ct.c_void_p(X.data_ptr()), ct.c_void_p(T.data_ptr()),
                                              X.shape[0], int(batch), n, float(lr), buf.ctypes.data))
            losses[done:done + n] = buf
            done += n
        return losses[:steps]

    def alpha_samples(self, i: int = 0):
        """Starter inputs (z, s) [C*N, 20], targets (alpha* - 2)/s [C*N],
        scales s [C*N] and flags [C*N] (0 invalid, 1 valid, 2 valid and served
        by the learned starter) of the current state of box i (device tensors)."""
        import torch
        b = self.boxes[i]
        m = self.C * b.n
        feat = torch.empty((m, self.MLP_IN), dtype=torch.float32, device=self.device)
        tgt = torch.empty(m, dtype=torch.float32, device=self.device)
        scl = torch.empty(m, dtype=torch.float32, device=self.device)
        val = torch.empty(m, dtype=torch.int32, device=self.device)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        self._check(self.L.elbm_alpha_samples(self.h, i, ct.c_void_p(feat.data_ptr()), ct.c_void_p(tgt.data_ptr()),
                                              ct.c_void_p(scl.data_ptr()), ct.c_void_p(val.data_ptr())))
        return feat, tgt, scl, val

    # ---------------------------------------------------- launch mapping
    def set_launch(self, xcd_remap: int, graph_steps: int, tile: int = 0, sweep_priority: int = 0,
                   stencil_lds: int = 0):
        l = elbm_launch(int(xcd_remap), int(graph_steps), int(tile), int(sweep_priority), int(stencil_lds))
        self._check(self.L.elbm_set_launch(self.h, ct.byref(l)))

    @staticmethod
    def _launch_dict(l) -> dict:
        return {"xcd_remap": l.xcd_remap, "graph_steps": l.graph_steps, "tile": l.tile,
                "sweep_priority": l.sweep_priority, "stencil_lds": l.stencil_lds}

    def get_launch(self) -> dict:
        l = elbm_launch()
        self._check(self.L.elbm_get_launch(self.h, ct.byref(l)))
        return self._launch_dict(l)

    def autotune(self, steps_per_trial: int = 32):
        """Chooses the launch mapping in four timed passes (collision tile
        0..3, then XCD order 0, 1, then field-chain priority 0, 1, then
        graph length 2, 4, 8); returns it and each candidate's ms per step in
        that order.  The trial steps advance the state like ordinary steps
        (22 trials + 60 in all)."""
        import torch
        best = elbm_launch()
        ms = np.zeros(TUNE_CANDIDATES)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        self._check(self.L.elbm_autotune(self.h, int(steps_per_trial), ct.byref(best), ms.ctypes.data))
        return self._launch_dict(best), ms
