"""HIP path vs the CPU oracle, element by element on the same seeded inputs.

Error metric per field X: max_r |X_gpu - X_oracle| / max_r |X_oracle|
(field-max normalisation: point-wise relative error of near-zero velocities
is ill-conditioned).  Bars: 1e-12 with FP64 storage, 1e-5 on densities,
velocity and potential with FP32 storage after 100 steps.
"""
import os
import sys

import numpy as np
import pytest

from paper_1612_05404_amd import inputs

pytestmark = pytest.mark.gpu

NTHREADS = min(16, os.cpu_count() or 1)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def elbm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1612_05404_amd import elbm as E
    E.load()
    return E


def rel(a, b):
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / den) if den > 0 else float(np.abs(a - b).max())


def compare(lat, i, o, tol, fields=("rhoA", "rhoB", "ux", "uy", "uz", "phi", "q"), report=None):
    import oracle as ora
    rho, u = lat.read_moments(i)
    phi = lat.read_potential(i)
    q = lat.read_charge(i)
    orho, ou = o.field(ora.F_RHO), o.field(ora.F_UPH)
    got = {"rhoA": (rho[0], orho[0]), "ux": (u[0], ou[0]), "uy": (u[1], ou[1]), "uz": (u[2], ou[2]),
           "phi": (phi, o.field(ora.F_PHI)), "q": (q, o.field(ora.F_Q))}
    if rho.shape[0] > 1:
        got["rhoB"] = (rho[1], orho[1])
    errs = {k: rel(*got[k]) for k in fields if k in got}
    if report is not None:
        report.update(errs)
    _say(f"    field errors: " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, bad
    return errs


def alpha_conditioning(fp, lat_id=0):
    """Rounding allowance of alpha at each node from the conditioning of the
    entropy balance (Eqs. entropic, H) in the populations themselves: alpha
    depends on Delta = f_eq(f) - f, formed by cancellation, so a relative
    change of eps in each f_p moves Delta_p by eps / |x_p| relative
    (x = Delta / f) and alpha by about eps / x_rms, x_rms^2 = sum_p f_p x_p^2 /
    sum_p f_p: near equilibrium (x_rms ~ 1e-5) two correct solvers differ in
    the 11th digit.  Measured with the oracle's own solver under random 1-ulp
    changes of f on the 2-D jet: at most 24 eps / x_rms; the allowance is
    64 eps / x_rms (at most 1e-6).  fp: pulled populations [C][Q][...] of the step that
    solved for alpha; returns [C][...]."""
    import oracle as ora
    c, w = ora.lattice(lat_id)
    C, Q = fp.shape[0], fp.shape[1]
    f = fp.reshape(C, Q, -1)
    out = np.zeros((C, f.shape[2]))
    for s in range(C):
        fs = f[s]
        rho = fs.sum(axis=0)
        ok = rho > 0
        with np.errstate(all="ignore"):
            u = np.einsum("pa,pn->an", c.astype(np.float64), fs) / np.where(ok, rho, 1.0)
            cu = np.einsum("pa,an->pn", c.astype(np.float64), u)
            uu = (u * u).sum(axis=0)
            feq = w[:, None] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu)
            x = (feq - fs) / fs
            xrms = np.sqrt((fs * x * x).sum(axis=0) / rho)
            allow = np.minimum(64.0 * 2.220446049250313e-16 / xrms, 1e-6)
        out[s] = np.where(ok & np.isfinite(allow), allow, 0.0)
    return out.reshape((C,) + fp.shape[2:])


def check_alpha(al, it, oal, oit, tol=1e-11, label="alpha", allowance=None):
    """Alpha of two solvers on the same states: the same fallback nodes, and
    the largest relative difference over every node both solved within tol
    (plus, where given, a per-node allowance from the conditioning of the
    entropy balance, alpha_conditioning)."""
    fb, ofb = it < 0, oit < 0
    both = (it >= 0) & (oit >= 0) & (oal > 0)
    err = np.abs(al - oal)[both] / oal[both]
    emax = float(err.max()) if err.size else 0.0
    bar = tol + (allowance[both] if allowance is not None else 0.0)
    worst = float((err / bar).max()) if err.size else 0.0
    _say(f"    {label}: max rel err {emax:.2e} over {int(both.sum())} solves; fallbacks {int(fb.sum())} / "
         f"{int(ofb.sum())}; update counts equal {np.mean(it == oit):.4f}"
         + (f"; largest error over its bar {worst:.3f}" if allowance is not None else ""))
    assert np.array_equal(fb, ofb), "fallback nodes differ"
    assert worst <= 1.0 if allowance is not None else emax <= tol, emax
    return emax


def run_both(elbm, params, boxes, dtype, steps, name, launch=None, guess=None):
    import oracle as ora
    _say(f"[gpu parity] {name}: dtype={dtype} steps={steps} boxes={[(b.nx, b.ny, b.nz) for b in boxes]}"
         f" launch={launch} guess={guess}")
    lat = elbm.Lattice(params, boxes, dtype) if guess is None else elbm.Lattice(params, boxes, dtype, alpha_guess=guess)
    if launch is not None:
        lat.set_launch(*launch)
    lat.step(steps, record=True)
    lat.sync()
    oras = []
    for b in boxes:
        o = ora.Oracle(params, b, nthreads=NTHREADS)
        o.step(steps)
        oras.append(o)
    return lat, oras


def test_drop32_fp64_parity_100_steps(elbm):
    # Plain-method workload at full size: 32^3 periodic drop, FP64, 100 steps.
    wl = inputs.drop32()
    lat, (o,) = run_both(elbm, wl.params, wl.boxes, "f64", 100, "drop32")
    compare(lat, 0, o, 1e-12)
    import oracle as ora
    al, it = lat.read_alpha(0)
    check_alpha(al, it, o.field(ora.F_ALPHA), o.iters())
    assert np.mean(it == o.iters()) > 0.99
    d = lat.diagnostics(0)
    _say(f"    diag {d}")


def test_series_starter_same_alpha_fewer_iterations(elbm):
    # The series starter changes only where Newton starts: fields match the
    # oracle at the FP64 bar, alpha matches the plain solver's, and the mean
    # number of Newton updates drops.
    import oracle as ora
    wl = inputs.drop32()
    _say("[gpu parity] drop32 with the series starter: f64, 100 steps")
    plain = elbm.Lattice(wl.params, wl.boxes, "f64")
    ser = elbm.Lattice(wl.params, wl.boxes, "f64", alpha_guess="series")
    plain.step(100, record=True)
    ser.step(100, record=True)
    o = ora.Oracle(wl.params, wl.boxes[0], nthreads=NTHREADS)
    o.step(100)
    compare(ser, 0, o, 1e-12)
    a0, i0 = plain.read_alpha(0)
    a1, i1 = ser.read_alpha(0)
    check_alpha(a1, i1, a0, i0, label="alpha series vs plain")
    d0, d1 = plain.diagnostics(0), ser.diagnostics(0)
    _say(f"    mean updates plain {d0['mean_newton_iters']:.3f} series {d1['mean_newton_iters']:.3f}")
    assert d1["mean_newton_iters"] < 0.8 * d0["mean_newton_iters"]


def test_ragged_multibox_all_terms_fp64(elbm):
    # Several boxes in one launch, sizes that are not multiples of the block,
    # every term on: surface charge with curvature, external field, Carreau.
    p = inputs.base_params(Q_b=0.03, Q_s=0.3, carreau=1, nu0=0.5, nu_inf=0.05, lam=10.0, n_flow=0.5,
                           sor_sweeps=6, sor_omega=1.5)
    b0 = inputs.droplet_box(10, 6, 8, 2.5, seed=11)
    b0.info.update(E_ext=[1e-3, 0.0, 2e-3])
    b1 = inputs.droplet_box(12, 14, 16, 4.0, seed=12, walls_z=True, phi_bottom=0.0, phi_top=-0.02)
    b2 = inputs.droplet_box(16, 16, 16, 5.0, seed=13)
    b2.info.update(Q_b=0.01, Q_s=0.1, n_flow=0.8, E_ext=[0.0, 5e-4, 0.0])
    lat, oras = run_both(elbm, p, [b0, b1, b2], "f64", 30, "ragged multibox")
    for i, o in enumerate(oras):
        compare(lat, i, o, 1e-12)


def test_poisson_odd_sweeps_small_boxes_fp64(elbm):
    # The Poisson sweeps on boxes smaller than one 256-node block (periodic
    # edges of 4 and 6, a bounded edge of 5), an odd sweep count and Dirichlet
    # walls, against the oracle.  (Fields
    # are compared relative to their largest value, so every box carries a
    # field with an x component: a velocity that vanishes by symmetry would
    # leave only rounding noise to compare.)
    p = inputs.base_params(Q_b=0.02, Q_s=0.2, sor_sweeps=5, sor_omega=1.4)
    b0 = inputs.droplet_box(4, 6, 10, 1.5, seed=21)
    b0.info.update(E_ext=[1e-3, 1e-3, 0.0])
    b1 = inputs.droplet_box(6, 6, 5, 1.5, seed=22, walls_z=True, phi_bottom=0.0, phi_top=-0.01)
    b1.info.update(E_ext=[1e-3, 0.0, 0.0])
    b2 = inputs.droplet_box(10, 4, 12, 2.0, seed=23)
    b2.info.update(E_ext=[2e-3, 0.0, 1e-3])
    lat, oras = run_both(elbm, p, [b0, b1, b2], "f64", 12, "tiny boxes, 5 sweeps")
    for i, o in enumerate(oras):
        compare(lat, i, o, 1e-12)


def test_efield_walls_carreau_fp64(elbm):
    # Reduced geometry of the drop between electrodes: walls + Dirichlet planes, Carreau.
    wl = inputs.efield_drop(nx=16, ny=16, nz=32)
    lat, (o,) = run_both(elbm, wl.params, wl.boxes, "f64", 100, "efield 16x16x32 f64")
    compare(lat, 0, o, 1e-12)


def storage_rounding_error(params, box, steps):
    """Field errors of the oracle when only its populations are rounded to FP32
    after every step: the error FP32 population storage alone brings."""
    import oracle as ora
    ref = ora.Oracle(params, box, nthreads=NTHREADS)
    emu = ora.Oracle(params, box, nthreads=NTHREADS)
    for _ in range(steps):
        emu.set_populations(emu.field(ora.F_POP).astype(np.float32).astype(np.float64))
        emu.step(1)
        ref.step(1)
    u, ue = ref.field(ora.F_UPH), emu.field(ora.F_UPH)
    r, re = ref.field(ora.F_RHO), emu.field(ora.F_RHO)
    return {"rhoA": rel(re[0], r[0]), "rhoB": rel(re[1], r[1]), "ux": rel(ue[0], u[0]),
            "uy": rel(ue[1], u[1]), "uz": rel(ue[2], u[2]),
            "phi": rel(emu.field(ora.F_PHI), ref.field(ora.F_PHI))}


def check_fp32(lat, o, params, box, steps, i=0):
    # Densities, velocity and potential within 1e-5 of the FP64 oracle (field-
    # max normalised).  The error that FP32 storage of the populations alone
    # brings (the oracle with its populations rounded after every step) is
    # reported beside it.
    errs = compare(lat, i, o, 1e-5, fields=("rhoA", "rhoB", "ux", "uy", "uz", "phi"))
    store = storage_rounding_error(params, box, steps)
    _say("    FP32-storage-only oracle errors: " + " ".join(f"{k}={v:.2e}" for k, v in store.items()))
    return errs


def test_efield_fp32_100_steps(elbm):
    # FP32 populations, FP64 fields, FP64 alpha against the FP64 oracle.
    wl = inputs.efield_drop(nx=32, ny=32, nz=64)
    lat, (o,) = run_both(elbm, wl.params, wl.boxes, "f32", 100, "efield 32x32x64 f32")
    check_fp32(lat, o, wl.params, wl.boxes[0], 100)
    compare(lat, 0, o, 1e-4, fields=("q",))


def test_efield_fp32all_100_steps(elbm):
    # FP32 populations and FP32 fields: the error is reported for every field;
    # the bound is the one derived for single-precision stencils of psi and phi.
    wl = inputs.efield_drop(nx=32, ny=32, nz=64)
    lat, (o,) = run_both(elbm, wl.params, wl.boxes, "f32all", 100, "efield 32x32x64 f32all")
    compare(lat, 0, o, 1e-3, fields=("rhoA", "rhoB", "phi", "q"))
    compare(lat, 0, o, 3e-2, fields=("ux", "uy", "uz"))


def test_efield_full_size_fp32(elbm):
    # The benchmark's workload at its full size (64x64x128, FP32), 100 steps,
    # in the launch mapping and with the starter the benchmark times (8x4x8
    # bricks for k_alpha, 4-step graphs, k_alpha beside the sweeps with the
    # sweeps' waves at raised priority, series root).
    wl = inputs.efield_drop()
    lat, (o,) = run_both(elbm, wl.params, wl.boxes, "f32", 100, "efield 64x64x128 f32", launch=(0, 4, 2, 1),
                         guess="series")
    check_fp32(lat, o, wl.params, wl.boxes[0], 100)


@pytest.mark.parametrize("curvature,electrostriction", [(0, 1), (1, 0), (0, 0)])
def test_term_switches_fp64(elbm, curvature, electrostriction):
    # The curvature weight of the surface charge and the electrostriction force
    # switched off one at a time and together, FP64, against the oracle.
    p = inputs.base_params(Q_b=0.03, Q_s=0.3, E_ext=[0.0, 0.0, 1e-3], sor_sweeps=6, sor_omega=1.5,
                           curvature=curvature, electrostriction=electrostriction)
    b = inputs.droplet_box(16, 16, 24, 5.0, seed=31)
    lat, (o,) = run_both(elbm, p, [b], "f64", 60, f"switches curvature={curvature} electrostriction={electrostriction}")
    compare(lat, 0, o, 1e-12)


def test_single_component_fp64(elbm):
    # The paper's own model: one Shan-Chen fluid, G = -5, liquid 1.93 / vapour 0.156.
    b = inputs.droplet_box(16, 16, 16, 5.0, seed=21, ncomp=1, rho_in=1.93, rho_out=0.156)
    p = inputs.Params(ncomp=1, G=[[-5.0, 0.0], [0.0, 0.0]], Q_b=0.2, Q_s=2.0, sor_sweeps=6, sor_omega=1.6)
    lat, (o,) = run_both(elbm, p, [b], "f64", 50, "single component")
    compare(lat, 0, o, 1e-12, fields=("rhoA", "ux", "uy", "uz", "phi", "q"))


def test_jet_geometry_small_fp64(elbm):
    # Inlet disk in a plate, outlet plane, Dirichlet electrodes, generator charge model.
    wl = inputs.jet(nx=16, ny=16, nz=32, r_noz=3.0)
    lat, (o,) = run_both(elbm, wl.params, wl.boxes, "f64", 30, "jet 16x16x32")
    compare(lat, 0, o, 1e-12)


def test_jet_full_size_fp32(elbm):
    # The jet at its full size (128x128x512, FP32 populations, Carreau, inlet
    # disk, outlet plane, electrodes, generator charge) in a tuned launch
    # mapping (XCD-aware order, 8-step graphs, 8x8x4 collision tiles), 3 steps against the FP64
    # oracle on every node at the FP32 bar.
    import oracle as ora
    wl = inputs.jet()
    b = wl.boxes[0]
    _say(f"[gpu parity] jet {b.nx}x{b.ny}x{b.nz} f32, 3 steps, launch (remap 1, graph 8, tile 8x8x4)")
    lat = elbm.Lattice(wl.params, wl.boxes, "f32")
    lat.set_launch(1, 8, 1)
    lat.step(3, record=True)
    lat.sync()
    o = ora.Oracle(wl.params, b, nthreads=NTHREADS)
    o.step(3)
    compare(lat, 0, o, 1e-5)
    d = lat.diagnostics(0)
    _say(f"    diag: collisions {d['n_collisions']} fallbacks {d['n_fallback']} negative {d['n_negative']}")
    assert d["n_collisions"] > 0


@pytest.mark.parametrize("guess", ["standard", "mlp"])
def test_jet_reduced_fp32_100_steps(elbm, guess):
    # The jet geometry with its full nozzle (radius 8, perturbed inlet disk,
    # Poiseuille inflow 0.02, collector plane, electrodes, generator charge,
    # Carreau n = 0.4) in a reduced 48x48x128 box, FP32 populations, 100 steps,
    # with plain Newton from 2 and with the learned starter (the stored
    # network): every field within the FP32 bar of the FP64 oracle.
    import oracle as ora
    from paper_1612_05404_amd import learned
    wl = inputs.jet(nx=48, ny=48, nz=128, r_noz=8.0)
    b = wl.boxes[0]
    _say(f"[gpu parity] jet {b.nx}x{b.ny}x{b.nz} nozzle r 8, f32, 100 steps, starter {guess}")
    lat = elbm.Lattice(wl.params, wl.boxes, "f32", alpha_guess=guess)
    if guess == "mlp":
        lat.mlp_set_weights(learned.load_weights())
    lat.step(100, record=True)
    lat.sync()
    o = ora.Oracle(wl.params, b, nthreads=NTHREADS)
    o.step(100)
    compare(lat, 0, o, 1e-5, fields=("rhoA", "rhoB", "ux", "uy", "uz", "phi"))
    compare(lat, 0, o, 1e-4, fields=("q",))
    al, it = lat.read_alpha(0)
    oal, oit = o.field(ora.F_ALPHA), o.iters()
    fluid = (b.node_type & 3) == inputs.FLUID
    both = (it >= 0) & (oit >= 0) & fluid[None]
    err = np.abs(al - oal)[both] / oal[both]
    _say(f"    alpha vs oracle (FP32 populations on the GPU): max rel {err.max():.2e}")
    d = lat.diagnostics(0)
    _say(f"    diag: collisions {d['n_collisions']} fallbacks {d['n_fallback']} negative {d['n_negative']} "
         f"mean updates {d['mean_newton_iters']:.4f}")
    lat.close()


def test_conservation_and_checkpoint(elbm):
    # Periodic FP64 drop: each component's mass is constant to rounding, and
    # get/set of the populations + potential resumes bit-exactly.
    wl = inputs.drop32(n=16)
    _say("[gpu] conservation + checkpoint 16^3")
    lat = elbm.Lattice(wl.params, wl.boxes, "f64")
    d0 = lat.diagnostics(0)
    lat.step(50, record=True)
    d1 = lat.diagnostics(0)
    for s in range(2):
        assert abs(d1["mass"][s] - d0["mass"][s]) <= 1e-13 * d0["mass"][s]
    f50, phi50 = lat.get_populations(0), lat.read_potential(0)
    lat.step(50, record=True)
    f100 = lat.get_populations(0)
    lat2 = elbm.Lattice(wl.params, wl.boxes, "f64")
    lat2.set_populations(0, f50)
    lat2.set_potential(0, phi50)
    lat2.step(50, record=True)
    assert np.array_equal(lat2.get_populations(0), f100)


def test_graph_replay_matches_direct_launches(elbm):
    # Steps replayed from the captured two-step graph equal directly launched
    # steps bit for bit, replay after replay, with eager work and
    # synchronisation in between.
    wl = inputs.efield_drop(nx=16, ny=16, nz=32)
    _say("[gpu] graph replay vs direct launches, efield 16x16x32 f32")
    g = elbm.Lattice(wl.params, wl.boxes, "f32", alpha_guess="series")
    d = elbm.Lattice(wl.params, wl.boxes, "f32", alpha_guess="series")
    d.set_graphs(False)
    for rep in range(4):
        g.step(9, record=True)      # 4 graph pairs + 1 recorded direct step
        d.step(9, record=True)
        g.sync()
        d.sync()
        assert np.array_equal(g.get_populations(0), d.get_populations(0)), rep
        assert np.array_equal(g.read_potential(0), d.read_potential(0)), rep
        rho_g, u_g = g.read_moments(0)
        rho_d, u_d = d.read_moments(0)
        assert np.array_equal(rho_g, rho_d) and np.array_equal(u_g, u_d), rep
    assert g.diagnostics(0)["n_collisions"] == d.diagnostics(0)["n_collisions"]


def test_alpha_stream_order_does_not_change_results(elbm):
    # k_alpha runs on the library's second stream beside the Poisson sweeps,
    # or in order on one stream when phase timing is on: it reads only the
    # populations, so both give the same step bit for bit (learned starter
    # included), graph-replayed or launched directly.
    wl = inputs.efield_drop(nx=16, ny=16, nz=32)
    _say("[gpu] two streams vs one stream (phase timing), efield 16x16x32 f32, series and learned starters")
    from paper_1612_05404_amd import learned
    for guess in ("series", "mlp"):
        a = elbm.Lattice(wl.params, wl.boxes, "f32", alpha_guess=guess)
        b = elbm.Lattice(wl.params, wl.boxes, "f32", alpha_guess=guess)
        if guess == "mlp":
            w = learned.load_weights()
            a.mlp_set_weights(w)
            b.mlp_set_weights(w)
        b.set_timing(True)
        for rep in range(3):
            a.step(7, record=True)
            b.step(7, record=True)
            a.sync()
            b.sync()
            assert np.array_equal(a.get_populations(0), b.get_populations(0)), (guess, rep)
            assert np.array_equal(a.read_alpha(0)[0], b.read_alpha(0)[0]), (guess, rep)
        ph = b.timing()
        assert ph["steps"] == 21 and ph["alpha"] > 0 and ph["collide"] > 0
        assert a.diagnostics(0)["mean_newton_iters"] == b.diagnostics(0)["mean_newton_iters"]
        a.close()
        b.close()


def test_nonfinite_is_reported(elbm):
    # A NaN planted from the host propagates and sets the sticky error word.
    wl = inputs.drop32(n=16)
    _say("[gpu] non-finite error path 16^3")
    lat = elbm.Lattice(wl.params, wl.boxes, "f64")
    f = lat.get_populations(0)
    f[0, 3, 5, 5, 5] = np.nan
    lat.set_populations(0, f)
    lat.step(2, record=False)
    with pytest.raises(elbm.ElbmError) as e:
        lat.sync()
    assert e.value.status == elbm.ELBM_ENONFINITE


def test_large_box_fp64_parity(elbm):
    # A box of 2^20 nodes (the e-field drop's walls and electrodes at
    # 128x128x64), where the Poisson half sweeps run one thread per node pair:
    # FP64, 6 steps, every field against the oracle at the FP64 bar.
    wl = inputs.efield_drop(nx=128, ny=128, nz=64)
    p = wl.params.with_(sor_sweeps=9)
    lat, (o,) = run_both(elbm, p, wl.boxes, "f64", 6, "e-field drop 128x128x64 (pair sweeps)")
    compare(lat, 0, o, 1e-12)
