"""Batched ensembles: uneven droplet boxes advanced together in one launch per
phase (captured step graphs), against single-box runs, the CPU oracle and
every launch mapping the autotuner chooses from."""
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


def _fields(lat, i):
    rho, u = lat.read_moments(i)
    return rho, u, lat.read_potential(i), lat.read_charge(i)


def _same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


def test_ensemble_equals_single_box_runs(elbm):
    # Every box of a batched run must be bit-identical to the same box run
    # alone: per-box parameters, per-box reductions, no cross-box coupling.
    wl = inputs.ensemble(nboxes=6, edges=(24, 32))
    _say(f"[gpu ensemble] 6 boxes {[b.nx for b in wl.boxes]} f32, 24 steps, batched vs alone")
    lat = elbm.Lattice(wl.params, wl.boxes, "f32")
    lat.step(24, record=True)
    for i, b in enumerate(wl.boxes):
        one = elbm.Lattice(wl.params, [b], "f32")
        one.step(24, record=True)
        assert _same(_fields(lat, i), _fields(one, 0)), f"box {i} differs"
        d_all, d_one = lat.diagnostics(i), one.diagnostics(0)
        assert d_all["mean_newton_iters"] == d_one["mean_newton_iters"]
        one.close()
    lat.close()


def test_launch_mappings_give_identical_results(elbm):
    # XCD-aware block order and longer graphs change scheduling only.
    wl = inputs.ensemble(nboxes=5, edges=(24, 32, 48))
    _say("[gpu ensemble] launch mappings, 5 boxes f32, 24 steps")
    ref = None
    for remap, gs, tile, prio, lds in ((0, 2, 0, 0, 0), (1, 2, 0, 1, 1), (0, 8, 1, 0, 0), (1, 4, 2, 1, 0),
                                       (0, 2, 3, 1, 1), (1, 8, 3, 0, 0), (0, 2, 0, 0, 1)):
        lat = elbm.Lattice(wl.params, wl.boxes, "f32")
        lat.set_launch(remap, gs, tile, prio, lds)
        assert lat.get_launch() == {"xcd_remap": remap, "graph_steps": gs, "tile": tile, "sweep_priority": prio,
                                    "stencil_lds": lds}
        lat.step(24, record=True)
        got = [_fields(lat, i) + (lat.read_alpha(i)[0],) for i in range(len(wl.boxes))]
        if ref is None:
            ref = got
        else:
            assert all(_same(a, b) for a, b in zip(got, ref)), (remap, gs, tile, prio, lds)
        lat.close()
    lat = elbm.Lattice(wl.params, wl.boxes, "f32")
    try:
        for bad in ((0, 3, 0), (2, 2, 0), (0, 2, 4), (0, 2, 0, 2), (0, 2, 0, 0, 2)):
            with pytest.raises(elbm.ElbmError):
                lat.set_launch(*bad)
    finally:
        lat.close()


def test_ensemble_fp64_matches_oracle(elbm):
    # Three boxes with their own field, charge, Carreau exponent and SOR
    # factor, FP64, against the oracle box by box at the FP64 bar.
    import oracle as ora
    from test_gpu_parity import compare
    wl = inputs.ensemble(nboxes=3, edges=(24,))
    _say("[gpu ensemble] 3 boxes 24^3 f64 vs oracle, 30 steps")
    lat = elbm.Lattice(wl.params, wl.boxes, "f64")
    lat.set_launch(1, 4, 3)
    lat.step(30, record=True)
    for i, b in enumerate(wl.boxes):
        o = ora.Oracle(wl.params, b, nthreads=NTHREADS)
        o.step(30)
        _say(f"    box {i}: E_z {b.info['E_ext'][2]:.2e} Q_b {b.info['Q_b']:.3e} n {b.info['n_flow']:.3f}")
        compare(lat, i, o, 1e-12)
    lat.close()


def test_full_ensemble_sampled(elbm):
    # The full 256-box ensemble (27.5 M nodes, FP32, learned starter with the
    # stored network) in an XCD-aware mapping with 8x4x8 alpha tiles, 100
    # steps: a 24^3 and a 64^3 box equal the same boxes run alone bit for bit,
    # and both match the FP64 oracle at the FP32 bar.
    import oracle as ora
    from test_gpu_parity import compare
    from paper_1612_05404_amd import learned
    wl = inputs.ensemble()
    edges = [b.nx for b in wl.boxes]
    i24, i64 = edges.index(24), edges.index(64)
    _say(f"[gpu ensemble] full: {len(wl.boxes)} boxes, {wl.nodes} nodes, 100 steps; sampled boxes {i24}, {i64}")
    w = learned.load_weights()
    lat = elbm.Lattice(wl.params, wl.boxes, "f32", alpha_guess="mlp")
    lat.mlp_set_weights(w)
    lat.set_launch(1, 4, 2)
    lat.step(100, record=True)
    lat.sync()
    for i in (i24, i64):
        one = elbm.Lattice(wl.params, [wl.boxes[i]], "f32", alpha_guess="mlp")
        one.mlp_set_weights(w)
        one.step(100, record=True)
        assert _same(_fields(lat, i), _fields(one, 0)), f"box {i} differs"
        one.close()
        o = ora.Oracle(wl.params, wl.boxes[i], nthreads=NTHREADS)
        o.step(100)
        _say(f"    box {i} ({edges[i]}^3) vs oracle")
        compare(lat, i, o, 1e-5, fields=("rhoA", "rhoB", "ux", "uy", "uz", "phi"))
    lat.close()


def test_autotune_keeps_results(elbm):
    # The autotuner times all mappings, keeps the fastest and leaves the
    # state where the same number of plain steps leaves it.
    wl = inputs.ensemble(nboxes=4, edges=(24, 32))
    _say("[gpu ensemble] autotune, 4 boxes f32")
    a = elbm.Lattice(wl.params, wl.boxes, "f32")
    best, ms = a.autotune(16)
    _say(f"    best {best}; ms/step per candidate {np.round(ms, 4).tolist()}")
    assert np.all(np.isfinite(ms)) and np.all(ms > 0)
    assert best == a.get_launch()
    # passes: tile 0..3, then XCD order 0..1, then Poisson-branch priority
    # 0..1, then graph length 2, 4, 8
    assert len(ms) == 11
    assert ms[best["tile"]] == ms[:4].min()
    assert ms[4 + best["xcd_remap"]] == ms[4:6].min()
    assert ms[6 + best["sweep_priority"]] == ms[6:8].min()
    assert ms[8 + {2: 0, 4: 1, 8: 2}[best["graph_steps"]]] == ms[8:].min()
    b = elbm.Lattice(wl.params, wl.boxes, "f32")
    b.step(22 * 16 + 60, record=False)
    a.step(1, record=True)
    b.step(1, record=True)
    for i in range(len(wl.boxes)):
        assert _same(_fields(a, i), _fields(b, i)), i
    a.close()
    b.close()
