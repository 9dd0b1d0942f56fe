"""Learned alpha starter on the GPU: matrix-core forward pass and gradient
against the FP64 numpy reference, training on the library's kernels, the
sample kernel against the CPU oracle, and the starter's effect on the update
(same alpha and fields, fewer Newton updates)."""
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


def _host(elbm):
    """A small lattice whose context hosts the network buffers."""
    wl = inputs.drop32(n=8)
    return elbm.Lattice(wl.params, wl.boxes, "f64", alpha_guess="mlp")


def _random_net(seed):
    from oracle import mlp
    rng = np.random.default_rng(seed)
    w = mlp.init_weights(seed, scale_out=0.5)
    w[mlp.OFF_B1:mlp.OFF_W2] = rng.normal(scale=0.3, size=32)
    w[mlp.OFF_B2:mlp.OFF_W3] = rng.normal(scale=0.3, size=32)
    w[mlp.OFF_B3] = 0.1
    return w.astype(np.float32)


@pytest.mark.parametrize("M", [1, 64, 1000, 70001])
def test_forward_matches_bf16_reference(elbm, M):
    # 1000 and 70001 are ragged against both the 64-node wave tile and the
    # 256-thread block; a wrong matrix-core lane layout gives O(1) errors.
    import torch
    from oracle import mlp
    _say(f"[gpu mlp] forward M={M}")
    lat = _host(elbm)
    w = _random_net(11)
    lat.mlp_set_weights(w)
    assert np.array_equal(lat.mlp_get_weights(), w)
    rng = np.random.default_rng(M)
    X = rng.uniform(-1, 1, (M, 20)).astype(np.float32)
    y = lat.mlp_forward(torch.from_numpy(X).cuda()).cpu().numpy().astype(np.float64)
    ref = mlp.forward(w.astype(np.float64), X, bf16=True)
    ref64 = mlp.forward(w.astype(np.float64), X)
    scale = np.abs(ref).max()
    d = np.abs(y - ref) / scale
    _say(f"    |y - y_bf16ref|/max|y|: median {np.median(d):.2e} max {d.max():.2e}; vs FP64 ref max "
         f"{np.abs(y - ref64).max() / scale:.2e}")
    assert np.median(d) <= 2e-5
    assert d.max() <= 5e-3
    assert np.abs(y - ref64).max() <= 5e-2 * scale
    lat.close()


def test_gradient_matches_oracle(elbm):
    import torch
    from oracle import mlp
    _say("[gpu mlp] gradient vs FP64 numpy, M=5000")
    lat = _host(elbm)
    w = _random_net(12)
    lat.mlp_set_weights(w)
    rng = np.random.default_rng(5)
    X = rng.uniform(-1, 1, (5000, 20)).astype(np.float32)
    T = rng.normal(size=5000).astype(np.float32)
    g, L = lat.mlp_grad(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda())
    L0, g0 = mlp.loss_and_grad(w.astype(np.float64), X.astype(np.float64), T.astype(np.float64))
    _say(f"    loss gpu {L:.6e} oracle {L0:.6e}")
    assert L == pytest.approx(L0, rel=1e-2)
    for name, a, b in [("W1", 0, 640), ("b1", 640, 672), ("W2", 672, 1696), ("b2", 1696, 1728),
                       ("w3", 1728, 1760), ("b3", 1760, 1761)]:
        ga, gb = g[a:b].astype(np.float64), g0[a:b]
        relerr = np.linalg.norm(ga - gb) / np.linalg.norm(gb)
        cos = float(ga @ gb / (np.linalg.norm(ga) * np.linalg.norm(gb)))
        _say(f"    {name}: rel L2 err {relerr:.2e} cosine {cos:.6f}")
        assert relerr <= 3e-2 and cos >= 0.999
    lat.close()


def test_training_fits_a_teacher_network(elbm):
    # Targets from a fixed teacher network; the student starts elsewhere and
    # must fit them with the library's forward/backward/Adam kernels.
    import torch
    from oracle import mlp
    _say("[gpu mlp] training on teacher targets")
    lat = _host(elbm)
    teacher = _random_net(21).astype(np.float64)
    rng = np.random.default_rng(6)
    X = rng.uniform(-1, 1, (20000, 20)).astype(np.float32)
    T = mlp.forward(teacher, X).astype(np.float32)
    Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    lat.mlp_set_weights(mlp.init_weights(3).astype(np.float32))
    _, L_start = lat.mlp_grad(Xd, Td)
    losses = lat.mlp_train(Xd, Td, batch=1024, steps=3000, lr=3e-3)
    _, L_end = lat.mlp_grad(Xd, Td)
    w = lat.mlp_get_weights()
    L_cpu = mlp.loss(w.astype(np.float64), X, T)
    _say(f"    loss start {L_start:.3e} end {L_end:.3e} (FP64 forward of the trained weights {L_cpu:.3e}); "
         f"first/last batch {losses[0]:.3e}/{losses[-1]:.3e}")
    assert np.all(np.isfinite(losses))
    assert L_end < 0.05 * L_start
    assert L_cpu < 0.1 * L_start
    lat.close()


def test_training_arguments_are_checked(elbm):
    import torch
    lat = _host(elbm)
    X = torch.zeros((10, 20), device="cuda")
    T = torch.zeros(10, device="cuda")
    with pytest.raises(elbm.ElbmError):
        lat.mlp_train(X, T, batch=0, steps=1, lr=1e-3)
    with pytest.raises(elbm.ElbmError):
        lat.mlp_set_weights(np.zeros(10, np.float32))
    lat.close()


def test_alpha_samples_match_oracle(elbm):
    # Features, scale and target (alpha* - 2)/s of every fluid node against
    # the oracle's pulled populations and its FP64 alpha root.
    import oracle as ora
    from oracle import mlp
    wl = inputs.drop32(n=16)
    _say("[gpu mlp] alpha samples vs oracle, 16^3 drop, 5 steps")
    lat = elbm.Lattice(wl.params, wl.boxes, "f64")
    lat.step(5, record=False)
    feat, tgt, scl, val = lat.alpha_samples(0)
    feat, tgt, scl, val = (t.cpu().numpy() for t in (feat, tgt, scl, val))
    o = ora.Oracle(wl.params, wl.boxes[0], nthreads=NTHREADS)
    o.step(6)
    pulled = o.field(ora.F_PULLED)  # [C][19][z][y][x]: the pull of step 6 is the state after step 5
    C = pulled.shape[0]
    nz, ny, nx = pulled.shape[2:]
    c, wts = ora.lattice()
    n_checked = 0
    rng = np.random.default_rng(0)
    picks = rng.choice(nx * ny * nz, size=1500, replace=False)
    for s in range(C):
        for n in picks:
            z, y, x = n // (nx * ny), (n // nx) % ny, n % nx
            f = pulled[s, :, z, y, x]
            rho = f.sum()
            u = (c.T @ f) / rho
            fe = ora.feq(rho, u)
            zr, sr, ok = mlp.starter_features(f, fe)
            k = s * nx * ny * nz + n
            a, it = ora.alpha(f, fe, u, rho)
            ok = ok and it >= 0
            assert bool(val[k]) == ok, (s, n)
            if not ok:
                continue
            n_checked += 1
            assert np.abs(feat[k, :19] - zr).max() <= 1e-6
            assert feat[k, 19] == pytest.approx(sr, rel=1e-6)
            assert scl[k] == pytest.approx(sr, rel=1e-6)
            t = (a - 2.0) / sr
            assert tgt[k] == pytest.approx(t, rel=1e-5, abs=1e-6), (s, n, tgt[k], t)
    _say(f"    checked {n_checked} valid samples")
    assert n_checked > 1000
    lat.close()


def _trained_on_drop(elbm, steps=3000):
    """Samples from a run of the 32^3 drop, a short training run, the weights."""
    from paper_1612_05404_amd import learned
    wl = inputs.drop32()
    lat = elbm.Lattice(wl.params, wl.boxes, "f64", alpha_guess="mlp")
    X, T = learned.collect(lat, snapshots=40, every=3)
    lat.mlp_set_weights(learned.init_weights(1))
    losses = learned.train(lat, X, T, steps=steps, batch=4096, lr=3e-3, lr_end=2e-4)
    w = lat.mlp_get_weights()
    lat.close()
    return w, losses, X.shape[0]


def _same_state(elbm, wl, dtype, steps, modes, weights=None):
    """Lattices of the given starters, all holding the state a plain run
    reaches after `steps` steps."""
    ref = elbm.Lattice(wl.params, wl.boxes, dtype)
    ref.step(steps, record=False)
    f, phi = ref.get_populations(0), ref.read_potential(0)
    ref.close()
    out = {}
    for mode in modes:
        L = elbm.Lattice(wl.params, wl.boxes, dtype, alpha_guess=mode)
        if mode == "mlp":
            L.mlp_set_weights(weights)
        L.set_populations(0, f)
        L.set_potential(0, phi)
        out[mode] = L
    return out


def _one_step_iters(runs):
    """Served-node mask (flag 2 of the sample kernel) and, per starter, alpha,
    per-node update counts and diagnostics of one recorded step."""
    _, _, _, val = runs["mlp"].alpha_samples(0)
    served = val.cpu().numpy() == 2
    res = {}
    for mode, L in runs.items():
        L.step(1, record=True)
        al, it = L.read_alpha(0)
        res[mode] = (al.reshape(-1), it.reshape(-1), L.diagnostics(0))
    return served, res


def test_learned_starter_parity_and_fewer_iterations(elbm):
    # Train on the method's own samples, then: (1) the 32^3 FP64 drop with the
    # learned starter matches the oracle at the FP64 bar after 100 steps;
    # (2) from one shared state, alpha equals the plain solver's, the mean
    # update count is far below plain Newton from 2 and never above the
    # series starter alone, and on the nodes the network serves it saves
    # updates over the start from 2 that the series starter falls back to.
    import oracle as ora
    w, losses, m = _trained_on_drop(elbm)
    _say(f"[gpu mlp] trained on {m} served drop samples: batch loss {losses[:20].mean():.3e} -> "
         f"{losses[-200:].mean():.3e}")
    assert losses[-200:].mean() < 0.7 * losses[:20].mean()
    wl = inputs.drop32()
    lrn = elbm.Lattice(wl.params, wl.boxes, "f64", alpha_guess="mlp")
    lrn.mlp_set_weights(w)
    lrn.step(100, record=True)
    o = ora.Oracle(wl.params, wl.boxes[0], nthreads=NTHREADS)
    o.step(100)
    from test_gpu_parity import compare
    compare(lrn, 0, o, 1e-12)
    lrn.close()
    runs = _same_state(elbm, wl, "f64", 60, ("standard", "series", "mlp"), w)
    served, res = _one_step_iters(runs)
    a0, i0, d0 = res["standard"]
    a1, i1, d1 = res["mlp"]
    _, i2, d2 = res["series"]
    from test_gpu_parity import check_alpha
    check_alpha(a1, i1, a0, i0, label="alpha learned vs plain")
    sv = served & (i1 >= 0) & (i2 >= 0)
    _say(f"    mean updates standard {d0['mean_newton_iters']:.4f} "
         f"series {d2['mean_newton_iters']:.4f} learned {d1['mean_newton_iters']:.4f}; on the {int(sv.sum())} "
         f"served nodes series {i2[sv].mean():.3f} learned {i1[sv].mean():.3f}")
    assert d1["n_fallback"] <= d0["n_fallback"]
    assert d1["mean_newton_iters"] < 0.5 * d0["mean_newton_iters"]
    assert d1["mean_newton_iters"] <= d2["mean_newton_iters"]
    assert sv.sum() > 50 and i1[sv].mean() < i2[sv].mean()
    for L in runs.values():
        L.close()


@pytest.mark.skipif(not os.path.exists(os.path.join(os.path.dirname(__file__), "..", "paper_1612_05404_amd",
                                                    "alpha_mlp_weights.npy")),
                    reason="no stored network")
def test_stored_network_on_field_drop(elbm):
    # The stored network on the drop under a field (FP32 populations, reduced
    # 32x32x64 box), from one shared state: same alpha, and on the served
    # nodes fewer updates than the series starter's fallback start from 2.
    from paper_1612_05404_amd import learned
    wl = inputs.efield_drop(nx=32, ny=32, nz=64)
    _say("[gpu mlp] stored network, field drop 32x32x64 f32")
    runs = _same_state(elbm, wl, wl.dtype, 50, ("standard", "series", "mlp"), learned.load_weights())
    served, res = _one_step_iters(runs)
    a0, i0, d0 = res["standard"]
    a1, i1, d1 = res["mlp"]
    _, i2, d2 = res["series"]
    from test_gpu_parity import check_alpha
    check_alpha(a1, i1, a0, i0, label="alpha learned vs plain")  # alpha is 0 at non-fluid nodes
    sv = served & (i1 >= 0) & (i2 >= 0)
    _say(f"    mean updates standard {d0['mean_newton_iters']:.4f} "
         f"series {d2['mean_newton_iters']:.4f} learned {d1['mean_newton_iters']:.4f}; on the {int(sv.sum())} "
         f"served nodes series {i2[sv].mean():.3f} learned {i1[sv].mean():.3f}")
    assert d1["mean_newton_iters"] <= d2["mean_newton_iters"] < d0["mean_newton_iters"]
    if sv.sum() > 50:
        assert i1[sv].mean() < i2[sv].mean()
    for L in runs.values():
        L.close()
