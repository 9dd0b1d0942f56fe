"""The allocation-free entry point (elbm_mlp_grad_noalloc) through the C ABI:
bitwise equal to elbm_mlp_grad's gradient and loss, on two calls in a row
(the second with fewer samples, so the scratch holds the first call's
partials when it starts)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_noalloc_gradient_equals_allocating_entry_point():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1612_05404_amd import elbm, inputs, learned
    elbm.load()
    wl = inputs.drop32(n=16)
    lat = elbm.Lattice(wl.params, wl.boxes, "f64", alpha_guess="mlp")
    lat.mlp_set_weights(learned.init_weights(11))
    gen = torch.Generator(device="cpu").manual_seed(5)
    X = (torch.rand((50000, 20), generator=gen) * 2.0 - 1.0).to("cuda:0")
    T = (torch.rand(50000, generator=gen) - 0.5).to("cuda:0")
    G = torch.empty(lat.MLP_NPARAM + 1, dtype=torch.float32, device="cuda:0")
    for M in (50000, 777):
        _say(f"[gpu no-alloc] mlp gradient, M = {M}")
        lat.mlp_grad_noalloc(X[:M], T[:M], G)
        lat.sync()
        got = G.cpu().numpy()
        ref, loss = lat.mlp_grad(X[:M], T[:M])
        assert np.array_equal(got[:-1], ref), float(np.abs(got[:-1] - ref).max())
        assert got[-1] == np.float32(loss)
        assert np.abs(ref).max() > 0.0
    lat.close()
