"""Seeded input generators shared by both sides (no method arithmetic)."""
import numpy as np

from paper_1612_05404_amd import inputs


def test_splitmix64_reference_vector():
    # First outputs of SplitMix64 from state 0 (Steele, Lea and Flood's
    # generator, as in its public reference implementation).
    got = [int(v) for v in inputs.splitmix64(0, np.arange(3))]
    assert got == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_uniform_draws_are_seeded_and_in_range():
    a = inputs.uniform01(7, 10000)
    assert np.array_equal(a, inputs.uniform01(7, 10000))
    assert not np.array_equal(a, inputs.uniform01(8, 10000))
    assert a.min() >= 0.0 and a.max() < 1.0 and abs(a.mean() - 0.5) < 0.01
    assert np.array_equal(inputs.uniform01(7, 5, offset=3), a[3:8])
    xi = inputs.jitter_draws(5, 2, 100)
    assert xi.shape == (2, 19, 100) and xi.min() >= -1.0 and xi.max() < 1.0


def test_workload_shapes():
    wl = inputs.efield_drop()
    b = wl.boxes[0]
    assert (b.nx, b.ny, b.nz) == (64, 64, 128) and wl.dtype == "f32"
    assert (b.node_type[0] & 3).all() and (b.node_type[-1] & 3).all()  # electrode walls
    wl = inputs.drop32()
    assert wl.nodes == 32 ** 3 and wl.dtype == "f64"
    e = inputs.ensemble(nboxes=16)
    assert len(e.boxes) == 16 and all(b.nx in (24, 32, 48, 64) for b in e.boxes)
    assert all(b.info["Q_b"] > 0 for b in e.boxes)
