"""The seeded workload generator: determinism and the statistics it promises."""
import numpy as np

from paper_1803_00005_amd import synth


def test_same_seed_same_arrays():
    w = synth.WORKLOADS["rgb64_n3_L16"]
    g1, c1 = synth.make_workload(w)
    g2, c2 = synth.make_workload(w)
    np.testing.assert_array_equal(g1, g2)
    np.testing.assert_array_equal(c1, c2)
    assert g1.dtype == np.float32 and c1.dtype == np.float32
    assert g1.shape == (3, 64, 64) and c1.shape == (64, 64, 16)


def test_small_workload_statistics():
    w = synth.WORKLOADS["rgb64_n3_L16"]
    g, c, d = synth.make_workload(w, with_disparity=True)
    # integer region disparities in [0, 15]
    assert np.all(d == np.round(d)) and d.min() >= 0 and d.max() <= 15
    # cost is the truncated |l - d| / 16 plus N(0, 0.01^2)
    base = np.minimum(np.abs(np.arange(16)[None, None, :] - d[:, :, None]) / 16.0, 0.5)
    resid = c - base
    assert abs(resid.mean()) < 1e-3 and 0.009 < resid.std() < 0.011
    # the true disparity is the argmin of the noiseless cost
    assert np.all(np.argmin(base, axis=2) == d)
    # colours in [0, 1] plus sigma 0.02 noise, not clamped
    assert -0.15 < g.min() < 0.05 and 0.95 < g.max() < 1.15


def test_voronoi_tie_goes_to_lower_index():
    seeds = np.array([[1.0, 0.5], [0.0, 0.5]])
    reg = synth.voronoi_regions(seeds, 1, 2)
    # pixel 0 centre (0.5, 0.5) is equidistant from both seeds
    assert reg[0, 0] == 0
    assert reg[0, 1] == 0


def test_bf16_rounding_is_nearest_even():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9, -2.5], dtype=np.float32)
    r = synth._round_bf16(x)
    np.testing.assert_array_equal(r, np.array([1.0, 1.0, 1.0 + 2 ** -6, 1.0, -2.5], dtype=np.float32))


def test_batch_and_request_specs_are_seeded():
    a = synth.make_batch_specs(8)
    b = synth.make_batch_specs(8)
    assert a == b
    assert {s.degree for s in synth.make_batch_specs(64)} == {1, 2, 3}
    reqs = synth.make_request_specs(50)
    t = np.array([r[0] for r in reqs])
    assert np.all(np.diff(t) >= 0) and t[0] == 0.0
    assert all(r[1].n in (9, 19) for r in reqs)
