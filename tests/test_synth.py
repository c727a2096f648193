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


def test_rounded_cost_workloads_round_the_float32_costs():
    import dataclasses
    w = synth.WORKLOADS["rgb64_n3_L16"]
    _, c32 = synth.make_workload(w)
    # round to nearest: within half a unit in the last place of the type
    # (8 and 11 significand bits; float16 subnormals below 2^-14 have a fixed
    # spacing of 2^-24)
    for dt, rel_tol, abs_tol in (("bf16", 2.0 ** -8, 0.0), ("f16", 2.0 ** -11, 2.0 ** -25)):
        _, c = synth.make_workload(dataclasses.replace(w, cost_dtype=dt))
        assert np.all(np.abs(c - c32) <= rel_tol * np.abs(c32) + abs_tol)
        assert np.array_equal(synth.round_cost(c, dt), c)   # already representable
    # f16 values are exactly what numpy's float16 conversion gives
    _, c16 = synth.make_workload(dataclasses.replace(w, cost_dtype="f16"))
    assert np.array_equal(c16, c32.astype(np.float16).astype(np.float32))
