"""Parity of the HIP path with the FP64 oracle (run on an MI355X).

Bar: filtered costs within |Z - Z*| <= 1e-4 * max(|Z*|, max|V|) elementwise
(float32, bfloat16 and float16 costs; the 16-bit cases compare against the
oracle on the same rounded costs, and the full-size ones also state their
end-to-end error against the oracle on the unrounded float32 costs),
winner-takes-all labels equal wherever the oracle's two smallest costs differ
by at least 1e-5.  Integer box sums are compared bit for bit.  The named
workloads are compared at full size, every element and every label.
"""
import dataclasses
import json

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import banded  # noqa: E402
from oracle import hgf_oracle as O  # noqa: E402
from paper_1803_00005_amd import hgf, synth  # noqa: E402

pytestmark = pytest.mark.gpu

REL_TOL = 1e-4
TIE_GAP = 1e-5


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = hgf.Context(0)
    yield c
    c.close()


def dev():
    return torch.device("cuda", 0)


def to_dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a)).to(dev())
    return t.to(dtype) if dtype is not None else t


TORCH_COST = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}


def gpu_filter(ctx, guide, cost, w, **kw):
    cdt = TORCH_COST[w.cost_dtype]
    Z, lab = ctx.filter(to_dev(guide), to_dev(cost, cdt), radius=w.radius, eps=w.eps,
                        degree=w.degree, basis=w.basis, **kw)
    torch.cuda.synchronize()
    return Z.cpu().numpy().astype(np.float64), lab.cpu().numpy()


def oracle_filter(guide, cost, w, reg="covariance"):
    G = O.guidance(guide, w.degree, w.basis)
    if reg == "ridge":
        return O.filter_ridge(G, cost, w.radius, w.eps)
    return O.filter_covariance(G, cost, w.radius, w.eps)


def check(Z, lab, Zo, cost, what):
    scale = np.maximum(np.abs(Zo), np.abs(cost).max())
    rel = np.abs(Z - Zo) / scale
    worst = np.unravel_index(np.argmax(rel), rel.shape)
    say(f"{what}: max rel err {rel.max():.3e} at {worst}, rms abs {np.sqrt(np.mean((Z - Zo) ** 2)):.3e}")
    assert rel.max() <= REL_TOL, f"{what}: filtered costs off by {rel.max():.3e} at {worst}"
    if lab is not None:
        ok = (lab == O.wta(Zo)) | O.near_tie_mask(Zo, TIE_GAP)
        assert ok.all(), f"{what}: {int((~ok).sum())} labels differ away from near ties"


def W(name, **kw):
    base = dict(name=name, height=40, width=50, regions=8, labels=16, radius=4, eps=1e-4,
                degree=1, disparity="planar", seed=7)
    base.update(kw)
    return synth.Workload(**base)


CASES = [
    synth.WORKLOADS["rgb64_n3_L16"],
    W("n9_r9_ragged", height=70, width=130, regions=10, labels=60, radius=9, degree=2,
      disparity="smooth_region", seed=11),
    W("n19_r9_two_chunks", height=52, width=90, regions=9, labels=70, radius=9, eps=1e-3,
      degree=3, seed=12),
    W("gray_n1_r2", height=23, width=37, guide_channels=1, labels=5, radius=2, seed=13),
    W("power_n6_r7", height=40, width=50, basis="power", degree=2, labels=20, radius=7, seed=14),
    W("n4_gray_power_r1", height=17, width=70, guide_channels=1, basis="power", degree=4,
      labels=3, radius=1, eps=1e-3, seed=15),
    W("n9_r4_bf16", height=45, width=77, degree=2, labels=33, radius=4, cost_dtype="bf16", seed=16),
    W("n19_r4_bf16", height=30, width=70, degree=3, labels=40, radius=4, eps=1e-3,
      cost_dtype="bf16", seed=17),
    W("n2_m2", height=21, width=33, guide_channels=2, degree=1, labels=9, radius=2, seed=18),
    W("single_pixel", height=1, width=1, labels=7, radius=4, degree=2, seed=19),
    W("single_row", height=1, width=83, labels=5, radius=9, degree=2, seed=20),
    W("narrower_than_window", height=9, width=5, labels=4, radius=9, degree=1, seed=21),
    W("one_label", height=33, width=41, labels=1, radius=4, degree=2, seed=22),
    W("one_label_n19_ragged", height=37, width=300, labels=1, radius=9, degree=3, eps=1e-3,
      seed=24),
    W("one_label_bf16", height=41, width=29, labels=1, radius=2, degree=2, cost_dtype="bf16",
      seed=25),
    W("tall_n3_r7", height=140, width=20, labels=12, radius=7, degree=1, seed=23),
    # every radius of the compiled set (0 is the degenerate 1 x 1 window:
    # zero covariance, a = 0, Z = Y)
    W("r0_n3", height=19, width=23, labels=9, radius=0, degree=1, seed=40),
    W("r3_n9_ragged", height=47, width=75, labels=40, radius=3, degree=2, seed=41),
    W("r5_n6_power", height=38, width=91, basis="power", degree=2, labels=65, radius=5, seed=42),
    W("r6_n19", height=33, width=57, labels=20, radius=6, degree=3, eps=1e-3, seed=43),
    W("r8_n4_gray", height=50, width=44, guide_channels=1, basis="power", degree=4, labels=18,
      radius=8, eps=1e-3, seed=44),
    # channel counts between 9 and 19
    W("n10_gray_monomial", height=35, width=70, guide_channels=1, degree=10, labels=24,
      radius=4, eps=1e-3, seed=45),
    W("n12_rgb_power_d4", height=40, width=66, basis="power", degree=4, labels=33, radius=7,
      eps=1e-3, seed=46),
    W("n14_m2_monomial_d4", height=31, width=80, guide_channels=2, degree=4, labels=17,
      radius=2, eps=1e-3, seed=47),
    W("n15_rgb_power_d5", height=29, width=52, basis="power", degree=5, labels=8, radius=1,
      eps=1e-3, seed=48),
    W("n18_rgb_power_d6", height=37, width=45, basis="power", degree=6, labels=12, radius=9,
      eps=1e-2, seed=49),
    # float16 costs
    W("n9_r9_f16", height=52, width=81, degree=2, labels=70, radius=9, cost_dtype="f16", seed=50),
    W("n19_r4_f16", height=30, width=70, degree=3, labels=20, radius=4, eps=1e-3,
      cost_dtype="f16", seed=51),
    W("one_label_f16", height=27, width=33, labels=1, radius=3, degree=2, cost_dtype="f16",
      seed=52),
    # the narrow strips of n <= 3 at r <= 4: several strips with a ragged last
    # one, two label chunks, 16-bit costs
    W("n3_r1_bf16_two_chunks", height=61, width=150, labels=70, radius=1, degree=1,
      cost_dtype="bf16", seed=53),
    W("n3_r4_f16_ragged", height=45, width=170, labels=20, radius=4, degree=1, cost_dtype="f16",
      seed=54),
    W("n1_gray_r3_ragged", height=70, width=131, guide_channels=1, labels=33, radius=3, seed=55),
]


@pytest.mark.parametrize("w", CASES, ids=[c.name for c in CASES])
def test_filter_matches_oracle(ctx, w):
    say(f"case {w.name}: {w.height}x{w.width} n={w.n} L={w.labels} r={w.radius} {w.cost_dtype}")
    guide, cost = synth.make_workload(w)
    Z, lab = gpu_filter(ctx, guide, cost, w)
    Zo = oracle_filter(guide, cost, w)
    check(Z, lab, Zo, cost, w.name)


# the float64 solve (stats_dtype = f64): covariance records and c, a, b in float64
F64_CASES = [c for c in CASES if c.name in (
    "rgb64_n3_L16", "n9_r9_ragged", "n19_r9_two_chunks", "n19_r4_bf16", "n12_rgb_power_d4",
    "r0_n3", "one_label", "one_label_n19_ragged", "n9_r9_f16", "gray_n1_r2")]


@pytest.mark.parametrize("w", F64_CASES, ids=[c.name for c in F64_CASES])
def test_float64_solve_matches_oracle(ctx, w):
    say(f"f64 solve case {w.name}: {w.height}x{w.width} n={w.n} L={w.labels} r={w.radius}")
    guide, cost = synth.make_workload(w)
    Z, lab = gpu_filter(ctx, guide, cost, w, stats_dtype="f64")
    Zo = oracle_filter(guide, cost, w)
    check(Z, lab, Zo, cost, w.name + " f64 solve")


RIDGE_CASES = [
    # the paper's experimental setting: lambda = 0.05, r = 7, power basis of degree 2 on colour
    W("ridge_paper_power_d2_r7", height=40, width=60, basis="power", degree=2, labels=24,
      radius=7, eps=0.05, seed=31),
    W("ridge_n3_r4", height=35, width=44, degree=1, labels=16, radius=4, eps=0.05, seed=32),
    W("ridge_gray_n1_r2", height=25, width=19, guide_channels=1, degree=1, labels=6, radius=2,
      eps=0.01, seed=33),
    W("ridge_n9_r9", height=48, width=66, degree=2, labels=20, radius=9, eps=0.05, seed=34),
    W("ridge_n19_r4", height=30, width=44, degree=3, labels=20, radius=4, eps=0.05, seed=35),
    # one slice of a gray image under the power basis: the setting of Tables 1-2
    W("ridge_gray_power_L1", height=70, width=300, guide_channels=1, basis="power", degree=5,
      labels=1, radius=7, eps=0.05, seed=36),
    W("ridge_n9_L1", height=40, width=90, degree=2, labels=1, radius=4, eps=0.05, seed=37),
    W("ridge_n12_r5", height=36, width=58, basis="power", degree=4, labels=30, radius=5,
      eps=0.05, seed=38),
    # the gray sweep's other one-label kernels (n = 3 and 7, the setting of Tables 1-2)
    W("ridge_gray_power_n3_L1", height=90, width=130, guide_channels=1, basis="power",
      degree=3, labels=1, radius=7, eps=0.05, seed=53),
    W("ridge_gray_power_n7_L1", height=75, width=160, guide_channels=1, basis="power",
      degree=7, labels=1, radius=7, eps=0.05, seed=54),
    W("ridge_r0_n3", height=17, width=21, degree=1, labels=6, radius=0, eps=0.05, seed=39),
]


@pytest.mark.parametrize("w", RIDGE_CASES, ids=[c.name for c in RIDGE_CASES])
def test_ridge_form_matches_oracle(ctx, w):
    say(f"ridge case {w.name}: {w.height}x{w.width} n={w.n} L={w.labels} r={w.radius} lambda={w.eps}")
    guide, cost = synth.make_workload(w)
    Z, lab = gpu_filter(ctx, guide, cost, w, reg="ridge")
    Zo = oracle_filter(guide, cost, w, reg="ridge")
    check(Z, lab, Zo, cost, w.name)


@pytest.mark.parametrize("shape,r", [((1, 1, 1), 0), ((2, 7, 9), 1), ((3, 33, 70), 4),
                                     ((1, 5, 3), 9), ((2, 129, 67), 9)])
def test_box_sum_bit_exact(shape, r):
    say(f"box sum {shape} r={r}")
    rng = np.random.default_rng(sum(shape) + r)
    x = rng.integers(-1000, 1000, size=shape).astype(np.float32)
    out = hgf.box_sum(to_dev(x), r)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), O.box_sum(x, r).astype(np.float32))


@pytest.mark.parametrize("D", [1, 2, 3, 7, 10, 11, 13, 16, 19, 20])
def test_spd_inverse_matches_lu(D):
    say(f"spd inverse D={D}")
    rng = np.random.default_rng(D)
    X = rng.uniform(0, 1, size=(500, 3 * D + 2, D))
    A = np.einsum("bki,bkj->bij", X, X) + 1e-3 * np.eye(D)
    Minv = hgf.spd_inverse(to_dev(A))
    torch.cuda.synchronize()
    Mg = Minv.cpu().numpy()
    Mo = O.lu_inverse(A)
    rel = np.abs(Mg - Mo).max(axis=(1, 2)) / np.abs(Mo).max(axis=(1, 2))
    cond = np.linalg.cond(A)
    assert np.all(rel <= 1e-15 * cond * D * 10), f"max rel {rel.max():.2e}"
    # the full result is exactly symmetric (Prop. 1 builds a symmetric inverse)
    np.testing.assert_array_equal(Mg, np.swapaxes(Mg, 1, 2))


@pytest.mark.parametrize("w,stats", [(CASES[1], "f32"), (CASES[2], "f32"), (CASES[2], "f64"),
                                     (RIDGE_CASES[0], "f32"),
                                     # n <= 4: the inverse computed inside the moment kernel
                                     (CASES[0], "f32"), (CASES[0], "f64"), (RIDGE_CASES[1], "f32"),
                                     (RIDGE_CASES[2], "f32")],
                         ids=["n9", "n19", "n19_f64", "ridge_n6", "n3_fused", "n3_fused_f64",
                              "ridge_n3_fused", "ridge_n1_fused"])
def test_guide_statistics_match_oracle(ctx, w, stats):
    reg = "ridge" if w.name.startswith("ridge") else "covariance"
    say(f"guide statistics {w.name} ({reg}, {stats})")
    guide, _ = synth.make_workload(w)
    g = hgf.Guide(ctx, to_dev(guide), labels=w.labels, radius=w.radius, eps=w.eps,
                  degree=w.degree, basis=w.basis, reg=reg, stats_dtype=stats)
    mu, minv, shift = g.export()
    torch.cuda.synchronize()
    # the float32 covariance records hold the float64 inverse rounded to float32
    unit = 2.0 ** -24 if minv.dtype == torch.float32 else 2.0 ** -53
    mu, minv, shift = mu.cpu().numpy(), minv.cpu().numpy().astype(np.float64), shift.cpu().numpy()
    g.close()
    G = O.guidance(guide, w.degree, w.basis)
    n, H, Wd = G.shape
    D = n + 1 if reg == "ridge" else n
    iu = np.triu_indices(D)
    Mfull = np.zeros((H, Wd, D, D))
    Mfull[:, :, iu[0], iu[1]] = minv
    Mfull[:, :, iu[1], iu[0]] = minv
    N = O.window_counts(H, Wd, w.radius)
    if reg == "covariance":
        mu_o, M_o = O.guide_statistics(guide, w.degree, w.radius, w.eps, w.basis)
        np.testing.assert_allclose(mu + shift[None, None, :], mu_o, rtol=0, atol=1e-12)
        A = np.linalg.inv(M_o)
    else:
        G1 = np.concatenate([np.ones((1, H, Wd)), G])
        A = np.empty((H, Wd, D, D))
        for i in range(D):
            for j in range(D):
                A[:, :, i, j] = O.box_sum(G1[i] * G1[j], w.radius)
        A += w.eps * np.eye(D)
        assert np.allclose(A[:, :, 0, 0], N + w.eps)
    resid = np.abs(np.einsum("hwij,hwjk->hwik", Mfull, A) - np.eye(D)).max()
    cond = np.linalg.cond(A).max()
    say(f"  max |M A - E| = {resid:.3e}, max cond = {cond:.3e}")
    assert resid <= (1e-13 + 4 * unit) * cond * D


def test_two_phase_chunks_equal_plain_path(ctx):
    w = CASES[2]
    say(f"two-phase chunks vs plain: {w.name}")
    guide, cost = synth.make_workload(w)
    Zp, labp = gpu_filter(ctx, guide, cost, w)
    g = hgf.Guide(ctx, to_dev(guide), labels=w.labels, radius=w.radius, eps=w.eps, degree=w.degree)
    H, Wd, L = cost.shape
    best = torch.empty((H, Wd), dtype=torch.float32, device=dev())
    lab = torch.empty((H, Wd), dtype=torch.int32, device=dev())
    Zc = np.empty((H, Wd, L))
    for l0, l1 in [(0, 30), (30, 31), (31, 70)]:
        chunk = to_dev(cost[:, :, l0:l1])
        out = torch.empty(chunk.shape, dtype=torch.float32, device=dev())
        g.filter(chunk, l0, out=out, best=best, labels=lab)
        torch.cuda.synchronize()
        Zc[:, :, l0:l1] = out.cpu().numpy()
    g.close()
    np.testing.assert_array_equal(Zc, Zp)
    np.testing.assert_array_equal(lab.cpu().numpy(), labp)
    np.testing.assert_array_equal(best.cpu().numpy(), Zp.astype(np.float32).min(axis=2))


def test_two_phase_one_label_equals_plain_path(ctx):
    """A one-label filter through the two-phase interface (per-pixel keys merged
    by the caller's running minimum) equals the plain call (labels written
    directly) bit for bit."""
    w = [c for c in CASES if c.name == "one_label"][0]
    say(f"two-phase one-label vs plain: {w.name}")
    guide, cost = synth.make_workload(w)
    Zp, labp = gpu_filter(ctx, guide, cost, w)
    g = hgf.Guide(ctx, to_dev(guide), labels=1, radius=w.radius, eps=w.eps, degree=w.degree)
    H, Wd, _ = cost.shape
    best = torch.empty((H, Wd), dtype=torch.float32, device=dev())
    lab = torch.empty((H, Wd), dtype=torch.int32, device=dev())
    out = torch.empty((H, Wd, 1), dtype=torch.float32, device=dev())
    g.filter(to_dev(cost), 0, out=out, best=best, labels=lab)
    torch.cuda.synchronize()
    g.close()
    np.testing.assert_array_equal(out.cpu().numpy().astype(np.float64), Zp)
    np.testing.assert_array_equal(lab.cpu().numpy(), labp)
    np.testing.assert_array_equal(best.cpu().numpy(), Zp[:, :, 0].astype(np.float32))


def test_batch_equals_individual(ctx):
    ws = [CASES[0], CASES[1], CASES[4], CASES[6]]
    say("batch of 4 vs individual calls")
    items, singles = [], []
    for w in ws:
        guide, cost = synth.make_workload(w)
        cdt = torch.bfloat16 if w.cost_dtype == "bf16" else torch.float32
        items.append(dict(guide=to_dev(guide), cost=to_dev(cost, cdt), radius=w.radius,
                          eps=w.eps, degree=w.degree, basis=w.basis))
        singles.append(gpu_filter(ctx, guide, cost, w))
    res = ctx.filter_batch(items)
    torch.cuda.synchronize()
    for (Zb, lb), (Zs, ls) in zip(res, singles):
        np.testing.assert_array_equal(Zb.cpu().numpy(), Zs)
        np.testing.assert_array_equal(lb.cpu().numpy(), ls)


def test_deterministic(ctx):
    w = CASES[1]
    say(f"determinism {w.name}")
    guide, cost = synth.make_workload(w)
    Z1, l1 = gpu_filter(ctx, guide, cost, w)
    Z2, l2 = gpu_filter(ctx, guide, cost, w)
    np.testing.assert_array_equal(Z1, Z2)
    np.testing.assert_array_equal(l1, l2)


def test_labels_only_and_out_only(ctx):
    w = CASES[0]
    say("labels-only and out-only calls")
    guide, cost = synth.make_workload(w)
    Z, lab = gpu_filter(ctx, guide, cost, w)
    Z2, _ = ctx.filter(to_dev(guide), to_dev(cost), radius=w.radius, eps=w.eps, degree=w.degree,
                       want_labels=False)
    _, lab2 = ctx.filter(to_dev(guide), to_dev(cost), radius=w.radius, eps=w.eps,
                         degree=w.degree, want_out=False)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(Z2.cpu().numpy(), Z)
    np.testing.assert_array_equal(lab2.cpu().numpy(), lab)


def test_small_workspace_rejected(ctx):
    w = CASES[0]
    say("undersized workspace")
    guide, cost = synth.make_workload(w)
    ws = torch.empty(1024, dtype=torch.uint8, device=dev())
    with pytest.raises(hgf.HGFError) as ei:
        ctx.filter(to_dev(guide), to_dev(cost), radius=w.radius, eps=w.eps, degree=w.degree,
                   workspace=ws)
    assert ei.value.status == hgf.HGF_E_INVALID


# ---------------------------------------------------------------------------
# full-size workloads: every element and every label against the oracle
# (computed by output tiles with a 2r halo in worker processes: exact)
# ---------------------------------------------------------------------------

_ORACLE = {}


def full_oracle(name):
    """Oracle Z of a named workload at full size (cached for the module)."""
    if name not in _ORACLE:
        w = synth.WORKLOADS[name]
        guide, cost = synth.make_workload(w)
        say(f"  oracle {name}: {banded.default_workers()} workers")
        _ORACLE[name] = banded.filter_image(O.guidance(guide, w.degree, w.basis), cost,
                                            w.radius, w.eps)
    return _ORACLE[name]


def parity_report(Z, lab, Zo, vmax, what):
    """Every-element comparison with the numbers the design notes record."""
    rel = np.abs(Z - Zo) / np.maximum(np.abs(Zo), vmax)
    two = np.partition(Zo, 1, axis=2)
    gap = two[..., 1] - two[..., 0]
    wta = O.wta(Zo)
    mism = lab != wta
    # the GPU's error at the oracle's two best labels: a label can only flip
    # where it reaches half the gap
    rows, cols = np.indices(lab.shape)
    best2 = np.argpartition(Zo, 1, axis=2)[..., :2]
    err2 = np.abs(Z[rows, cols, best2[..., 0]] - Zo[rows, cols, best2[..., 0]])
    err2 = np.maximum(err2, np.abs(Z[rows, cols, best2[..., 1]] - Zo[rows, cols, best2[..., 1]]))
    rep = {
        "case": what, "elements": int(Z.size), "max_rel": float(rel.max()),
        "max_abs": float(np.abs(Z - Zo).max()), "rms_abs": float(np.sqrt(np.mean((Z - Zo) ** 2))),
        "label_mismatches": int(mism.sum()),
        "label_mismatches_gap_ge_1e-5": int((mism & (gap >= TIE_GAP)).sum()),
        "near_tie_pixels": int((gap < TIE_GAP).sum()),
        "max_abs_err_at_top2": float(err2.max()),
        "mismatch_gaps": [float(g) for g in np.sort(gap[mism])[:8]],
    }
    say("[parity] " + json.dumps(rep))
    return rep


# (workload, solve precision); the bfloat16 / float16 ones also state their
# end-to-end error against the oracle on the unrounded float32 costs
FULL = [("voronoi450x375_n9_L60", "f32"), ("voronoi1242x375_n19_L128", "f32"),
        ("voronoi1242x375_n19_L128", "f64"), ("voronoi1242x375_n19_L128_bf16", "f32"),
        ("voronoi1242x375_n19_L128_bf16", "f64"), ("voronoi1242x375_n19_L128_f16", "f64")]
# End-to-end bound of the 16-bit cost forms against the oracle on the float32
# costs, relative to max |V| like the float32 bar: the input rounding alone is
# up to 2^-9 (bfloat16) / 2^-12 (float16) of each cost, and the filter is an
# average of the costs with weights of either sign.  Measured on the n = 19
# workload: 1.18e-3 (bfloat16) and 1.19e-4 (float16), with either solve
# precision; frozen at about 1.7 times that.
E2E_BOUND = {"bf16": 2e-3, "f16": 2e-4}


@pytest.mark.parametrize("name,stats", FULL, ids=[f"{n}-{s}" for n, s in FULL])
def test_full_size_every_element(ctx, name, stats):
    w = synth.WORKLOADS[name]
    say(f"full size {name}, {stats} solve")
    guide, cost = synth.make_workload(w)
    Z, lab = gpu_filter(ctx, guide, cost, w, stats_dtype=stats)
    vmax = float(np.abs(cost).max())
    Zo = full_oracle(name)
    rep = parity_report(Z, lab, Zo, vmax, f"{name} {stats}")
    assert rep["max_rel"] <= REL_TOL
    assert rep["label_mismatches_gap_ge_1e-5"] == 0
    # labels are the argmin of the returned costs, lowest label on ties
    assert np.array_equal(lab, np.argmin(Z.astype(np.float32), axis=2))
    if w.cost_dtype != "f32":
        ref = full_oracle(name.rsplit("_", 1)[0])   # the same workload, float32 costs
        _, cost32 = synth.make_workload(dataclasses.replace(w, cost_dtype="f32"))
        e2e = float(np.max(np.abs(Z - ref)) / np.abs(cost32).max())
        say(f"[parity] {json.dumps({'case': name + ' ' + stats, 'end_to_end_vs_f32_costs': e2e})}")
        assert e2e <= E2E_BOUND[w.cost_dtype]


@pytest.mark.parametrize("name", ["voronoi450x375_n9_L60", "voronoi1242x375_n19_L128"])
def test_full_size_two_phase_equals_plain(ctx, name):
    """Resident guide, labels in uneven chunks (one of more than 64 labels, so
    the call runs several launch groups): bit for bit the plain call."""
    w = synth.WORKLOADS[name]
    say(f"two-phase vs plain at full size: {name}")
    guide, cost = synth.make_workload(w)
    Zp, labp = gpu_filter(ctx, guide, cost, w)
    g = hgf.Guide(ctx, to_dev(guide), labels=w.labels, radius=w.radius, eps=w.eps,
                  degree=w.degree)
    H, Wd, L = cost.shape
    best = torch.empty((H, Wd), dtype=torch.float32, device=dev())
    lab = torch.empty((H, Wd), dtype=torch.int32, device=dev())
    Zc = np.empty((H, Wd, L))
    cuts = [0, 7, 7 + min(100, L - 8), L]
    for l0, l1 in zip(cuts[:-1], cuts[1:]):
        chunk = to_dev(cost[:, :, l0:l1])
        out = torch.empty(chunk.shape, dtype=torch.float32, device=dev())
        g.filter(chunk, l0, out=out, best=best, labels=lab)
        torch.cuda.synchronize()
        Zc[:, :, l0:l1] = out.cpu().numpy()
    g.close()
    np.testing.assert_array_equal(Zc, Zp)
    np.testing.assert_array_equal(lab.cpu().numpy(), labp)


def _sample_points(H, Wd, k, seed):
    rng = np.random.default_rng(seed)
    pts = {(0, 0), (0, Wd - 1), (H - 1, 0), (H - 1, Wd - 1), (H // 2, Wd // 2), (5, Wd - 3),
           (H - 4, 7)}
    while len(pts) < k:
        pts.add((int(rng.integers(0, H)), int(rng.integers(0, Wd))))
    return sorted(pts)


def test_largest_image_sampled(ctx):
    """The largest image of the batched and serving mixes: 1920 x 1080, n = 19,
    256 labels, r = 9 (about 10 GB of coefficient workspace per 64-label
    chunk, so the call runs its labels in several launch groups).  Every
    output is checked by properties that hold at any size; 24 pixels against
    the oracle, each computed exactly from its (4r+1)^2 neighbourhood."""
    w = W("largest_n19_L256", height=1080, width=1920, regions=40, labels=256, radius=9,
          eps=1e-3, degree=3, seed=61)
    say(f"largest image {w.height}x{w.width} n={w.n} L={w.labels}")
    guide, cost = synth.make_workload(w)
    per_chunk = w.pixels * (w.n + 1) * 64 * 4
    assert (12 << 30) // per_chunk < (w.labels + 63) // 64   # several launch groups
    Z, lab = gpu_filter(ctx, guide, cost, w)
    assert np.isfinite(Z).all()
    assert np.array_equal(lab, np.argmin(Z.astype(np.float32), axis=2))
    pts = _sample_points(w.height, w.width, 24, 98)
    Zo = O.filter_points(O.guidance(guide, w.degree, w.basis), cost, w.radius, w.eps, pts)
    idx = tuple(np.array(pts).T)
    check(Z[idx], lab[idx], Zo, cost, w.name + " sampled")


LG = W("launch_groups_n9", height=61, width=77, regions=9, labels=200, radius=4, degree=2,
       seed=60)


def test_launch_groups_match_oracle(ctx):
    """A group size of one 64-label chunk runs the 200 labels in four launch
    groups one after another: bit for bit the one-group call, and the oracle."""
    say("launch groups: 4 groups of one chunk vs one group")
    guide, cost = synth.make_workload(LG)
    Z1, lab1 = gpu_filter(ctx, guide, cost, LG)
    small = hgf.Context(0)
    small.set_group_bytes(LG.height * LG.width * (LG.n + 1) * 64 * 4)
    Zg, labg = gpu_filter(small, guide, cost, LG)
    small.close()
    np.testing.assert_array_equal(Zg, Z1)
    np.testing.assert_array_equal(labg, lab1)
    check(Zg, labg, oracle_filter(guide, cost, LG), cost, "four launch groups")
    # the two-phase form with one chunk of 150 labels: three launch groups in one call
    g = hgf.Guide(ctx, to_dev(guide), labels=LG.labels, radius=LG.radius, eps=LG.eps,
                  degree=LG.degree)
    best = torch.empty((LG.height, LG.width), dtype=torch.float32, device=dev())
    lab = torch.empty((LG.height, LG.width), dtype=torch.int32, device=dev())
    Zc = np.empty_like(Z1)
    for l0, l1 in ((0, 150), (150, 200)):
        out = torch.empty((LG.height, LG.width, l1 - l0), dtype=torch.float32, device=dev())
        g.filter(to_dev(cost[:, :, l0:l1]), l0, out=out, best=best, labels=lab)
        torch.cuda.synchronize()
        Zc[:, :, l0:l1] = out.cpu().numpy()
    g.close()
    np.testing.assert_array_equal(Zc, Z1)
    np.testing.assert_array_equal(lab.cpu().numpy(), lab1)


def test_errors_are_kept_per_context(ctx):
    """hgf_last_error(ctx) holds the detail of that context's last failed call."""
    import ctypes
    lib = hgf.lib()
    other = hgf.Context(0)
    guide, cost = synth.make_workload(CASES[0])
    g, c = to_dev(guide), to_dev(cost)
    ws = torch.empty(1 << 20, dtype=torch.uint8, device=dev())
    H, Wd, L = cost.shape

    def call(c_, **kw):
        p = hgf.make_params(H, Wd, L, **kw)
        return lib.hgf_filter(c_.handle, ctypes.byref(p), g.data_ptr(), c.data_ptr(), None,
                              ws.data_ptr(), ws.data_ptr(), ws.numel(), None)

    assert call(ctx, radius=4, eps=-1.0, degree=1) == hgf.HGF_E_INVALID
    assert call(other, radius=12, eps=1e-3, degree=1) == hgf.HGF_E_UNSUPPORTED
    assert b"eps" in lib.hgf_last_error(ctx.handle)
    assert b"radius=12" in lib.hgf_last_error(other.handle)
    other.close()


def test_nan_costs_do_not_crash(ctx):
    """Non-finite inputs have no defined result (the running sums carry a NaN on
    down the strip), but the call must complete, keep every label in range
    (NaN keys sort above every number) and leave later calls unaffected."""
    w = CASES[0]
    say("nan costs")
    guide, cost = synth.make_workload(w)
    bad = cost.copy()
    bad[5, 7, :] = np.nan
    bad[20, 30, 3] = np.inf
    Z, lab = gpu_filter(ctx, guide, bad, w)
    assert np.all((lab >= 0) & (lab < w.labels))
    Z2, lab2 = gpu_filter(ctx, guide, cost, w)
    check(Z2, lab2, oracle_filter(guide, cost, w), cost, "clean call after non-finite input")


def _random_case(k):
    """A seeded random configuration across the compiled set: guidance
    channels, basis and degree (n <= 19), radius 0..9, ragged sizes from one
    pixel up, label counts around the 64-lane chunks, cost dtype, solve
    precision and regularisation form."""
    rng = np.random.default_rng(4000 + k)
    m = int(rng.integers(1, 4))
    basis = "power" if rng.random() < 0.3 else "monomial"
    while True:
        d = int(rng.integers(1, 7 if basis == "power" else 4))
        n = m * d if basis == "power" else int(np.prod(range(d + 1, d + m + 1)) // np.prod(range(1, m + 1))) - 1
        if n <= 19:
            break
    reg = "ridge" if rng.random() < 0.25 else "covariance"
    cost_dtype = "f32" if reg == "ridge" else str(rng.choice(["f32", "f32", "bf16", "f16"]))
    stats = "f32" if reg == "ridge" else str(rng.choice(["f32", "f64"]))
    if reg == "ridge":
        eps = 0.05
    else:
        eps = 1e-4 if n <= 9 else (1e-3 if n <= 14 else 1e-2)
        if basis == "power" and d >= 4:
            eps = 1e-2
    w = W(f"rand{k}", height=int(rng.integers(1, 61)), width=int(rng.integers(1, 91)),
          guide_channels=m, basis=basis, degree=d,
          labels=int(rng.choice([1, 2, 5, 16, 33, 64, 65, 100, 130])),
          radius=int(rng.integers(0, 10)), eps=eps, cost_dtype=cost_dtype, seed=5000 + k)
    assert w.n == n
    return w, reg, stats


RANDOM = [_random_case(k) for k in range(24)]


@pytest.mark.parametrize("case", RANDOM,
                         ids=[f"{w.name}-n{w.n}-r{w.radius}-L{w.labels}-{w.height}x{w.width}-"
                              f"{reg}-{w.cost_dtype}-{st}" for w, reg, st in RANDOM])
def test_random_configurations_match_oracle(ctx, case):
    w, reg, stats = case
    say(f"random case {w.name}: {w.height}x{w.width} m={w.guide_channels} {w.basis} d={w.degree} "
        f"n={w.n} L={w.labels} r={w.radius} {reg} eps={w.eps} {w.cost_dtype} {stats}")
    guide, cost = synth.make_workload(w)
    Z, lab = gpu_filter(ctx, guide, cost, w, reg=reg, stats_dtype=stats)
    Zo = oracle_filter(guide, cost, w, reg=reg)
    check(Z, lab, Zo, cost, w.name)


RANDOM_SPLIT = [(w, reg, st) for w, reg, st in RANDOM if w.labels >= 2 and w.cost_dtype == "f32"]


@pytest.mark.parametrize("case", RANDOM_SPLIT, ids=[f"{w.name}-L{w.labels}-{reg}-{st}"
                                                    for w, reg, st in RANDOM_SPLIT])
def test_random_label_splits_equal_plain_path(ctx, case):
    """The two-phase form over random label chunks returns the plain call's
    costs and labels bit for bit (results do not depend on label chunking)."""
    w, reg, stats = case
    guide, cost = synth.make_workload(w)
    Zp, labp = gpu_filter(ctx, guide, cost, w, reg=reg, stats_dtype=stats)
    H, Wd, L = cost.shape
    rng = np.random.default_rng(6000 + L + H)
    cuts = sorted(set(int(c) for c in rng.integers(1, L, size=min(3, L - 1))))
    bounds = list(zip([0] + cuts, cuts + [L]))
    say(f"label splits {w.name}: {bounds}")
    g = hgf.Guide(ctx, to_dev(guide), labels=L, radius=w.radius, eps=w.eps, degree=w.degree,
                  basis=w.basis, reg=reg, stats_dtype=stats)
    best = torch.empty((H, Wd), dtype=torch.float32, device=dev())
    lab = torch.empty((H, Wd), dtype=torch.int32, device=dev())
    Zc = np.empty((H, Wd, L))
    for l0, l1 in bounds:
        chunk = to_dev(cost[:, :, l0:l1])
        out = torch.empty(chunk.shape, dtype=torch.float32, device=dev())
        g.filter(chunk, l0, out=out, best=best, labels=lab)
        torch.cuda.synchronize()
        Zc[:, :, l0:l1] = out.cpu().numpy()
    g.close()
    np.testing.assert_array_equal(Zc, Zp)
    np.testing.assert_array_equal(lab.cpu().numpy(), labp)
