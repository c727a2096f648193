"""Parity of the HIP path with the FP64 oracle (run on an MI355X).

Bar: filtered costs within |Z - Z*| <= 1e-4 * max(|Z*|, max|V|) elementwise
(float32 and bfloat16 costs; the bfloat16 cases compare against the oracle on
the same rounded costs), winner-takes-all labels equal wherever the
oracle's two smallest costs differ by at least 1e-5.  Integer box sums are
compared bit for bit.
"""
import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")

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


def gpu_filter(ctx, guide, cost, w, **kw):
    cdt = torch.bfloat16 if w.cost_dtype == "bf16" else torch.float32
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
]


@pytest.mark.parametrize("w", CASES, ids=[c.name for c in CASES])
def test_filter_matches_oracle(ctx, w):
    say(f"case {w.name}: {w.height}x{w.width} n={w.n} L={w.labels} r={w.radius} {w.cost_dtype}")
    guide, cost = synth.make_workload(w)
    Z, lab = gpu_filter(ctx, guide, cost, w)
    Zo = oracle_filter(guide, cost, w)
    check(Z, lab, Zo, cost, w.name)


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


@pytest.mark.parametrize("w", [CASES[1], CASES[2], RIDGE_CASES[0]], ids=["n9", "n19", "ridge_n6"])
def test_guide_statistics_match_oracle(ctx, w):
    reg = "ridge" if w.name.startswith("ridge") else "covariance"
    say(f"guide statistics {w.name} ({reg})")
    guide, _ = synth.make_workload(w)
    g = hgf.Guide(ctx, to_dev(guide), labels=w.labels, radius=w.radius, eps=w.eps,
                  degree=w.degree, basis=w.basis, reg=reg)
    mu, minv, shift = g.export()
    torch.cuda.synchronize()
    # the covariance form stores the float64 inverse rounded to float32
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
# full-size workloads: every output at sampled pixels, computed one by one
# ---------------------------------------------------------------------------

def _sample_points(H, Wd, k, seed):
    rng = np.random.default_rng(seed)
    pts = {(0, 0), (0, Wd - 1), (H - 1, 0), (H - 1, Wd - 1), (H // 2, Wd // 2), (5, Wd - 3),
           (H - 4, 7)}
    while len(pts) < k:
        pts.add((int(rng.integers(0, H)), int(rng.integers(0, Wd))))
    return sorted(pts)


@pytest.mark.parametrize("name", ["voronoi450x375_n9_L60", "voronoi1242x375_n19_L128",
                                  "voronoi1242x375_n19_L128_bf16"])
def test_full_size_sampled(ctx, name):
    w = synth.WORKLOADS[name]
    say(f"full size {name}")
    guide, cost = synth.make_workload(w)
    Z, lab = gpu_filter(ctx, guide, cost, w)
    pts = _sample_points(w.height, w.width, 24, 99)
    G = O.guidance(guide, w.degree, w.basis)
    Zo = O.filter_points(G, cost, w.radius, w.eps, pts)
    idx = tuple(np.array(pts).T)
    check(Z[idx], lab[idx], Zo, cost, name + " sampled")
    # properties that hold at every pixel: labels are the argmin of the returned costs
    assert np.array_equal(lab, np.argmin(Z.astype(np.float32), axis=2))
    assert np.isfinite(Z).all()


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
