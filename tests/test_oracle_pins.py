"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test checks the oracle against an independent statement of the method:
explicit per-window least squares (the definition, Eq. 6 and Sec. 5.1),
the scalar guided-filter closed form (n = 1), invariants of the covariance
form, the eps -> infinity limit, the Woodbury closed form of Prop. 1, and
brute-force loops for the box filter and winner-takes-all.  A dropped term,
a wrong sign or index, or a transposed operand in the oracle fails at least
one of them.
"""
import math

import numpy as np
import pytest

from oracle import hgf_oracle as O


# ----------------------------------------------------------------------------
# brute-force helpers (written here, independent of the oracle's code)
# ----------------------------------------------------------------------------

def _window(H, W, r, y, x):
    return (max(0, y - r), min(H, y + r + 1), max(0, x - r), min(W, x + r + 1))


def _brute_fit(G, V, r, reg, mode):
    """Per-pixel coefficients by explicit least squares over the window's rows.

    covariance mode: min sum (Y - a.G - b)^2 + (reg * N_p) |a|^2 (intercept free);
    ridge mode:      min sum (Y - w0 - w.G)^2 + reg |w|^2 (all n+1 penalised).
    Solved as an augmented least-squares problem with numpy.linalg.lstsq (SVD).
    """
    n, H, W = G.shape
    L = V.shape[2]
    coef = np.zeros((H, W, n + 1, L))
    for y in range(H):
        for x in range(W):
            y0, y1, x0, x1 = _window(H, W, r, y, x)
            X = np.concatenate([np.ones(((y1 - y0) * (x1 - x0), 1)),
                                G[:, y0:y1, x0:x1].reshape(n, -1).T], axis=1)
            Y = V[y0:y1, x0:x1].reshape(-1, L).astype(np.float64)
            Np = X.shape[0]
            if mode == "covariance":
                P = np.concatenate([np.zeros((n, 1)), math.sqrt(reg * Np) * np.eye(n)], axis=1)
            else:
                P = math.sqrt(reg) * np.eye(n + 1)
            A = np.concatenate([X, P], axis=0)
            B = np.concatenate([Y, np.zeros((P.shape[0], L))], axis=0)
            coef[y, x] = np.linalg.lstsq(A, B, rcond=None)[0]
    return coef


def _brute_aggregate(G, coef, r):
    """Z(q) = mean over p in Omega_q of (w_p(0) + sum_i w_p(i) G_i(q)), by explicit loops (Eq. 7)."""
    n, H, W = G.shape
    L = coef.shape[3]
    Z = np.zeros((H, W, L))
    for y in range(H):
        for x in range(W):
            y0, y1, x0, x1 = _window(H, W, r, y, x)
            g = np.concatenate([[1.0], G[:, y, x]])
            acc = np.zeros(L)
            for py in range(y0, y1):
                for px in range(x0, x1):
                    acc += g @ coef[py, px]
            Z[y, x] = acc / ((y1 - y0) * (x1 - x0))
    return Z


def _rand_problem(rng, H, W, m, d, L, basis="monomial"):
    I = rng.uniform(0, 1, size=(m, H, W))
    G = O.guidance(I, d, basis)
    V = rng.uniform(0, 0.5, size=(H, W, L))
    return I, G, V


# ----------------------------------------------------------------------------
# guidance synthesis
# ----------------------------------------------------------------------------

def test_monomial_order_rgb_degree2():
    e = O.guidance_exponents(3, 2, "monomial")
    assert e == [(1, 0, 0), (0, 1, 0), (0, 0, 1), (2, 0, 0), (1, 1, 0), (1, 0, 1),
                 (0, 2, 0), (0, 1, 1), (0, 0, 2)]


def test_monomial_order_rgb_degree3_tail():
    e = O.guidance_exponents(3, 3, "monomial")
    assert len(e) == 19
    assert e[9:] == [(3, 0, 0), (2, 1, 0), (2, 0, 1), (1, 2, 0), (1, 1, 1), (1, 0, 2),
                     (0, 3, 0), (0, 2, 1), (0, 1, 2), (0, 0, 3)]


@pytest.mark.parametrize("m,d", [(1, 1), (1, 4), (3, 1), (3, 2), (3, 3), (2, 5)])
def test_channel_counts(m, d):
    assert O.num_channels(m, d, "monomial") == len(O.guidance_exponents(m, d, "monomial"))
    assert O.num_channels(m, d, "power") == len(O.guidance_exponents(m, d, "power")) == m * d


def test_power_basis_is_paper_map():
    # G_{(i-1)d + j} = I_i^j, channel-major (Sec. 4.2)
    rng = np.random.default_rng(0)
    I = rng.uniform(0, 1, size=(3, 4, 5))
    G = O.guidance(I, 2, "power")
    for i in range(3):
        for j in range(1, 3):
            np.testing.assert_array_equal(G[i * 2 + (j - 1)], I[i] ** j)


def test_monomial_values():
    rng = np.random.default_rng(1)
    I = rng.uniform(0, 1, size=(3, 3, 4))
    G = O.guidance(I, 3, "monomial")
    R, Gc, B = I
    np.testing.assert_allclose(G[4], R * Gc, rtol=0, atol=1e-15)    # RG
    np.testing.assert_allclose(G[13], R * Gc * B, rtol=0, atol=1e-15)  # RGB
    np.testing.assert_allclose(G[18], B ** 3, rtol=0, atol=1e-15)


# ----------------------------------------------------------------------------
# box filter and window counts (Prop. 2, clipped windows)
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("H,W,r", [(1, 1, 0), (1, 1, 3), (5, 7, 1), (6, 4, 2), (3, 9, 5), (8, 8, 0)])
def test_box_sum_bruteforce(H, W, r):
    rng = np.random.default_rng(H * 100 + W * 10 + r)
    X = rng.integers(-50, 50, size=(2, H, W)).astype(np.float64)
    ref = np.zeros_like(X)
    cnt = np.zeros((H, W))
    for y in range(H):
        for x in range(W):
            y0, y1, x0, x1 = _window(H, W, r, y, x)
            ref[:, y, x] = X[:, y0:y1, x0:x1].sum(axis=(1, 2))
            cnt[y, x] = (y1 - y0) * (x1 - x0)
    np.testing.assert_array_equal(O.box_sum(X, r), ref)       # integers: exact
    np.testing.assert_array_equal(O.window_counts(H, W, r), cnt)


# ----------------------------------------------------------------------------
# P1: the whole definition against explicit per-window least squares
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("r", [0, 1, 2, 3])
@pytest.mark.parametrize("m,d", [(1, 1), (3, 1), (3, 2)])
def test_covariance_vs_bruteforce(r, m, d):
    rng = np.random.default_rng(10 * r + m + 100 * d)
    I, G, V = _rand_problem(rng, 7, 9, m, d, 3)
    eps = 1e-2
    Z = O.filter_covariance(G, V, r, eps)
    Zb = _brute_aggregate(G, _brute_fit(G, V, r, eps, "covariance"), r)
    np.testing.assert_allclose(Z, Zb, rtol=1e-9, atol=1e-11)


@pytest.mark.parametrize("r", [0, 1, 3])
@pytest.mark.parametrize("m,d,basis", [(1, 2, "power"), (3, 1, "monomial"), (3, 2, "power")])
def test_ridge_vs_bruteforce(r, m, d, basis):
    rng = np.random.default_rng(7 + r + 10 * d)
    I, G, V = _rand_problem(rng, 6, 8, m, d, 2, basis)
    lam = 0.05
    Z = O.filter_ridge(G, V, r, lam)
    Zb = _brute_aggregate(G, _brute_fit(G, V, r, lam, "ridge"), r)
    np.testing.assert_allclose(Z, Zb, rtol=1e-9, atol=1e-11)


def test_covariance_small_eps_vs_bruteforce():
    # smaller eps, larger conditioning: still the definition to 1e-7 relative
    rng = np.random.default_rng(3)
    I, G, V = _rand_problem(rng, 8, 6, 3, 2, 2)
    Z = O.filter_covariance(G, V, 2, 1e-4)
    Zb = _brute_aggregate(G, _brute_fit(G, V, 2, 1e-4, "covariance"), 2)
    np.testing.assert_allclose(Z, Zb, rtol=1e-7, atol=1e-9)


# ----------------------------------------------------------------------------
# P2: n = 1 is the scalar guided filter (closed form)
# ----------------------------------------------------------------------------

def test_gray_guided_filter_closed_form():
    rng = np.random.default_rng(5)
    H, W, r, eps = 10, 11, 2, 1e-3
    I = rng.uniform(0, 1, size=(H, W))
    Y = rng.uniform(0, 1, size=(H, W))
    a = np.zeros((H, W))
    b = np.zeros((H, W))
    for y in range(H):
        for x in range(W):
            y0, y1, x0, x1 = _window(H, W, r, y, x)
            wi = I[y0:y1, x0:x1]
            wy = Y[y0:y1, x0:x1]
            mi, my = wi.mean(), wy.mean()
            a[y, x] = ((wi * wy).mean() - mi * my) / (wi.var() + eps)
            b[y, x] = my - a[y, x] * mi
    Z = np.zeros((H, W))
    for y in range(H):
        for x in range(W):
            y0, y1, x0, x1 = _window(H, W, r, y, x)
            Z[y, x] = a[y0:y1, x0:x1].mean() * I[y, x] + b[y0:y1, x0:x1].mean()
    Zo = O.filter_covariance(O.guidance(I[None], 1), Y[:, :, None], r, eps)[:, :, 0]
    np.testing.assert_allclose(Zo, Z, rtol=1e-11, atol=1e-13)


# ----------------------------------------------------------------------------
# P3/P4/P5: invariants and limits
# ----------------------------------------------------------------------------

def test_constant_slice_stays_constant_covariance_only():
    rng = np.random.default_rng(6)
    I, G, _ = _rand_problem(rng, 9, 10, 3, 2, 1)
    V = np.full((9, 10, 2), 0.37)
    Zc = O.filter_covariance(G, V, 2, 1e-4)
    np.testing.assert_allclose(Zc, 0.37, rtol=0, atol=1e-12)
    Zr = O.filter_ridge(G, V, 2, 0.05)
    # the ridge form penalises the intercept, so a constant is shrunk: the two forms differ
    assert np.max(np.abs(Zr - 0.37)) > 1e-5


def test_guidance_channel_reproduced_for_small_eps():
    rng = np.random.default_rng(7)
    I, G, _ = _rand_problem(rng, 12, 11, 3, 1, 1)
    V = np.stack([G[1], 0.3 * G[0] - 0.7 * G[2] + 0.2], axis=2)
    Z = O.filter_covariance(G, V, 2, 1e-9)
    np.testing.assert_allclose(Z, V, rtol=0, atol=2e-5)


def test_large_eps_is_double_box_mean():
    rng = np.random.default_rng(8)
    I, G, V = _rand_problem(rng, 9, 7, 3, 2, 2)
    r = 2
    Z = O.filter_covariance(G, V, r, 1e12)
    H, W = 9, 7
    A1 = np.zeros((H, W, 2))
    for y in range(H):
        for x in range(W):
            y0, y1, x0, x1 = _window(H, W, r, y, x)
            A1[y, x] = V[y0:y1, x0:x1].reshape(-1, 2).mean(axis=0)
    A2 = np.zeros_like(A1)
    for y in range(H):
        for x in range(W):
            y0, y1, x0, x1 = _window(H, W, r, y, x)
            A2[y, x] = A1[y0:y1, x0:x1].reshape(-1, 2).mean(axis=0)
    np.testing.assert_allclose(Z, A2, rtol=0, atol=1e-10)


# ----------------------------------------------------------------------------
# P6/P7: linearity, slice independence, symmetries
# ----------------------------------------------------------------------------

def test_linearity_and_slice_independence():
    rng = np.random.default_rng(9)
    I, G, V1 = _rand_problem(rng, 10, 9, 3, 2, 3)
    V2 = rng.uniform(-1, 1, size=V1.shape)
    r, eps = 2, 1e-3
    Z = O.filter_covariance(G, 0.3 * V1 - 1.7 * V2, r, eps)
    np.testing.assert_allclose(Z, 0.3 * O.filter_covariance(G, V1, r, eps)
                               - 1.7 * O.filter_covariance(G, V2, r, eps), rtol=0, atol=1e-11)
    for l in range(3):
        Zl = O.filter_covariance(G, V1[:, :, l:l + 1], r, eps)[:, :, 0]
        np.testing.assert_allclose(O.filter_covariance(G, V1, r, eps)[:, :, l], Zl, rtol=0, atol=1e-12)


def test_channel_translation_and_permutation_invariance():
    rng = np.random.default_rng(10)
    I, G, V = _rand_problem(rng, 9, 8, 3, 2, 2)
    r, eps = 2, 1e-3
    Z = O.filter_covariance(G, V, r, eps)
    shift = rng.uniform(-3, 3, size=(G.shape[0], 1, 1))
    np.testing.assert_allclose(O.filter_covariance(G + shift, V, r, eps), Z, rtol=0, atol=1e-10)
    perm = rng.permutation(G.shape[0])
    np.testing.assert_allclose(O.filter_covariance(G[perm], V, r, eps), Z, rtol=0, atol=1e-11)


def test_transpose_and_flip_equivariance():
    rng = np.random.default_rng(11)
    I, G, V = _rand_problem(rng, 9, 6, 3, 1, 2)
    r, eps = 2, 1e-3
    Z = O.filter_covariance(G, V, r, eps)
    Zt = O.filter_covariance(G.transpose(0, 2, 1), V.transpose(1, 0, 2), r, eps)
    np.testing.assert_allclose(Zt, Z.transpose(1, 0, 2), rtol=0, atol=1e-12)
    Zf = O.filter_covariance(G[:, ::-1, :], V[::-1], r, eps)
    np.testing.assert_allclose(Zf, Z[::-1], rtol=0, atol=1e-12)


def test_shift_of_cost_is_equivariant():
    rng = np.random.default_rng(12)
    I, G, V = _rand_problem(rng, 8, 8, 3, 2, 2)
    Z = O.filter_covariance(G, V, 2, 1e-4)
    np.testing.assert_allclose(O.filter_covariance(G, V + 5.0, 2, 1e-4), Z + 5.0, rtol=0, atol=1e-10)


# ----------------------------------------------------------------------------
# P8: Prop. 1 against the Woodbury closed form; readout Eq. 5
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("n1,N,lam", [(1, 9, 0.05), (4, 25, 0.05), (10, 361, 0.05), (20, 81, 1e-2)])
def test_prop1_alpha_is_scaled_inverse(n1, N, lam):
    rng = np.random.default_rng(n1 + N)
    X = np.concatenate([np.ones((N, 1)), rng.uniform(0, 1, size=(N, n1 - 1))], axis=1)
    K = X.T @ X
    alpha = O.prop1_alpha(K, lam)
    closed = -np.linalg.inv(lam * np.eye(n1) + K) / lam
    np.testing.assert_allclose(alpha, closed, rtol=1e-9, atol=1e-12 * np.abs(closed).max())
    # the |Omega|-space statement of Prop. 1 itself
    lhs = np.linalg.inv(lam * np.eye(N) + X @ X.T)
    rhs = np.eye(N) / lam + X @ alpha @ X.T
    np.testing.assert_allclose(rhs, lhs, rtol=0, atol=1e-9 * np.abs(lhs).max())


def test_prop1_printed_base_case_is_off():
    rng = np.random.default_rng(13)
    X = np.concatenate([np.ones((25, 1)), rng.uniform(0, 1, size=(25, 3))], axis=1)
    K = X.T @ X
    lam = 0.05
    closed = -np.linalg.inv(lam * np.eye(4) + K) / lam
    printed = O.prop1_alpha(K, lam, printed_base_case=True)
    assert np.max(np.abs(printed - closed)) > 0.1 * np.abs(closed).max()


def test_prop1_scalar_case():
    # n = 0: the window regression reduces to w0 = S_Y / (lambda + N)
    lam, N, SY = 0.05, 225.0, 1.0
    alpha = O.prop1_alpha(np.array([[N]]), lam)
    w = O.prop1_readout(np.array([[N]]), np.array([SY]), lam, alpha)
    assert abs(w[0] - SY / (lam + N)) < 1e-15


def test_prop1_readout_solves_ridge():
    rng = np.random.default_rng(14)
    X = np.concatenate([np.ones((49, 1)), rng.uniform(0, 1, size=(49, 6))], axis=1)
    y = rng.uniform(0, 1, size=49)
    lam = 0.05
    K = X.T @ X
    b = X.T @ y
    w = O.prop1_readout(K, b, lam, O.prop1_alpha(K, lam))
    ref = np.linalg.lstsq(np.concatenate([X, math.sqrt(lam) * np.eye(7)]),
                          np.concatenate([y, np.zeros(7)]), rcond=None)[0]
    np.testing.assert_allclose(w, ref, rtol=1e-8, atol=1e-10)


# ----------------------------------------------------------------------------
# guide statistics, sampled points, WTA
# ----------------------------------------------------------------------------

def test_guide_statistics_inverse():
    rng = np.random.default_rng(15)
    I = rng.uniform(0, 1, size=(3, 6, 7))
    mu, M = O.guide_statistics(I, 2, 1, 1e-3)
    G = O.guidance(I, 2)
    y, x = 2, 3
    win = G[:, 1:4, 2:5].reshape(9, -1)
    np.testing.assert_allclose(mu[y, x], win.mean(axis=1), rtol=1e-13)
    S = np.cov(win, bias=True) + 1e-3 * np.eye(9)
    np.testing.assert_allclose(M[y, x] @ S, np.eye(9), atol=1e-9)


def test_filter_points_match_full():
    rng = np.random.default_rng(16)
    I, G, V = _rand_problem(rng, 23, 29, 3, 2, 3)
    r, eps = 3, 1e-3
    Z = O.filter_covariance(G, V, r, eps)
    pts = [(0, 0), (22, 28), (11, 14), (3, 27), (20, 1)]
    np.testing.assert_allclose(O.filter_points(G, V, r, eps, pts), Z[tuple(np.array(pts).T)],
                               rtol=0, atol=1e-12)
    Zr = O.filter_ridge(G, V, r, 0.05)
    np.testing.assert_allclose(O.filter_points(G, V, r, 0.05, pts, mode="ridge"),
                               Zr[tuple(np.array(pts).T)], rtol=0, atol=1e-12)


@pytest.mark.parametrize("mode,r,tiles", [("covariance", 3, (2, 1)), ("ridge", 1, (3, 2)), ("covariance", 1, (1, 1))])
def test_banded_oracle_equals_whole_image(mode, r, tiles):
    """The tile driver (output tiles with a 2r halo, in spawned worker processes)
    reproduces the whole-image oracle: the locality argument of Eq. 7 /
    Eq. 11 (an output row needs coefficients within r, which need inputs
    within r) holds exactly, clipped windows included."""
    from oracle import banded
    rng = np.random.default_rng(7 + r)
    I = rng.uniform(0, 1, size=(3, 23, 17))
    G = O.guidance(I, 2)
    V = rng.uniform(0, 1, size=(23, 17, 5))
    full = O.filter_covariance(G, V, r, 1e-3) if mode == "covariance" else O.filter_ridge(G, V, r, 0.05)
    Zb = banded.filter_image(G, V, r, 1e-3 if mode == "covariance" else 0.05, mode=mode,
                             tiles=tiles, workers=2, label_chunk=2)
    np.testing.assert_allclose(Zb, full, rtol=0, atol=1e-12)


def test_wta_lowest_label_on_ties_and_near_tie_mask():
    Z = np.array([[[3.0, 1.0, 1.0, 2.0], [0.5, 0.5, 0.1, 0.1]]])
    np.testing.assert_array_equal(O.wta(Z), [[1, 2]])
    Z2 = np.array([[[1.0, 1.0 + 2e-6, 3.0], [1.0, 1.1, 0.0]]])
    np.testing.assert_array_equal(O.near_tie_mask(Z2), [[True, False]])


def test_condition_number_bound_small_workload():
    # P12: cond(Sigma_p + eps E) <= (trace bound + eps) / eps on the small colour workload
    from paper_1803_00005_amd.synth import WORKLOADS, make_workload
    w = WORKLOADS["rgb64_n3_L16"]
    I, _ = make_workload(w)
    mu, M = O.guide_statistics(I, w.degree, w.radius, w.eps)
    ev = np.linalg.eigvalsh(np.linalg.inv(M))
    cond = ev[..., -1] / ev[..., 0]
    G = O.guidance(I, w.degree)
    bound = (np.sum((G.max(axis=(1, 2)) - G.min(axis=(1, 2))) ** 2) / 4 + w.eps) / w.eps
    assert np.all(cond <= bound)
    assert np.all(ev[..., 0] >= w.eps * (1 - 1e-9))


# ----------------------------------------------------------------------------
# regression fixtures (written by tests/golden/make_golden.py from the oracle)
# ----------------------------------------------------------------------------

def test_golden_regression_fixtures():
    import os
    import sys
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    sys.path.insert(0, here)
    try:
        import make_golden
    finally:
        sys.path.pop(0)
    for name, Z in make_golden.cases():
        ref = np.loadtxt(os.path.join(here, name)).reshape(Z.shape)
        np.testing.assert_allclose(Z, ref, rtol=1e-13, atol=1e-15)
