"""FP64 CPU oracle for the hardware-efficient guided filter (HGF).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this module: only the tests, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` use it.  It shares no code with the HIP path.

What it computes (paper: "Hardware-Efficient Guided Image Filtering For
Multi-Label Problem", Dai et al., arXiv 1803.00005):

* Polynomial guidance G_1..G_n synthesized from the input guidance I
  (Sec. 4.2, Eqs. 8 and the colour form that follows it).  Two bases:
  ``"power"`` is the paper's per-channel map G_{(i-1)d+j} = I_i^j (n = m d);
  ``"monomial"`` is every monomial of total degree 1..d of the m channels in
  graded lexicographic order (n = C(m+d, d) - 1), the polynomial space a
  degree-d colour model spans.
* Box filter B (Prop. 2): the sum over the square window of side 2r+1
  centred at p, clipped to the image.  The window count N_p = B(1)(p) is the
  normaliser of the average operator A(X) = B(X)/B(G_0) (Sec. 4.3, Eq. 11).
* Covariance (guided-filter) form, intercept left free (Sec. 5.1, Eqs. 12-13):
  per pixel p, solve (Sigma_p + eps E) a_p = c_p with the window covariance
  Sigma_p of the guidance and the window covariance c_p of guidance and cost
  slice, then b_p = ybar_p - a_p^T mu_p.  Solved by LU with partial pivoting
  (LAPACK gesv through ``numpy.linalg.solve``) in FP64.
* Ridge form, every coefficient penalised (Sec. 4.1, Eq. 6, closed form
  Eq. 2): (lambda E + X^T X) w_p = X^T Y over the window rows X = [1, G(q)].
* Aggregation (Sec. 4.1, Eq. 7; Eq. 11): Z(q) is the mean over p in Omega_q
  of the window-p prediction at q, i.e. Z = A(a) . G + A(b).
* Winner-takes-all (Sec. 1): label(q) = argmin_l Z_l(q), lowest label on ties.
* Prop. 1: the recursive Sherman-Morrison coefficients alpha, with the base
  case read as alpha^0_00 = -1 / (lambda (lambda + G_00)) (the printed base
  case lacks the 1/lambda factor; the derivation from the Sherman-Morrison
  formula that the proof names gives this one).

Arrays: guidance ``I`` is [m][H][W]; cost ``V`` is [H][W][L]; outputs Z are
[H][W][L] float64, labels [H][W] int64.
"""
from __future__ import annotations

import itertools
import math
from typing import Iterable, Sequence

import numpy as np

__all__ = [
    "num_channels",
    "guidance_exponents",
    "guidance",
    "window_counts",
    "box_sum",
    "guide_statistics",
    "filter_covariance",
    "filter_ridge",
    "filter_points",
    "wta",
    "near_tie_mask",
    "prop1_alpha",
    "prop1_readout",
    "lu_inverse",
]


# ----------------------------------------------------------------------------
# Polynomial guidance (Sec. 4.2)
# ----------------------------------------------------------------------------

def guidance_exponents(m: int, d: int, basis: str = "monomial") -> list[tuple[int, ...]]:
    """Exponent tuples (e_1..e_m) of the n guidance channels, in channel order.

    ``power``: the paper's map G_{(i-1)d+j} = I_i^j, channel-major.
    ``monomial``: all monomials of total degree 1..d, graded, and within a
    degree lexicographic with channel 1 first (for RGB and d=2:
    R, G, B, R^2, RG, RB, G^2, GB, B^2).
    """
    if m < 1 or d < 1:
        raise ValueError("m and d must be >= 1")
    out: list[tuple[int, ...]] = []
    if basis == "power":
        for i in range(m):
            for j in range(1, d + 1):
                e = [0] * m
                e[i] = j
                out.append(tuple(e))
        return out
    if basis != "monomial":
        raise ValueError(f"unknown basis {basis!r}")
    for k in range(1, d + 1):
        for combo in itertools.combinations_with_replacement(range(m), k):
            e = [0] * m
            for c in combo:
                e[c] += 1
            out.append(tuple(e))
    return out


def num_channels(m: int, d: int, basis: str = "monomial") -> int:
    """n, the number of synthesized guidance channels (the constant G_0 excluded)."""
    if basis == "power":
        return m * d
    return math.comb(m + d, d) - 1


def guidance(I: np.ndarray, d: int, basis: str = "monomial") -> np.ndarray:
    """G_1..G_n as a float64 array [n][H][W]."""
    I = np.asarray(I, dtype=np.float64)
    if I.ndim == 2:
        I = I[None]
    m = I.shape[0]
    exps = guidance_exponents(m, d, basis)
    G = np.empty((len(exps),) + I.shape[1:], dtype=np.float64)
    for k, e in enumerate(exps):
        g = np.ones(I.shape[1:], dtype=np.float64)
        for c, p in enumerate(e):
            for _ in range(p):
                g = g * I[c]
        G[k] = g
    return G


# ----------------------------------------------------------------------------
# Box filter (Prop. 2) with clipped windows
# ----------------------------------------------------------------------------

def window_counts(H: int, W: int, r: int) -> np.ndarray:
    """N_p = |Omega_p| for the clipped (2r+1) x (2r+1) window, float64 [H][W]."""
    x = np.arange(W)
    y = np.arange(H)
    nx = np.minimum(x + r, W - 1) - np.maximum(x - r, 0) + 1
    ny = np.minimum(y + r, H - 1) - np.maximum(y - r, 0) + 1
    return (ny[:, None] * nx[None, :]).astype(np.float64)


def _box_axis(X: np.ndarray, r: int, axis: int) -> np.ndarray:
    n = X.shape[axis]
    c = np.cumsum(X, axis=axis, dtype=np.float64)
    zero_shape = list(X.shape)
    zero_shape[axis] = 1
    c = np.concatenate([np.zeros(zero_shape), c], axis=axis)
    idx = np.arange(n)
    hi = np.minimum(idx + r, n - 1) + 1
    lo = np.maximum(idx - r, 0)
    return np.take(c, hi, axis=axis) - np.take(c, lo, axis=axis)


def box_sum(X: np.ndarray, r: int) -> np.ndarray:
    """B(X): sum over the clipped square window of radius r, over the last two axes (H, W)."""
    X = np.asarray(X, dtype=np.float64)
    return _box_axis(_box_axis(X, r, X.ndim - 1), r, X.ndim - 2)


# ----------------------------------------------------------------------------
# Guidance statistics and the per-pixel inverse
# ----------------------------------------------------------------------------

def _window_moments(G: np.ndarray, r: int):
    """mu_p (n,H,W) and Sigma_p (H,W,n,n): window mean and covariance of G."""
    n, H, W = G.shape
    N = window_counts(H, W, r)
    mu = box_sum(G, r) / N
    Sigma = np.empty((H, W, n, n), dtype=np.float64)
    for i in range(n):
        for j in range(i, n):
            s = box_sum(G[i] * G[j], r) / N - mu[i] * mu[j]
            Sigma[:, :, i, j] = s
            Sigma[:, :, j, i] = s
    return N, mu, Sigma


def lu_inverse(A: np.ndarray) -> np.ndarray:
    """Inverse of each trailing square matrix by LU with partial pivoting (LAPACK getrf/getri)."""
    return np.linalg.inv(np.asarray(A, dtype=np.float64))


def guide_statistics(I: np.ndarray, d: int, r: int, eps: float, basis: str = "monomial"):
    """Per-pixel window mean mu_p [H][W][n] and inverse M_p = (Sigma_p + eps E)^-1 [H][W][n][n].

    The guidance part of the covariance form (Sec. 5.1); precomputed once per
    image and shared by every label slice (Sec. 5.3, the all-pair box filters
    computed once).
    """
    G = guidance(I, d, basis)
    n = G.shape[0]
    _, mu, Sigma = _window_moments(G, r)
    M = lu_inverse(Sigma + eps * np.eye(n))
    return np.ascontiguousarray(mu.transpose(1, 2, 0)), M


# ----------------------------------------------------------------------------
# The filter
# ----------------------------------------------------------------------------

def _label_chunk(n: int, H: int, W: int, L: int) -> int:
    per_label = (n + 4) * H * W * 8 * 4
    return int(max(1, min(L, (512 << 20) // max(1, per_label))))


def _solve_pixels(A: np.ndarray, B: np.ndarray, pixel_chunk: int = 32768) -> np.ndarray:
    """Solve A_p x_p = B_p for every pixel p: A (P, k, k), B (P, k, Lc), LU with partial pivoting."""
    out = np.empty_like(B)
    for p0 in range(0, A.shape[0], pixel_chunk):
        p1 = min(A.shape[0], p0 + pixel_chunk)
        out[p0:p1] = np.linalg.solve(A[p0:p1], B[p0:p1])
    return out


def filter_covariance(G: np.ndarray, V: np.ndarray, r: int, eps: float,
                      label_chunk: int | None = None) -> np.ndarray:
    """Covariance-form filter of every label slice of V under guidance G.

    G: [n][H][W] guidance channels (already synthesized); V: [H][W][L].
    Returns Z [H][W][L] float64.  Follows Sec. 5.1 (Eqs. 12-13: intercept
    free, eps on the window covariance) for the per-window fit and Sec. 4.1
    (Eq. 7) / Eq. 11 for the aggregation.
    """
    G = np.asarray(G, dtype=np.float64)
    n, H, W = G.shape
    V = np.asarray(V)
    if V.shape[:2] != (H, W):
        raise ValueError("cost and guidance sizes differ")
    L = V.shape[2]
    N, mu, Sigma = _window_moments(G, r)
    A = (Sigma + eps * np.eye(n)).reshape(H * W, n, n)
    mu_flat = mu.reshape(n, H * W).T                      # (P, n)
    Z = np.empty((H, W, L), dtype=np.float64)
    lc = label_chunk or _label_chunk(n, H, W, L)
    for l0 in range(0, L, lc):
        l1 = min(L, l0 + lc)
        Y = np.ascontiguousarray(np.asarray(V[:, :, l0:l1], dtype=np.float64).transpose(2, 0, 1))
        ybar = box_sum(Y, r) / N                          # (Lc, H, W)
        c = box_sum(G[:, None] * Y[None], r) / N          # (n, Lc, H, W)
        c -= mu[:, None] * ybar[None]
        rhs = c.reshape(n, l1 - l0, H * W).transpose(2, 0, 1)   # (P, n, Lc)
        a = _solve_pixels(A, np.ascontiguousarray(rhs))          # (P, n, Lc)
        b = ybar.reshape(l1 - l0, H * W).T - np.einsum("pnl,pn->pl", a, mu_flat)
        a_img = a.transpose(1, 2, 0).reshape(n, l1 - l0, H, W)
        b_img = b.T.reshape(l1 - l0, H, W)
        out = box_sum(b_img, r)
        out += np.einsum("nlhw,nhw->lhw", box_sum(a_img, r), G)
        Z[:, :, l0:l1] = (out / N).transpose(1, 2, 0)
    return Z


def filter_ridge(G: np.ndarray, V: np.ndarray, r: int, lam: float,
                 label_chunk: int | None = None) -> np.ndarray:
    """Ridge form of the paper (Eq. 6): every coefficient, intercept included, penalised by lambda.

    K_p = B(G_i G_j) over i, j = 0..n with G_0 = 1 (Prop. 2), right-hand side
    B(G_i Y); w_p = (lambda E + K_p)^-1 B(G Y) (Eq. 2); Z = A(W_0) + sum_i A(W_i) G_i (Eq. 11).
    """
    G = np.asarray(G, dtype=np.float64)
    n, H, W = G.shape
    L = V.shape[2]
    N = window_counts(H, W, r)
    G1 = np.concatenate([np.ones((1, H, W)), G], axis=0)  # (n+1, H, W)
    K = np.empty((H, W, n + 1, n + 1), dtype=np.float64)
    for i in range(n + 1):
        for j in range(i, n + 1):
            s = box_sum(G1[i] * G1[j], r)
            K[:, :, i, j] = s
            K[:, :, j, i] = s
    A = (K + lam * np.eye(n + 1)).reshape(H * W, n + 1, n + 1)
    Z = np.empty((H, W, L), dtype=np.float64)
    lc = label_chunk or _label_chunk(n + 1, H, W, L)
    for l0 in range(0, L, lc):
        l1 = min(L, l0 + lc)
        Y = np.ascontiguousarray(np.asarray(V[:, :, l0:l1], dtype=np.float64).transpose(2, 0, 1))
        rhs = box_sum(G1[:, None] * Y[None], r)           # (n+1, Lc, H, W)
        rhs = rhs.reshape(n + 1, l1 - l0, H * W).transpose(2, 0, 1)
        w = _solve_pixels(A, np.ascontiguousarray(rhs))   # (P, n+1, Lc)
        w_img = w.transpose(1, 2, 0).reshape(n + 1, l1 - l0, H, W)
        Bw = box_sum(w_img, r)
        out = Bw[0] + np.einsum("nlhw,nhw->lhw", Bw[1:], G)
        Z[:, :, l0:l1] = (out / N).transpose(1, 2, 0)
    return Z


def filter_points(G: np.ndarray, V: np.ndarray, r: int, eps: float,
                  points: Iterable[Sequence[int]], mode: str = "covariance") -> np.ndarray:
    """Z at selected pixels only, each computed exactly from the (4r+1)^2 neighbourhood it depends on.

    Z(q) uses (a_p, b_p) for p in Omega_q, and those use pixels within r of
    p, so every window involved lies inside the crop [q - 2r, q + 2r] clipped
    to the image, and is clipped there exactly as in the full image.
    Returns float64 [len(points)][L].
    """
    G = np.asarray(G)
    n, H, W = G.shape
    out = []
    for (qy, qx) in points:
        y0, y1 = max(0, qy - 2 * r), min(H, qy + 2 * r + 1)
        x0, x1 = max(0, qx - 2 * r), min(W, qx + 2 * r + 1)
        Gc = G[:, y0:y1, x0:x1]
        Vc = V[y0:y1, x0:x1]
        if mode == "covariance":
            Zc = filter_covariance(Gc, Vc, r, eps)
        else:
            Zc = filter_ridge(Gc, Vc, r, eps)
        out.append(Zc[qy - y0, qx - x0])
    return np.asarray(out)


def wta(Z: np.ndarray) -> np.ndarray:
    """label(q) = argmin_l Z_l(q); numpy's argmin keeps the first, i.e. lowest, label on ties."""
    return np.argmin(Z, axis=-1)


def near_tie_mask(Z: np.ndarray, gap: float = 1e-5) -> np.ndarray:
    """Pixels whose two smallest costs differ by less than ``gap`` (WTA may legitimately differ there)."""
    if Z.shape[-1] < 2:
        return np.zeros(Z.shape[:-1], dtype=bool)
    two = np.partition(Z, 1, axis=-1)[..., :2]
    return (two[..., 1] - two[..., 0]) < gap


# ----------------------------------------------------------------------------
# Prop. 1: the recursive Sherman-Morrison coefficients
# ----------------------------------------------------------------------------

def prop1_alpha(gram: np.ndarray, lam: float, printed_base_case: bool = False) -> np.ndarray:
    """alpha_ij of Prop. 1 for the Gram matrix G_ij = c_i^T c_j, i, j = 0..n.

    (lambda E + sum_i c_i c_i^T)^-1 = lambda^-1 E + sum_ij alpha_ij c_i c_j^T.
    The recursion runs kappa = 1..n: with beta = alpha^{k-1} g, g_m = G_{m kappa},
    gamma = -(1 + G_kk / lambda + g^T alpha^{k-1} g)^-1,
      alpha_ij <- alpha_ij + gamma beta_i beta_j   (i, j < kappa; F_ij = beta_i beta_j),
      alpha_i,kappa = alpha_kappa,i = gamma beta_i / lambda,
      alpha_kappa,kappa = gamma / lambda^2.
    Base case alpha_00 = -1 / (lambda (lambda + G_00)); ``printed_base_case``
    uses the form printed in the paper, -1 / (lambda + G_00), to show it is off.
    """
    K = np.asarray(gram, dtype=np.float64)
    n1 = K.shape[0]
    alpha = np.zeros((n1, n1), dtype=np.float64)
    if printed_base_case:
        alpha[0, 0] = -1.0 / (lam + K[0, 0])
    else:
        alpha[0, 0] = -1.0 / (lam * (lam + K[0, 0]))
    for k in range(1, n1):
        prev = alpha[:k, :k].copy()
        g = K[:k, k]
        beta = prev @ g
        gamma = -1.0 / (1.0 + K[k, k] / lam + g @ beta)
        alpha[:k, :k] = prev + gamma * np.outer(beta, beta)
        alpha[:k, k] = gamma * beta / lam
        alpha[k, :k] = gamma * beta / lam
        alpha[k, k] = gamma / (lam * lam)
    return alpha


def prop1_readout(gram: np.ndarray, rhs: np.ndarray, lam: float, alpha: np.ndarray) -> np.ndarray:
    """Eq. 5: w(k) = lambda^-1 G_{k,n+1} + sum_ij alpha_ij G_ki G_{j,n+1}, with rhs_j = G_{j,n+1}."""
    K = np.asarray(gram, dtype=np.float64)
    b = np.asarray(rhs, dtype=np.float64)
    return b / lam + K @ (alpha @ b)
