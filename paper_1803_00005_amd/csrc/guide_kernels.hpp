// Guidance statistics kernels, instantiated per channel count n in generated
// units (all radii and solve modes of one n per unit):
//   a2  window sums of G_i and G_i G_j (Prop. 2),
//   a3  per-pixel inverse of the regularised window system by the recursion
//       of Prop. 1 (bordering form, branch-free: every Schur complement is
//       at least the regulariser, so no pivot is ever needed).
// The dense batched SPD inverse of the Fig. 1(a) comparison shares the
// quad-lane recursion.
#pragma once

#include <type_traits>

#include "hgf_launch.hpp"

namespace hgf {
namespace gk {

// ---------------------------------------------------------------------------
// a2: window sums of the K = n + n(n+1)/2 guidance moments, float64, with
// vertical running sums (add the row entering the window, subtract the row
// leaving it) and horizontal running sums over strips of 64 state columns.
// The lanes of a wave are the 64 state columns of the strip during the
// vertical update: a lane loads the n guidance values of
// its column of the entering and the leaving row (a few contiguous loads, all
// in flight together) and updates the float64 running sums of the moments of
// that column.  Each of the block's waves holds KW consecutive moments (two
// waves up to nine channels, eight above; the waves read the same columns,
// from L1).  The sums then pass through LDS, transposed to lanes = moments,
// for the horizontal running sums and the coalesced stores of S[p][k]; the
// output columns are split into up to four parts summed by separate threads.
// Up to n = kFuseMaxN a row's window sums stay in LDS instead, and the kernel
// also computes each output pixel's inverse (a3).

// coef times the moments [K0, K0 + KW) of g (g_k, then g_i g_j, i <= j, in
// the packed order) added to the running sums vs[k - K0]
template <int NG, int K0, int KW>
__device__ __forceinline__ void add_moments(double (&vs)[KW], const double (&g)[NG], double coef) {
#pragma unroll
  for (int i = 0; i < NG; ++i)
    if (i >= K0 && i < K0 + KW) vs[i - K0] = fma(coef, g[i], vs[i - K0]);
#pragma unroll
  for (int i = 0; i < NG; ++i) {
    const double ci = coef * g[i];
#pragma unroll
    for (int j = i; j < NG; ++j) {
      const int k = NG + packed_index(i, j, NG);
      if (k >= K0 && k < K0 + KW) vs[k - K0] = fma(ci, g[j], vs[k - K0]);
    }
  }
}

// ---------------------------------------------------------------------------
// a3 for one pixel: from its window sums s (the K moments), its window count
// Np and the regulariser, the window means mu (covariance form; zero in the
// ridge form) and the packed inverse M of the regularised D x D system, by
// the bordering recursion described with invert_kernel below.  Used by the
// inverse kernels and by the moment kernel with the inverse fused in.
// ---------------------------------------------------------------------------
template <int D, int MODE>
__device__ __forceinline__ void pixel_inverse(const double* __restrict__ s, double Np, double eps,
                                              double (&mu)[MODE == kSolveRidge ? D - 1 : D],
                                              double (&M)[D * (D + 1) / 2]) {
  constexpr bool RIDGE = MODE == kSolveRidge;
  constexpr int NG = RIDGE ? D - 1 : D;
  const double invN = 1.0 / Np;
#pragma unroll
  for (int i = 0; i < NG; ++i) mu[i] = RIDGE ? 0.0 : s[i] * invN;

  // entry (i, j), i <= j, of the regularised system
  auto A = [&](int i, int j) -> double {
    if (!RIDGE) {
      return fma(s[NG + packed_index(i, j, NG)], invN, -mu[i] * mu[j]) + (i == j ? eps : 0.0);
    }
    if (i == 0) return (j == 0) ? Np + eps : s[j - 1];
    return s[NG + packed_index(i - 1, j - 1, NG)] + (i == j ? eps : 0.0);
  };

  M[0] = 1.0 / A(0, 0);
#pragma unroll
  for (int kap = 1; kap < D; ++kap) {
    double g[D];
    double u[D];
#pragma unroll
    for (int i = 0; i < kap; ++i) g[i] = A(i, kap);
#pragma unroll
    for (int i = 0; i < kap; ++i) {
      double acc = 0.0;
#pragma unroll
      for (int j = 0; j < kap; ++j)
        acc = fma(M[i <= j ? packed_index(i, j, D) : packed_index(j, i, D)], g[j], acc);
      u[i] = acc;
    }
    double schur = A(kap, kap);
#pragma unroll
    for (int i = 0; i < kap; ++i) schur = fma(-g[i], u[i], schur);
    const double inv = 1.0 / schur;
#pragma unroll
    for (int i = 0; i < kap; ++i) {
      const double ui = u[i] * inv;
#pragma unroll
      for (int j = i; j < kap; ++j) M[packed_index(i, j, D)] = fma(ui, u[j], M[packed_index(i, j, D)]);
      M[packed_index(i, kap, D)] = -ui;
    }
    M[packed_index(kap, kap, D)] = inv;
  }
}

// Channel counts whose moment kernel also computes the inverse, so that the
// window sums need not go through HBM: up to n = 9 the inverse (at most 55
// doubles of M) fits beside the moment sums in the registers; above, the
// quad-spread inverse kernel takes over.
constexpr int kFuseMaxN = 9;

// The system size of a solve mode for n guidance channels.
constexpr int system_size(int mode, int n) { return mode == kSolveRidge ? n + 1 : n; }

//
// FUSE < 0: the window sums go to S.  FUSE = a solve mode (n <= kFuseMaxN):
// a row's window sums stay in LDS and one thread per output pixel computes
// its inverse and stores the record and window means, as invert_kernel would.
template <int R, int NG, int KW, int FUSE>
__global__ __launch_bounds__((NG + NG * (NG + 1) / 2 + KW - 1) / KW * 64) void moments_kernel(
    const double* __restrict__ g64, int H, int W, int band_h, int strips,
    double* __restrict__ S, double eps, double* __restrict__ mu_out,
    void* __restrict__ minv_void) {
  constexpr int K = NG + NG * (NG + 1) / 2;
  constexpr int NWM = (K + KW - 1) / KW;  // waves of the block
  constexpr int SOUT = kStrip - 2 * R;
  constexpr int TS = kStrip + 1;  // LDS row stride of the transpose (doubles)
  // parts of the output columns summed by separate threads
  constexpr int NSPLIT = (NWM * 64) / K < 1 ? 1 : ((NWM * 64) / K > 4 ? 4 : (NWM * 64) / K);
  constexpr int JC = (SOUT + NSPLIT - 1) / NSPLIT;
  __shared__ double tr[K * TS];
  // the fused form's window sums of one output row, [SOUT][K]
  __shared__ double sp[FUSE >= 0 ? SOUT * K : 1];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
  const int bid = xcd_remap(static_cast<int>(blockIdx.x), static_cast<int>(gridDim.x));
  const int strip = __builtin_amdgcn_readfirstlane(bid % strips);
  const int band = __builtin_amdgcn_readfirstlane(bid / strips);
  const int x_out0 = strip * SOUT;
  const int xs = x_out0 - R;
  const int y0 = band * band_h;
  const int y1 = min(H, y0 + band_h);
  // this lane's state column; outside the image it reads a clamped column
  // with weight 0
  const int xr = xs + lane;
  const int xc = min(max(xr, 0), W - 1);
  const double w = (xr >= 0 && xr < W) ? 1.0 : 0.0;

  double vs[KW];
#pragma unroll
  for (int k = 0; k < KW; ++k) vs[k] = 0.0;

  auto load = [&](int yy, double (&g)[NG]) {
    const double* __restrict__ src = g64 + (static_cast<size_t>(yy) * W + xc) * NG;
#pragma unroll
    for (int i = 0; i < NG; ++i) g[i] = src[i];
  };
  // this wave's moments of g times coef added to its running sums
  auto add = [&](const double (&g)[NG], double coef) {
    static_assert(NWM <= 8, "at most eight moment waves");
    switch (wv) {
      case 0: add_moments<NG, 0 * KW, KW>(vs, g, coef); break;
      case 1: if constexpr (NWM > 1) add_moments<NG, 1 * KW, KW>(vs, g, coef); break;
      case 2: if constexpr (NWM > 2) add_moments<NG, 2 * KW, KW>(vs, g, coef); break;
      case 3: if constexpr (NWM > 3) add_moments<NG, 3 * KW, KW>(vs, g, coef); break;
      case 4: if constexpr (NWM > 4) add_moments<NG, 4 * KW, KW>(vs, g, coef); break;
      case 5: if constexpr (NWM > 5) add_moments<NG, 5 * KW, KW>(vs, g, coef); break;
      case 6: if constexpr (NWM > 6) add_moments<NG, 6 * KW, KW>(vs, g, coef); break;
      default: if constexpr (NWM > 7) add_moments<NG, 7 * KW, KW>(vs, g, coef); break;
    }
  };
  // add row ya (if a) and, with sign sgn_s, row ys (if sb); both rows' loads
  // are issued first
  auto update = [&](int ya, bool a, int ys, bool sb, double sgn_s) {
    double ga[NG], gs[NG];
    if (a) load(ya, ga);
    if (sb) load(ys, gs);
    if (a) add(ga, w);
    if (sb) add(gs, sgn_s * w);
  };

  // initial window, two rows per round
  {
    const int ra = max(0, y0 - R), rb = min(H - 1, y0 + R);
    for (int yy = ra; yy <= rb; yy += 2) update(yy, true, yy + 1, yy + 1 <= rb, 1.0);
  }
  for (int y = y0; y < y1; ++y) {
    if (y > y0) update(y + R, y + R < H, y - R - 1, y - R - 1 >= 0, -1.0);
    // transpose: lanes become moments
#pragma unroll
    for (int k = 0; k < KW; ++k)
      if (wv * KW + k < K) tr[(wv * KW + k) * TS + lane] = vs[k];
    __syncthreads();
    // horizontal running sums: thread t takes moment t mod K over the
    // output columns of part t / K
    const int t = static_cast<int>(threadIdx.x);
    const int j0 = (t / K) * JC;
    if (t < K * NSPLIT && j0 < SOUT) {
      const int kk = t % K;
      const double* __restrict__ row = tr + kk * TS + j0;
      // the output row origin is laundered so that the per-column store
      // addresses are formed as they are used, not hoisted out of the loop
      int ox = x_out0 + j0;
      asm volatile("" : "+v"(ox));
      double* __restrict__ srow = S + (static_cast<size_t>(y) * W + ox) * K + kk;
      double hs = 0.0;
#pragma unroll
      for (int c = 0; c <= 2 * R; ++c) hs += row[c];
#pragma unroll
      for (int j = 0; j < JC; ++j) {
        if (j0 + j < SOUT) {
          if (j > 0) hs += row[j + 2 * R] - row[j - 1];
          if (x_out0 + j0 + j < W) {
            if constexpr (FUSE < 0) {
              srow[static_cast<size_t>(j) * K] = hs;
            } else {
              sp[(j0 + j) * K + kk] = hs;
            }
          }
        }
      }
    }
    if constexpr (FUSE >= 0) {
      // the inverse of each output pixel of the row, from its window sums
      constexpr int D = system_size(FUSE, NG);
      constexpr int PD = D * (D + 1) / 2;
      constexpr int RW = minv_stride(FUSE, NG);
      using MT = typename std::conditional<FUSE != kSolveCov32, double, float>::type;
      __syncthreads();
      const int x = x_out0 + t;
      if (t < SOUT && x < W) {
        double mu[FUSE == kSolveRidge ? D - 1 : D];
        double M[PD];
        pixel_inverse<D, FUSE>(sp + t * K, static_cast<double>(window_count(x, y, W, H, R)),
                               eps, mu, M);
        const size_t p = static_cast<size_t>(y) * W + x;
        MT* __restrict__ rec = static_cast<MT*>(minv_void) + p * RW;
        constexpr int M0 = FUSE == kSolveRidge ? 0 : NG;
        if constexpr (FUSE != kSolveRidge) {
#pragma unroll
          for (int i = 0; i < NG; ++i) {
            mu_out[p * NG + i] = mu[i];
            rec[i] = static_cast<MT>(mu[i]);
          }
#pragma unroll
          for (int q = NG + PD; q < RW; ++q) rec[q] = MT(0);
        }
#pragma unroll
        for (int q = 0; q < PD; ++q) rec[M0 + q] = static_cast<MT>(M[q]);
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// a3: per-pixel inverse of the D x D window system by bordering, float64.
//
// Prop. 1 builds (lambda E + sum_i c_i c_i^T)^-1 = lambda^-1 E + sum alpha_ij c_i c_j^T
// by adding one channel kappa at a time (Sherman-Morrison); its alpha equals
// -lambda^-1 (lambda E + K)^-1 with K the Gram matrix of the channels added
// so far.  Written for M = -lambda alpha = (lambda E + K)^-1 the same
// recursion reads, with g = K[0:kappa, kappa] and u = M g:
//   s = lambda + K_kk - g^T u   (Schur complement; >= lambda, no pivoting)
//   M <- [[M + u u^T / s, -u / s], [-u^T / s, 1 / s]]
// which is the paper's update scaled by -lambda (gamma = -lambda / s,
// beta = -u / lambda).  Covariance form: K -> window covariance Sigma_p,
// lambda -> eps (Sec. 5.1 applies the same inverse to Eq. 13).  Ridge form:
// K -> raw window sums of [1, G][1, G]^T, lambda as given (Eq. 6).
// ---------------------------------------------------------------------------
// The inverse is computed in float64 and stored as the solve mode says:
// float32 or float64 covariance records (window means, then the packed
// inverse) or the packed float64 ridge inverse, whose raw-sum systems are far
// worse conditioned.
// The block's window sums (64 pixels x K, contiguous) are copied to LDS with
// coalesced direct-to-LDS loads, and its records gathered there again for
// contiguous stores.
template <int D, int MODE>
constexpr int invert_lds_doubles() {
  constexpr bool RIDGE = MODE == kSolveRidge;
  constexpr int NG = RIDGE ? D - 1 : D;
  constexpr int K = NG + NG * (NG + 1) / 2;
  constexpr int RW = minv_stride(MODE, NG);
  constexpr int out = RIDGE ? RW : (RW * minv_elem_bytes(MODE) + NG * 8 + 7) / 8;
  return 64 * (K > out ? K : out);
}

template <int D, int MODE>
__global__ __launch_bounds__(64) void invert_kernel(
    const double* __restrict__ S, int H, int W, int R, double eps,
    double* __restrict__ mu_out, void* __restrict__ minv_void) {
  constexpr bool RIDGE = MODE == kSolveRidge;
  using MT = typename std::conditional<MODE != kSolveCov32, double, float>::type;
  MT* __restrict__ minv_out = static_cast<MT*>(minv_void);
  constexpr int NG = RIDGE ? D - 1 : D;             // guidance channels n
  constexpr int K = NG + NG * (NG + 1) / 2;
  constexpr int PD = D * (D + 1) / 2;
  constexpr int RW = minv_stride(MODE, NG);
  __shared__ double Ss[invert_lds_doubles<D, MODE>()];
  const int lane = static_cast<int>(threadIdx.x);
  const int p0 = static_cast<int>(blockIdx.x) * 64;
  const int cnt = min(64, H * W - p0);
  {
    const int dwords = cnt * K * 2;
    const uint32_t* src = reinterpret_cast<const uint32_t*>(S + static_cast<size_t>(p0) * K);
    uint32_t* dst = reinterpret_cast<uint32_t*>(Ss);
    for (int base = 0; base < dwords; base += 64) {
      const int i = min(base + lane, dwords - 1);
      __builtin_amdgcn_global_load_lds(src + i, dst + base, 4, 0, 0);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }
  // lanes past the image work on their (unfilled) slot and store nothing
  const int p = min(p0 + lane, H * W - 1);
  const int y = p / W;
  const int x = p - y * W;
  const double Np = static_cast<double>(window_count(x, y, W, H, R));
  double mu[NG];
  double M[PD];
  pixel_inverse<D, MODE>(Ss + lane * K, Np, eps, mu, M);
  __syncthreads();  // every lane has read its window sums
  MT* __restrict__ ob = reinterpret_cast<MT*>(Ss);
  MT* __restrict__ rec = ob + lane * RW;
  constexpr int M0 = RIDGE ? 0 : NG;
  if (!RIDGE) {
    double* __restrict__ mb = reinterpret_cast<double*>(ob + 64 * RW);
#pragma unroll
    for (int i = 0; i < NG; ++i) {
      mb[lane * NG + i] = mu[i];
      rec[i] = static_cast<MT>(mu[i]);
    }
#pragma unroll
    for (int q = NG + PD; q < RW; ++q) rec[q] = MT(0);
  }
#pragma unroll
  for (int q = 0; q < PD; ++q) rec[M0 + q] = static_cast<MT>(M[q]);
  __syncthreads();
  MT* __restrict__ dst = minv_out + static_cast<size_t>(p0) * RW;
  if (!RIDGE) {
    // a record is a whole number of 16-byte units
    constexpr int U16 = RW * static_cast<int>(sizeof(MT)) / 16;
    const float4* __restrict__ src4 = reinterpret_cast<const float4*>(ob);
    float4* __restrict__ dst4 = reinterpret_cast<float4*>(dst);
    for (int e = lane; e < cnt * U16; e += 64) dst4[e] = src4[e];
    const double* __restrict__ mb = reinterpret_cast<const double*>(ob + 64 * RW);
    double* __restrict__ mdst = mu_out + static_cast<size_t>(p0) * NG;
    for (int e = lane; e < cnt * NG; e += 64) mdst[e] = mb[e];
  } else {
    for (int e = lane; e < cnt * RW; e += 64) dst[e] = ob[e];
  }
}

// Large systems (D >= 11): the same recursion with the rows of M spread over
// the kLpp = 4 lanes of a quad (lane q owns rows q, q + 4, ...), so the matrix
// stays in registers.  Values move within the quad by DPP broadcasts (plain
// vector ALU operations, no LDS round trip).  Every lane of the quad computes
// the same Schur complement, reduced in a fixed order.  Each step is a single
// rank-one update of the rows and columns in use; only the upper triangle of
// the result is stored.
constexpr int kLpp = 4;
// threads per block of the lane inverse: one wave (16 pixels); at n = 19 six
// such blocks fit a CU's LDS, and each stages its window sums while the
// others compute
constexpr int kInvBlock = 64;

// Value of lane K of this lane's quad.
template <int K>
__device__ __forceinline__ double quad_bcast(double v) {
  constexpr int ctrl = K | (K << 2) | (K << 4) | (K << 6);
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), ctrl, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), ctrl, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

// Sum over the quad, the same association in every lane.
__device__ __forceinline__ double quad_sum(double v) {
  constexpr int swap1 = 1 | (0 << 2) | (3 << 4) | (2 << 6);
  constexpr int swap2 = 2 | (3 << 2) | (0 << 4) | (1 << 6);
  auto perm = [](double x, auto ctrl_tag) {
    constexpr int c = decltype(ctrl_tag)::value;
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), c, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), c, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
  };
  v = v + perm(v, std::integral_constant<int, swap1>());
  return v + perm(v, std::integral_constant<int, swap2>());
}

// The bordered recursion of Prop. 1 (M = (lambda E + K)^-1 grown one row and
// column at a time) over the quad: on return lane q holds rows q, q + 4, ...
// of M in M[r][:].  A(i, j) returns entry (i, j), i <= j, of the system; each
// lane calls it for its own rows and for the diagonal.
template <int D, typename EntryFn>
__device__ __forceinline__ void quad_bordered_inverse(EntryFn A, int q,
                                                      double (&M)[(D + kLpp - 1) / kLpp][D]) {
  constexpr int NR = (D + kLpp - 1) / kLpp;
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int j = 0; j < D; ++j) M[r][j] = 0.0;
  if (q == 0) M[0][0] = 1.0 / A(0, 0);
  // value of quad lane k (k is a constant once the loops below are unrolled)
  auto bcast = [](double v, int k) -> double {
    switch (k) {
      case 0: return quad_bcast<0>(v);
      case 1: return quad_bcast<1>(v);
      case 2: return quad_bcast<2>(v);
      default: return quad_bcast<3>(v);
    }
  };
  // Row blocks r with kLpp * r >= kap hold no row of the current M: they are
  // skipped (kap and r are constants once the loops are unrolled).
#pragma unroll
  for (int kap = 1; kap < D; ++kap) {
    const int KB = kap / kLpp;  // row block of the new row kap
    // column kap of the system: lane q forms the entries j = q mod 4, j < kap
    double gq[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      if (kLpp * r >= kap) break;
      const int j = q + kLpp * r;
      gq[r] = (kLpp * r + kLpp - 1 < kap) ? A(j, kap) : ((j < kap) ? A(j, kap) : 0.0);
    }
    // u = M g for the owned rows (rows >= kap of M are zero, so is u there)
    double u[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) u[r] = 0.0;
#pragma unroll
    for (int j = 0; j < kap; ++j) {
      const double gj = bcast(gq[j / kLpp], j % kLpp);
#pragma unroll
      for (int r = 0; r < NR; ++r)
        if (kLpp * r < kap) u[r] = fma(M[r][j], gj, u[r]);
    }
    double part = 0.0;
#pragma unroll
    for (int r = 0; r < NR; ++r)
      if (kLpp * r < kap) part = fma(gq[r], u[r], part);
    const double inv = 1.0 / (A(kap, kap) - quad_sum(part));
    // With u_kap = -1 the bordered result
    //   [[M + u u^T / s, -u / s], [-u^T / s, 1 / s]]
    // is the one rank-one update M += u (u / s)^T over rows and columns <= kap.
    if (q == kap % kLpp) u[KB] = -1.0;
    double w[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r)
      if (r <= KB) w[r] = u[r] * inv;
#pragma unroll
    for (int j = 0; j <= kap; ++j) {
      const double wj = bcast(w[j / kLpp], j % kLpp);
#pragma unroll
      for (int r = 0; r < NR; ++r)
        if (r <= KB) M[r][j] = fma(u[r], wj, M[r][j]);
    }
  }
}

template <int D, int MODE>
__global__ __launch_bounds__(kInvBlock, 2) void invert_lanes_kernel(
    const double* __restrict__ S, int H, int W, int R, double eps,
    double* __restrict__ mu_out, void* __restrict__ minv_void) {
  constexpr bool RIDGE = MODE == kSolveRidge;
  using MT = typename std::conditional<MODE != kSolveCov32, double, float>::type;
  MT* __restrict__ minv_out = static_cast<MT*>(minv_void);
  constexpr int NG = RIDGE ? D - 1 : D;
  constexpr int K = NG + NG * (NG + 1) / 2;
  constexpr int PD = D * (D + 1) / 2;
  constexpr int NR = (D + kLpp - 1) / kLpp;  // rows per lane
  constexpr int RW = minv_stride(MODE, NG);
  // LDS doubles per pixel: its window sums, later its record and means
  constexpr int LW = (RW * static_cast<int>(sizeof(MT)) + NG * 8 + 7) / 8 > K
                         ? (RW * static_cast<int>(sizeof(MT)) + NG * 8 + 7) / 8
                         : K;
  const int q = threadIdx.x % kLpp;
  const int pr = static_cast<int>(blockIdx.x) * (kInvBlock / kLpp) + static_cast<int>(threadIdx.x) / kLpp;
  // lanes of a pixel past the image idle through the arithmetic on pixel 0
  // and store nothing (the broadcasts need every lane of the quad)
  const bool live = pr < H * W;
  const int p = live ? pr : 0;
  const int y = p / W;
  const int x = p - y * W;
  const double Np = static_cast<double>(window_count(x, y, W, H, R));
  const double invN = 1.0 / Np;

  // The block's window sums (64 pixels x K, contiguous) are copied to LDS
  // first with coalesced direct-to-LDS loads; the recursion then reads them
  // at LDS latency.
  __shared__ double Ss[(kInvBlock / kLpp) * LW];
  {
    const int p0 = static_cast<int>(blockIdx.x) * (kInvBlock / kLpp);
    const int cnt = min(kInvBlock / kLpp, H * W - p0);
    const int dwords = cnt * K * 2;
    const uint32_t* src = reinterpret_cast<const uint32_t*>(S + static_cast<size_t>(p0) * K);
    uint32_t* dst = reinterpret_cast<uint32_t*>(Ss);
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int base = wv * 64; base < dwords; base += kInvBlock) {
      const int i = min(base + lane, dwords - 1);
      __builtin_amdgcn_global_load_lds(src + i, dst + base, 4, 0, 0);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }
  const double* s = Ss + (static_cast<int>(threadIdx.x) / kLpp) * K;

  // one reciprocal per pixel; every entry is then formed with products only
  auto A = [&](int i, int j) -> double {
    if (!RIDGE) {
      const double mi = s[i] * invN, mj = s[j] * invN;
      return fma(s[NG + packed_index(i, j, NG)], invN, -mi * mj) + (i == j ? eps : 0.0);
    }
    if (i == 0) return (j == 0) ? Np + eps : s[j - 1];
    return s[NG + packed_index(i - 1, j - 1, NG)] + (i == j ? eps : 0.0);
  };

  double M[NR][D];
  quad_bordered_inverse<D>(A, q, M);
  if constexpr (!RIDGE) {
    // The block's records (and window means) are gathered in LDS, over the
    // window sums, and stored with contiguous 16-byte writes.
    constexpr int NP = kInvBlock / kLpp;
    static_assert(NP * RW * sizeof(MT) + NP * NG * sizeof(double) <= sizeof(Ss),
                  "records fit the staging area");
    const int m = static_cast<int>(threadIdx.x) / kLpp;
    double mq[NR];  // this lane's means mu_i, i = q mod 4
#pragma unroll
    for (int r = 0; r < NR; ++r)
      if (q + kLpp * r < NG) mq[r] = s[q + kLpp * r] * invN;
    __syncthreads();  // every lane has read its window sums
    MT* __restrict__ ob = reinterpret_cast<MT*>(Ss);
    double* __restrict__ mb = reinterpret_cast<double*>(ob + NP * RW);
    MT* __restrict__ o = ob + m * RW;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int i = q + kLpp * r;
      if (i < NG) {
        o[i] = static_cast<MT>(mq[r]);
        mb[m * NG + i] = mq[r];
        const int base = NG + packed_index(i, i, D) - i;  // (i, j) lies at base + j
#pragma unroll
        for (int j = 0; j < D; ++j)
          if (j >= i) o[base + j] = static_cast<MT>(M[r][j]);
      }
    }
    if (q == 0) {
#pragma unroll
      for (int e = NG + PD; e < RW; ++e) o[e] = MT(0);
    }
    __syncthreads();
    const int p0 = static_cast<int>(blockIdx.x) * NP;
    const int cnt = min(NP, H * W - p0);
    // a record is a whole number of 16-byte units
    constexpr int U16 = RW * static_cast<int>(sizeof(MT)) / 16;
    const float4* __restrict__ src4 = reinterpret_cast<const float4*>(ob);
    float4* __restrict__ dst4 = reinterpret_cast<float4*>(minv_out + static_cast<size_t>(p0) * RW);
    for (int e = static_cast<int>(threadIdx.x); e < cnt * U16; e += kInvBlock)
      dst4[e] = src4[e];
    double* __restrict__ mdst = mu_out + static_cast<size_t>(p0) * NG;
    for (int e = static_cast<int>(threadIdx.x); e < cnt * NG; e += kInvBlock) mdst[e] = mb[e];
  } else {
    if (!live) return;
    MT* __restrict__ o = minv_out + static_cast<size_t>(p) * RW;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int i = q + kLpp * r;
      if (i < D) {
        const int base = packed_index(i, i, D) - i;  // index of (i, j) is base + j
#pragma unroll
        for (int j = 0; j < D; ++j)
          if (j >= i) o[base + j] = static_cast<MT>(M[r][j]);
      }
    }
  }
}

// Dense batched form for D >= 11: the quad recursion above on matrices staged
// in LDS (16 per block), full D x D inverse written out.
constexpr int kSpdPerBlock = 16;

template <int D>
__global__ __launch_bounds__(kSpdPerBlock * kLpp) void spd_inverse_lanes_kernel(
    const double* __restrict__ a, double* __restrict__ out, int count) {
  constexpr int NR = (D + kLpp - 1) / kLpp;
  __shared__ double sa[kSpdPerBlock * D * D];
  const int b0 = static_cast<int>(blockIdx.x) * kSpdPerBlock;
  {
    const int cnt = min(kSpdPerBlock, count - b0);
    const int dwords = cnt * D * D * 2;
    const uint32_t* src = reinterpret_cast<const uint32_t*>(a + static_cast<size_t>(b0) * D * D);
    uint32_t* dst = reinterpret_cast<uint32_t*>(sa);
    const int lane = threadIdx.x & 63;
    for (int base = 0; base < dwords; base += 64) {
      const int i = min(base + lane, dwords - 1);
      __builtin_amdgcn_global_load_lds(src + i, dst + base, 4, 0, 0);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }
  const int q = threadIdx.x % kLpp;
  const int m = static_cast<int>(threadIdx.x) / kLpp;
  const bool live = b0 + m < count;
  const double* A_ = sa + (live ? m : 0) * D * D;
  double M[NR][D];
  quad_bordered_inverse<D>([&](int i, int j) { return A_[i * D + j]; }, q, M);
  if (!live) return;
  double* O = out + static_cast<size_t>(b0 + m) * D * D;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int i = q + kLpp * r;
    if (i < D) {
#pragma unroll
      for (int j = 0; j < D; ++j)
        if (j >= i) {
          O[i * D + j] = M[r][j];
          O[j * D + i] = M[r][j];  // the lower triangle mirrors the upper
        }
    }
  }
}

// Same recursion over a batch of dense SPD matrices (upper triangle read).
template <int D>
__global__ __launch_bounds__(64) void spd_inverse_kernel(const double* __restrict__ a,
                                                         double* __restrict__ out, int count) {
  constexpr int PD = D * (D + 1) / 2;
  const int b = static_cast<int>(blockIdx.x) * 64 + threadIdx.x;
  if (b >= count) return;
  const double* A = a + static_cast<size_t>(b) * D * D;
  double M[PD];
  M[0] = 1.0 / A[0];
#pragma unroll
  for (int kap = 1; kap < D; ++kap) {
    double g[D];
    double u[D];
#pragma unroll
    for (int i = 0; i < kap; ++i) g[i] = A[i * D + kap];
#pragma unroll
    for (int i = 0; i < kap; ++i) {
      double acc = 0.0;
#pragma unroll
      for (int j = 0; j < kap; ++j)
        acc = fma(M[i <= j ? packed_index(i, j, D) : packed_index(j, i, D)], g[j], acc);
      u[i] = acc;
    }
    double schur = A[kap * D + kap];
#pragma unroll
    for (int i = 0; i < kap; ++i) schur = fma(-g[i], u[i], schur);
    const double inv = 1.0 / schur;
#pragma unroll
    for (int i = 0; i < kap; ++i) {
      const double ui = u[i] * inv;
#pragma unroll
      for (int j = i; j < kap; ++j) M[packed_index(i, j, D)] = fma(ui, u[j], M[packed_index(i, j, D)]);
      M[packed_index(i, kap, D)] = -ui;
    }
    M[packed_index(kap, kap, D)] = inv;
  }
  double* O = out + static_cast<size_t>(b) * D * D;
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j)
      O[i * D + j] = M[i <= j ? packed_index(i, j, D) : packed_index(j, i, D)];
}


}  // namespace gk

// a2 for one (n, radius): window sums of the K = n + n(n+1)/2 moments, into
// S (FUSE < 0) or, with the inverse fused in (FUSE = the solve mode), straight
// to the window means and solve records.
template <int NG, int R, int FUSE>
hipError_t moments_nr(const double* g64, int H, int W, int target, double* S, double eps,
                      double* mu, void* minv, hipStream_t s) {
  constexpr int K = NG + NG * (NG + 1) / 2;
  // two waves for up to 64 moments; above, eight waves of up to 27 moments
  constexpr int KW = K <= 64 ? (K + 1) / 2 : (K + 7) / 8;
  constexpr int NWM = (K + KW - 1) / KW;
  StripGrid g = strip_grid(H, W, R, 1, target);
  hipLaunchKernelGGL((gk::moments_kernel<R, NG, KW, FUSE>),
                     dim3(static_cast<unsigned>(g.strips * g.bands)), dim3(NWM * 64), 0, s, g64,
                     H, W, g.band_h, g.strips, S, eps, mu, minv);
  return hipGetLastError();
}

template <int NG, int R>
hipError_t moments_r(const double* g64, int H, int W, int target, double* S, double eps,
                     int mode, double* mu, void* minv, int* fused, hipStream_t s) {
  if constexpr (NG <= gk::kFuseMaxN) {
    *fused = 1;
    switch (mode) {
      case kSolveCov32: return moments_nr<NG, R, kSolveCov32>(g64, H, W, target, S, eps, mu, minv, s);
      case kSolveCov64: return moments_nr<NG, R, kSolveCov64>(g64, H, W, target, S, eps, mu, minv, s);
      case kSolveRidge: return moments_nr<NG, R, kSolveRidge>(g64, H, W, target, S, eps, mu, minv, s);
      default: return hipErrorNotSupported;
    }
  } else {
    *fused = 0;
    return moments_nr<NG, R, -1>(g64, H, W, target, S, eps, mu, minv, s);
  }
}

template <int D, int MODE>
hipError_t invert_dm(const double* S, int H, int W, int R, double eps, double* mu, void* minv,
                     hipStream_t s) {
  const int P = H * W;
  if constexpr (D >= 11) {
    constexpr int per_block = gk::kInvBlock / gk::kLpp;
    hipLaunchKernelGGL((gk::invert_lanes_kernel<D, MODE>), dim3((P + per_block - 1) / per_block),
                       dim3(gk::kInvBlock), 0, s, S, H, W, R, eps, mu, minv);
  } else {
    hipLaunchKernelGGL((gk::invert_kernel<D, MODE>), dim3((P + 63) / 64), dim3(64), 0, s, S, H,
                       W, R, eps, mu, minv);
  }
  return hipGetLastError();
}

// a2 for n guidance channels, every compiled radius (with a3 fused in for
// n <= kFuseMaxN, which *fused reports).
template <int NG>
hipError_t moments_n(const double* g64, int H, int W, int R, int target, double* S, double eps,
                     int mode, double* mu, void* minv, int* fused, hipStream_t s) {
  static_assert(kMinRadius == 0 && kMaxRadius == 9, "the radius list below");
  switch (R) {
#define HGF_MOM(r) \
  case r: return moments_r<NG, r>(g64, H, W, target, S, eps, mode, mu, minv, fused, s);
    HGF_MOM(0)
    HGF_MOM(1)
    HGF_MOM(2)
    HGF_MOM(3)
    HGF_MOM(4)
    HGF_MOM(5)
    HGF_MOM(6)
    HGF_MOM(7)
    HGF_MOM(8)
    HGF_MOM(9)
#undef HGF_MOM
    default: return hipErrorNotSupported;
  }
}

// a3 for n guidance channels, every solve mode (the ridge system has n + 1 rows).
template <int NG>
hipError_t invert_n(const double* S, int H, int W, int R, double eps, int mode, double* mu,
                    void* minv, hipStream_t s) {
  switch (mode) {
    case kSolveCov32: return invert_dm<NG, kSolveCov32>(S, H, W, R, eps, mu, minv, s);
    case kSolveCov64: return invert_dm<NG, kSolveCov64>(S, H, W, R, eps, mu, minv, s);
    case kSolveRidge: return invert_dm<NG + 1, kSolveRidge>(S, H, W, R, eps, mu, minv, s);
    default: return hipErrorNotSupported;
  }
}

}  // namespace hgf
