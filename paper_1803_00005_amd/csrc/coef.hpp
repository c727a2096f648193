// a4 + a5: per-label box sums of the guidance x cost products and the per-pixel
// coefficient solve, fused.
//
// For every label slice Y of the cost volume and every pixel p (Sec. 4.3,
// Eq. 9 with Prop. 2; the covariance form of Sec. 5.1, Eqs. 12-13):
//   U = B(Y),  T_i = B(G_i Y)                       (window sums, i = 1..n)
//   covariance:  c = (T - mu U) / N_p,  a = M_p c,  b = U / N_p - a . mu
//   ridge:       [b; a] = M_p [U; T]               (M_p of the (n+1) system)
// with M_p the per-pixel inverse computed once per image.  The coefficient
// images [b, a_1..a_n] go to a float32 workspace [chunk][P][n+1][64].
//
// Mapping (gfx950, wave64): the 64 lanes of a wave are 64 labels of one
// pixel.  Everything per-pixel (M_p, mu_p, G(p), N_p) is wave-uniform and is
// read with scalar loads into SGPRs, so the n x n times n x 64 product runs
// as plain VALU FMAs with one scalar operand and no operand traffic.
// A workgroup owns a strip of 64 state columns (64 - 2R output columns) over a
// band of rows.  Its waves split the n + 1 product channels: each wave keeps
// float32 vertical running sums of its channels for all 64 columns in
// registers (add the row entering the window, subtract the row leaving it)
// and forms the horizontal window sums in registers with float64 running
// sums, so the only shared-memory traffic is one transpose of the finished
// window sums T, U per output pixel before the solve.  Bands restart the
// vertical sums, which bounds float32 drift to band_h + 2R additions.
#pragma once

#include "hgf_launch.hpp"

namespace hgf {

template <int R, int CPW, int NG, int RIDGE, typename TIN, int SIN>
__global__ __launch_bounds__(640) void coef_kernel(
    const TIN* __restrict__ cost, int cost_ld, const float* __restrict__ g32,
    const double* __restrict__ mu, const double* __restrict__ minv, float* __restrict__ ws,
    int H, int W, int label_count, int band_h, int strips, int bands) {
  constexpr int SOUT = SIN - 2 * R;
  constexpr int NCH = NG + 1;
  constexpr int NW = (NCH + CPW - 1) / CPW;
  constexpr int D = RIDGE ? NG + 1 : NG;
  constexpr int PD = D * (D + 1) / 2;
  constexpr int OC_RAW = 12800 / (NCH * 64);
  constexpr int OC = OC_RAW < 1 ? 1 : (OC_RAW > SOUT ? SOUT : OC_RAW);
  __shared__ float lds[OC * NCH * 64];

  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int bid = static_cast<int>(blockIdx.x);
  const int strip = bid % strips;
  bid /= strips;
  const int band = bid % bands;
  const int chunk = bid / bands;
  const int x_out0 = strip * SOUT;
  const int xs = x_out0 - R;
  const int y0 = band * band_h;
  const int y1 = min(H, y0 + band_h);
  const int lab = chunk * 64 + lane;
  // lanes past the last label read the last label's costs; their results are never used
  const int labc = min(lab, label_count - 1);
  const size_t P = static_cast<size_t>(H) * W;
  float* __restrict__ wsc = ws + static_cast<size_t>(chunk) * P * NCH * 64;

  float vs[CPW][SIN];
#pragma unroll
  for (int k = 0; k < CPW; ++k)
#pragma unroll
    for (int c = 0; c < SIN; ++c) vs[k][c] = 0.f;

  // Vertical update with row yy for all state columns.  Branch-free: columns
  // outside the image read a clamped pixel with weight 0.  The strip origin is
  // laundered so that the per-column offsets are recomputed for each row
  // rather than hoisted out of the row loop (64 live offsets would spill).
  auto acc_row = [&](int yy, bool add) {
    int xsl = xs;
    asm volatile("" : "+s"(xsl));
    const size_t rowp = static_cast<size_t>(yy) * W;
#pragma unroll
    for (int c = 0; c < SIN; ++c) {
      if ((c & 7) == 0) __builtin_amdgcn_sched_barrier(0);
      const int xr = xsl + c;
      const int xc = min(max(xr, 0), W - 1);
      const size_t p = rowp + xc;
      const float yv = load_cost<TIN>(cost, p * cost_ld + labc);
#pragma unroll
      for (int k = 0; k < CPW; ++k) {
        const int ch = wv * CPW + k;
        const int chc = ch < NCH ? ch : NCH - 1;
        float g = ldu(g32, p * NCH + chc);
        g = (xr == xc && ch < NCH) ? (add ? g : -g) : 0.f;
        vs[k][c] = fmaf(g, yv, vs[k][c]);
      }
    }
  };

  auto solve_store = [&](int x, int y, int q) {
    const size_t p = static_cast<size_t>(y) * W + x;
    float T[NCH];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) T[ch] = lds[(q * NCH + ch) * 64 + lane];
    double av[NG];
    double b;
    const double* __restrict__ mp = minv + p * PD;
    if (!RIDGE) {
      const double invN = 1.0 / static_cast<double>(window_count(x, y, W, H, R));
      const double U = static_cast<double>(T[0]);
      double c[NG];
#pragma unroll
      for (int i = 0; i < NG; ++i)
        c[i] = (static_cast<double>(T[i + 1]) - ldu(mu, p * NG + i) * U) * invN;
#pragma unroll
      for (int i = 0; i < NG; ++i) av[i] = 0.0;
#pragma unroll
      for (int i = 0; i < NG; ++i) {
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int j = i; j < NG; ++j) {
          const double m = ldu(mp, packed_index(i, j, D));
          av[i] = fma(m, c[j], av[i]);
          if (j != i) av[j] = fma(m, c[i], av[j]);
        }
      }
      b = U * invN;
#pragma unroll
      for (int i = 0; i < NG; ++i) b = fma(-av[i], ldu(mu, p * NG + i), b);
    } else {
      double v[D];
      double w[D];
#pragma unroll
      for (int i = 0; i < D; ++i) {
        v[i] = static_cast<double>(T[i]);
        w[i] = 0.0;
      }
#pragma unroll
      for (int i = 0; i < D; ++i) {
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int j = i; j < D; ++j) {
          const double m = ldu(mp, packed_index(i, j, D));
          w[i] = fma(m, v[j], w[i]);
          if (j != i) w[j] = fma(m, v[i], w[j]);
        }
      }
      b = w[0];
#pragma unroll
      for (int i = 0; i < NG; ++i) av[i] = w[i + 1];
    }
    float* __restrict__ o = wsc + p * NCH * 64 + lane;
    o[0] = static_cast<float>(b);
#pragma unroll
    for (int i = 0; i < NG; ++i) o[(i + 1) * 64] = static_cast<float>(av[i]);
  };

  for (int yy = max(0, y0 - R); yy <= min(H - 1, y0 + R); ++yy) acc_row(yy, true);
  for (int y = y0; y < y1; ++y) {
    if (y > y0) {
      if (y + R < H) acc_row(y + R, true);
      if (y - R - 1 >= 0) acc_row(y - R - 1, false);
    }
    double hs[CPW];
#pragma unroll
    for (int k = 0; k < CPW; ++k) {
      hs[k] = 0.0;
#pragma unroll
      for (int c = 0; c <= 2 * R; ++c) hs[k] += static_cast<double>(vs[k][c]);
    }
#pragma unroll
    for (int j = 0; j < SOUT; ++j) {
      if (j > 0) {
#pragma unroll
        for (int k = 0; k < CPW; ++k)
          hs[k] += static_cast<double>(vs[k][j + 2 * R]) - static_cast<double>(vs[k][j - 1]);
      }
      const int jj = j % OC;
#pragma unroll
      for (int k = 0; k < CPW; ++k) {
        const int ch = wv * CPW + k;
        if (ch < NCH) lds[(jj * NCH + ch) * 64 + lane] = static_cast<float>(hs[k]);
      }
      if (jj == OC - 1 || j == SOUT - 1) {
        __syncthreads();
        const int j0 = j - jj;
        for (int q = wv; q <= jj; q += NW) {
          const int x = x_out0 + j0 + q;
          if (x < W) solve_store(x, y, q);
        }
        __syncthreads();
      }
    }
  }
}

// Strip width (state columns) of the coefficient kernel.  Up to n = 9 one
// channel per wave and 64 columns; above, two channels per wave and a
// narrower strip so that ten waves fit the register file without spilling.
template <int NG>
constexpr int coef_strip() { return NG + 1 > 10 ? 38 : 64; }

template <int R, int NG, int RIDGE, typename TIN>
hipError_t coef_launch_t(const CoefLaunch& a, hipStream_t s) {
  constexpr int NCH = NG + 1;
  constexpr int CPW = NCH > 10 ? 2 : 1;
  constexpr int NW = (NCH + CPW - 1) / CPW;
  constexpr int SIN = coef_strip<NG>();
  const StripGrid& g = a.grid;
  const unsigned blocks = static_cast<unsigned>(g.strips * g.bands * g.chunks);
  hipLaunchKernelGGL((coef_kernel<R, CPW, NG, RIDGE, TIN, SIN>), dim3(blocks), dim3(NW * 64), 0, s,
                     static_cast<const TIN*>(a.cost), a.cost_ld, a.g32, a.mu, a.minv, a.ws, a.H,
                     a.W, a.label_count, g.band_h, g.strips, g.bands);
  return hipGetLastError();
}

template <int NG>
hipError_t coef_launch_n(const CoefLaunch& a, hipStream_t s) {
#define HGF_COEF_R(r)                                                        \
  case r:                                                                    \
    if (a.reg == 0) {                                                        \
      if (a.cost_bf16) return coef_launch_t<r, NG, 0, uint16_t>(a, s);       \
      return coef_launch_t<r, NG, 0, float>(a, s);                           \
    }                                                                        \
    if (a.cost_bf16) return hipErrorNotSupported;                            \
    return coef_launch_t<r, NG, 1, float>(a, s);
  switch (a.R) {
    HGF_COEF_R(1)
    HGF_COEF_R(2)
    HGF_COEF_R(4)
    HGF_COEF_R(7)
    HGF_COEF_R(9)
    default:
      return hipErrorNotSupported;
  }
#undef HGF_COEF_R
}

}  // namespace hgf
