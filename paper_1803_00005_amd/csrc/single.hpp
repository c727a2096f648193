// a4 - a7 for a single label slice (L = 1), with lanes as pixels.
//
// The label-lane kernels give each wave the 64 labels of one pixel; with one
// label 63 of the 64 lanes would idle.  Here every thread is one pixel (or one
// column of a band of rows) and the filter runs as separable box sums over
// planar float32 images [n+1][H][W] in the coefficient workspace:
//   1. vertical window sums of the n + 1 products G_ch Y (G_0 = 1)   (Eq. 9)
//   2. horizontal window sums (float64), the per-pixel solve, coefficients
//      [b, a_1..a_n] (covariance form, Sec. 5.1) or w = M [U; T] (ridge form,
//      Eq. 6)
//   3. vertical window sums of the n + 1 coefficient images
//   4. horizontal window sums (float64) and Z = sum_ch B(w_ch) G_ch / N (Eq. 11);
//      the label (the only one) or its winner-takes-all key.
// The same arithmetic as the label-lane path, in another summation order.
// Instantiated per channel count in generated units (every cost type and
// solve mode of one n per unit).
#pragma once

#include <type_traits>

#include "hgf_launch.hpp"

namespace hgf {
namespace sk {

constexpr int kSingleBand = 32;  // rows per thread of the vertical passes

// Vertical window sums of NCH channels for one column and a band of rows:
// PROD = 1 sums the products G_ch Y (G_0 = 1) of the guidance and the cost
// slice; PROD = 0 sums the planar images `in` [NCH][P].
template <int NCH, int PROD, typename TIN>
__global__ __launch_bounds__(256) void single_vbox_kernel(
    const float* __restrict__ g32, const TIN* __restrict__ cost, int cost_ld,
    const float* __restrict__ in, float* __restrict__ outv, int H, int W, int R) {
  const int x = static_cast<int>(blockIdx.x) * 256 + threadIdx.x;
  if (x >= W) return;
  const int y0 = static_cast<int>(blockIdx.y) * kSingleBand;
  const int y1 = min(H, y0 + kSingleBand);
  const size_t P = static_cast<size_t>(H) * W;
  auto value = [&](int y, float (&v)[NCH]) {
    const size_t p = static_cast<size_t>(y) * W + x;
    if (PROD) {
      const float yv = load_cost<TIN>(cost, p * cost_ld);
      v[0] = yv;
#pragma unroll
      for (int ch = 1; ch < NCH; ++ch) v[ch] = g32[ch * P + p] * yv;
    } else {
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) v[ch] = in[ch * P + p];
    }
  };
  float s[NCH];
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) s[ch] = 0.f;
  for (int y = max(0, y0 - R); y <= min(H - 1, y0 + R); ++y) {
    float v[NCH];
    value(y, v);
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) s[ch] += v[ch];
  }
  for (int y = y0; y < y1; ++y) {
    if (y > y0) {
      float a[NCH], b[NCH];
      const bool ea = y + R < H, lb = y - R - 1 >= 0;
      if (ea) value(y + R, a);
      if (lb) value(y - R - 1, b);
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) {
        if (ea) s[ch] += a[ch];
        if (lb) s[ch] -= b[ch];
      }
    }
    const size_t p = static_cast<size_t>(y) * W + x;
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) outv[ch * P + p] = s[ch];
  }
}

// float64 horizontal window sum of column-window [x - R, x + R] of row y of
// channel ch of a planar image.
__device__ __forceinline__ double hsum(const float* __restrict__ img, size_t row, int x, int W,
                                       int R) {
  double t = 0.0;
  const int xa = max(0, x - R), xb = min(W - 1, x + R);
  for (int xx = xa; xx <= xb; ++xx) t += static_cast<double>(img[row + xx]);
  return t;
}

// Horizontal sums and the per-pixel solve; coefficient images [NG+1][P].
// Both covariance records are applied in float64 here (the float32 record's
// elements widened), the ridge inverse too.
template <int NG, int MODE>
__global__ __launch_bounds__(256) void single_solve_kernel(const float* __restrict__ vbox,
                                                           const void* __restrict__ minv_void,
                                                           float* __restrict__ coef, int H,
                                                           int W, int R) {
  constexpr int NCH = NG + 1;
  constexpr bool RIDGE = MODE == kSolveRidge;
  constexpr int D = RIDGE ? NCH : NG;
  constexpr int RW = minv_stride(MODE, NG);
  using MT = typename std::conditional<MODE == kSolveCov32, float, double>::type;
  const size_t P = static_cast<size_t>(H) * W;
  const size_t p = static_cast<size_t>(blockIdx.x) * 256 + threadIdx.x;
  if (p >= P) return;
  const int y = static_cast<int>(p / W);
  const int x = static_cast<int>(p - static_cast<size_t>(y) * W);
  const size_t row = static_cast<size_t>(y) * W;
  double T[NCH];
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) T[ch] = hsum(vbox + ch * P, row, x, W, R);
  if constexpr (!RIDGE) {
    // record: mu_1..mu_n, then the packed inverse
    const MT* __restrict__ rec = static_cast<const MT*>(minv_void) + p * RW;
    const double invN = 1.0 / static_cast<double>(window_count(x, y, W, H, R));
    const double U = T[0];
    double c[NG], av[NG];
#pragma unroll
    for (int i = 0; i < NG; ++i) {
      c[i] = (T[i + 1] - static_cast<double>(rec[i]) * U) * invN;
      av[i] = 0.0;
    }
#pragma unroll
    for (int i = 0; i < NG; ++i) {
#pragma unroll
      for (int j = i; j < NG; ++j) {
        const double m = static_cast<double>(rec[NG + packed_index(i, j, D)]);
        av[i] = fma(m, c[j], av[i]);
        if (j != i) av[j] = fma(m, c[i], av[j]);
      }
    }
    double b = U * invN;
#pragma unroll
    for (int i = 0; i < NG; ++i) b = fma(-av[i], static_cast<double>(rec[i]), b);
    coef[p] = static_cast<float>(b);
#pragma unroll
    for (int i = 0; i < NG; ++i) coef[(i + 1) * P + p] = static_cast<float>(av[i]);
  } else {
    const double* __restrict__ mp = static_cast<const double*>(minv_void) + p * RW;
    double w[D];
#pragma unroll
    for (int i = 0; i < D; ++i) w[i] = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
#pragma unroll
      for (int j = i; j < D; ++j) {
        const double m = mp[packed_index(i, j, D)];
        w[i] = fma(m, T[j], w[i]);
        if (j != i) w[j] = fma(m, T[i], w[j]);
      }
    }
#pragma unroll
    for (int i = 0; i < D; ++i) coef[i * P + p] = static_cast<float>(w[i]);
  }
}

// Horizontal sums of the vertically summed coefficients, the output and the
// label (or its winner-takes-all key, when the caller merges label chunks).
template <int NG>
__global__ __launch_bounds__(256) void single_out_kernel(const float* __restrict__ vbox,
                                                         const float* __restrict__ g32,
                                                         float* __restrict__ out, int out_ld,
                                                         unsigned long long* __restrict__ keys,
                                                         int32_t* __restrict__ labels, int label,
                                                         int H, int W, int R) {
  constexpr int NCH = NG + 1;
  const size_t P = static_cast<size_t>(H) * W;
  const size_t p = static_cast<size_t>(blockIdx.x) * 256 + threadIdx.x;
  if (p >= P) return;
  const int y = static_cast<int>(p / W);
  const int x = static_cast<int>(p - static_cast<size_t>(y) * W);
  const size_t row = static_cast<size_t>(y) * W;
  double z = hsum(vbox, row, x, W, R);
#pragma unroll
  for (int ch = 1; ch < NCH; ++ch)
    z = fma(hsum(vbox + ch * P, row, x, W, R), static_cast<double>(g32[ch * P + p]), z);
  z /= static_cast<double>(window_count(x, y, W, H, R));
  const float zf = static_cast<float>(z);
  if (out != nullptr) out[p * out_ld] = zf;
  if (labels != nullptr)
    labels[p] = label;
  else if (keys != nullptr)
    atomicMin(&keys[p], wta_key(zf, label));
}

}  // namespace sk

template <int NG, typename TIN>
hipError_t single_launch_t(const SingleLaunch& a, hipStream_t s) {
  using namespace sk;
  constexpr int NCH = NG + 1;
  const size_t P = static_cast<size_t>(a.H) * a.W;
  float* v = a.ws;             // vertical sums [NCH][P]
  float* c = a.ws + NCH * P;   // coefficients [NCH][P]
  const dim3 vgrid(static_cast<unsigned>((a.W + 255) / 256),
                   static_cast<unsigned>((a.H + kSingleBand - 1) / kSingleBand));
  const unsigned pgrid = static_cast<unsigned>((P + 255) / 256);
  hipLaunchKernelGGL((single_vbox_kernel<NCH, 1, TIN>), vgrid, dim3(256), 0, s, a.g32,
                     static_cast<const TIN*>(a.cost), a.cost_ld, nullptr, v, a.H, a.W, a.R);
  if (a.mode == kSolveCov32)
    hipLaunchKernelGGL((single_solve_kernel<NG, kSolveCov32>), dim3(pgrid), dim3(256), 0, s, v,
                       a.minv, c, a.H, a.W, a.R);
  else if (a.mode == kSolveCov64)
    hipLaunchKernelGGL((single_solve_kernel<NG, kSolveCov64>), dim3(pgrid), dim3(256), 0, s, v,
                       a.minv, c, a.H, a.W, a.R);
  else
    hipLaunchKernelGGL((single_solve_kernel<NG, kSolveRidge>), dim3(pgrid), dim3(256), 0, s, v,
                       a.minv, c, a.H, a.W, a.R);
  hipLaunchKernelGGL((single_vbox_kernel<NCH, 0, float>), vgrid, dim3(256), 0, s, nullptr,
                     static_cast<const float*>(nullptr), 0, c, v, a.H, a.W, a.R);
  hipLaunchKernelGGL((single_out_kernel<NG>), dim3(pgrid), dim3(256), 0, s, v, a.g32, a.out,
                     a.out_ld, a.keys, a.labels, a.label, a.H, a.W, a.R);
  return hipGetLastError();
}

// Every cost type of one channel count.
template <int NG>
hipError_t single_launch_n(const SingleLaunch& a, hipStream_t s) {
  switch (a.cost_type) {
    case kCostF32: return single_launch_t<NG, float>(a, s);
    case kCostBF16: return single_launch_t<NG, bf16_t>(a, s);
    case kCostF16: return single_launch_t<NG, f16_t>(a, s);
    default: return hipErrorNotSupported;
  }
}

}  // namespace hgf
