// Guidance part of the filter, run once per image and shared by every label
// slice (the all-pair guidance box filters are computed once, Sec. 5.3):
//   a1  polynomial guidance synthesis (Sec. 4.2) and the channel shifts.
// The window sums (a2) and the per-pixel inverse (a3) are in
// guide_kernels.hpp, instantiated per channel count; this unit also launches
// the dense batched SPD inverse (Prop. 1 on its own, Fig. 1(a)).
#include <type_traits>

#include "guide_kernels.hpp"

namespace hgf {
namespace {

__device__ __forceinline__ double monomial(const MonoTable& t, int k, const float* iv) {
  double v = 1.0;
  for (int c = 0; c < t.m; ++c) {
    const double x = static_cast<double>(iv[c]);
    for (int e = 0; e < t.e[k][c]; ++e) v *= x;
  }
  return v;
}

// ---------------------------------------------------------------------------
// a1: the channel shifts and the synthesized guidance.  The covariance form
// is invariant to a constant shift of each guidance channel, so any constant
// is exact; the shift only centres the values for float32 conditioning.  It
// is the channel mean over a fixed grid of at most 16 x 16 pixels, reduced by
// one block in a fixed order (deterministic).
// ---------------------------------------------------------------------------
constexpr int kShiftGrid = kShiftRows;  // sample grid: at most 16 x 16 pixels

// One block of kShiftRows x kShiftRows threads, one sample each.  The
// samples' monomials go to LDS; then kShiftParts threads per channel each add
// a quarter of the samples in index order, and one thread per channel adds
// the quarters in order (a fixed order: the shift is deterministic).
constexpr int kShiftThreads = kShiftGrid * kShiftGrid;
constexpr int kShiftParts = 4;
constexpr int kShiftPart = kShiftThreads / kShiftParts;
static_assert(kMaxD * kShiftParts <= kShiftThreads, "one thread per channel part");

__global__ __launch_bounds__(kShiftThreads) void guide_shift_kernel(
    const float* __restrict__ I, int H, int W, MonoTable t, int centre,
    double* __restrict__ shift) {
  __shared__ double sv[kMaxD * kShiftThreads];
  __shared__ double part[kMaxD * kShiftParts];
  const int sy = (H + kShiftGrid - 1) / kShiftGrid, sx = (W + kShiftGrid - 1) / kShiftGrid;
  const int ny = (H + sy - 1) / sy, nx = (W + sx - 1) / sx;
  const size_t P = static_cast<size_t>(H) * W;
  const int tid = static_cast<int>(threadIdx.x);
  const int gy = tid / kShiftGrid, gx = tid % kShiftGrid;
  const bool in = gy < ny && gx < nx;
  float iv[4] = {0.f, 0.f, 0.f, 0.f};
  if (in) {
    const size_t p = static_cast<size_t>(gy * sy) * W + gx * sx;
    for (int c = 0; c < t.m; ++c) iv[c] = I[static_cast<size_t>(c) * P + p];
  }
  for (int k = 0; k < t.n; ++k) sv[k * kShiftThreads + tid] = in ? monomial(t, k, iv) : 0.0;
  __syncthreads();
  const int k = tid / kShiftParts, q = tid % kShiftParts;
  if (k < t.n) {
    const double* __restrict__ src = sv + k * kShiftThreads + q * kShiftPart;
    double acc = 0.0;
    for (int i = 0; i < kShiftPart; ++i) acc += src[i];
    part[k * kShiftParts + q] = acc;
  }
  __syncthreads();
  if (tid < t.n) {
    double tot = 0.0;
#pragma unroll
    for (int j = 0; j < kShiftParts; ++j) tot += part[tid * kShiftParts + j];
    shift[tid] = centre ? tot / static_cast<double>(ny * nx) : 0.0;
  }
}

// g32 holds n + 1 planar channels [n+1][P], channel 0 being the constant
// G_0 = 1, so the per-label kernels index the multiplier of every box channel
// uniformly and read 16 consecutive columns of one channel with one scalar load.
// The block's 256 pixels of g64 [P][n] are one contiguous run of 256 n
// doubles: they are gathered in LDS and stored by consecutive lanes.
__global__ __launch_bounds__(256) void guide_synth_kernel(
    const float* __restrict__ I, int P, MonoTable t, const double* __restrict__ shift,
    float* __restrict__ g32, double* __restrict__ g64) {
  __shared__ double st[256 * kMaxN];
  const int p0 = static_cast<int>(blockIdx.x) * 256;
  const int p = p0 + static_cast<int>(threadIdx.x);
  if (p < P) {
    float iv[4] = {0.f, 0.f, 0.f, 0.f};
    for (int c = 0; c < t.m; ++c) iv[c] = I[static_cast<size_t>(c) * P + p];
    g32[p] = 1.0f;
    for (int k = 0; k < t.n; ++k) {
      const double g = monomial(t, k, iv) - shift[k];
      st[threadIdx.x * t.n + k] = g;
      g32[static_cast<size_t>(k + 1) * P + p] = static_cast<float>(g);
    }
  }
  __syncthreads();
  const int count = min(256, P - p0) * t.n;
  double* __restrict__ dst = g64 + static_cast<size_t>(p0) * t.n;
  for (int e = static_cast<int>(threadIdx.x); e < count; e += 256) dst[e] = st[e];
}

}  // namespace

hipError_t launch_guide_mean(const float* I, int H, int W, const MonoTable& t, double* shift,
                             bool centre, hipStream_t s) {
  hipLaunchKernelGGL(guide_shift_kernel, dim3(1), dim3(kShiftThreads), 0, s, I, H, W, t,
                     centre ? 1 : 0, shift);
  return hipGetLastError();
}

hipError_t launch_guide_synth(const float* I, int H, int W, const MonoTable& t,
                              const double* shift, float* g32, double* g64, hipStream_t s) {
  const int P = H * W;
  const unsigned blocks = static_cast<unsigned>((P + 255) / 256);
  hipLaunchKernelGGL(guide_synth_kernel, dim3(blocks), dim3(256), 0, s, I, P, t, shift, g32,
                     g64);
  return hipGetLastError();
}

hipError_t launch_spd_inverse(const double* a, double* minv, int D, int count, hipStream_t s) {
  const unsigned blocks = static_cast<unsigned>((count + 63) / 64);
  switch (D) {
#define HGF_SPD(d)                                                                        \
  case d:                                                                                 \
    if constexpr (d >= 11) {                                                              \
      const unsigned lb = static_cast<unsigned>((count + gk::kSpdPerBlock - 1) / gk::kSpdPerBlock); \
      hipLaunchKernelGGL(gk::spd_inverse_lanes_kernel<d>, dim3(lb), dim3(gk::kSpdPerBlock * gk::kLpp), 0, \
                         s, a, minv, count);                                              \
    } else {                                                                              \
      hipLaunchKernelGGL(gk::spd_inverse_kernel<d>, dim3(blocks), dim3(64), 0, s, a, minv,     \
                         count);                                                          \
    }                                                                                     \
    return hipGetLastError();
    HGF_SPD(1)
    HGF_SPD(2)
    HGF_SPD(3)
    HGF_SPD(4)
    HGF_SPD(5)
    HGF_SPD(6)
    HGF_SPD(7)
    HGF_SPD(8)
    HGF_SPD(9)
    HGF_SPD(10)
    HGF_SPD(11)
    HGF_SPD(12)
    HGF_SPD(13)
    HGF_SPD(14)
    HGF_SPD(15)
    HGF_SPD(16)
    HGF_SPD(17)
    HGF_SPD(18)
    HGF_SPD(19)
    HGF_SPD(20)
#undef HGF_SPD
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace hgf