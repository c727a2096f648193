// Winner-takes-all key handling, the standalone box sum and the dispatch of
// the output kernels (a6 + a7) over the compiled channel counts.  The output
// kernel itself is in out.hpp, instantiated per channel count in out_n*.hip.
#include "hgf_launch.hpp"

namespace hgf {
namespace {

__global__ __launch_bounds__(256) void key_fill_kernel(unsigned long long* __restrict__ keys,
                                                       size_t count) {
  const size_t i = static_cast<size_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i < count) keys[i] = ~0ull;
}

__global__ __launch_bounds__(256) void key_finalize_kernel(
    const unsigned long long* __restrict__ keys, size_t count, float* __restrict__ best,
    int32_t* __restrict__ labels, int merge) {
  const size_t i = static_cast<size_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i >= count) return;
  unsigned long long key = keys[i];
  if (merge) {
    const float ob = best != nullptr ? best[i] : 0.f;
    const int ol = labels != nullptr ? labels[i] : 0;
    const unsigned long long old = wta_key(ob, ol);
    if (old <= key) return;
  }
  if (best != nullptr) best[i] = ordered_to_float(static_cast<uint32_t>(key >> 32));
  if (labels != nullptr) labels[i] = static_cast<int32_t>(key & 0xffffffffu);
}

// Standalone box sum: vertical running sums per (channel, column), then a
// horizontal window sum per pixel read from the vertical result.
__global__ __launch_bounds__(256) void box_vertical_kernel(const float* __restrict__ in,
                                                           float* __restrict__ tmp, int C, int H,
                                                           int W, int R) {
  const int idx = static_cast<int>(blockIdx.x) * 256 + threadIdx.x;
  if (idx >= C * W) return;
  const int c = idx / W;
  const int x = idx - c * W;
  const float* src = in + static_cast<size_t>(c) * H * W + x;
  float* dst = tmp + static_cast<size_t>(c) * H * W + x;
  float s = 0.f;
  for (int y = 0; y <= min(R, H - 1); ++y) s += src[static_cast<size_t>(y) * W];
  for (int y = 0; y < H; ++y) {
    if (y > 0) {
      if (y + R < H) s += src[static_cast<size_t>(y + R) * W];
      if (y - R - 1 >= 0) s -= src[static_cast<size_t>(y - R - 1) * W];
    }
    dst[static_cast<size_t>(y) * W] = s;
  }
}

__global__ __launch_bounds__(256) void box_horizontal_kernel(const float* __restrict__ tmp,
                                                             float* __restrict__ out, int C,
                                                             int H, int W, int R) {
  const size_t idx = static_cast<size_t>(blockIdx.x) * 256 + threadIdx.x;
  const size_t total = static_cast<size_t>(C) * H * W;
  if (idx >= total) return;
  const size_t row = idx / W;
  const int x = static_cast<int>(idx - row * W);
  const float* src = tmp + row * W;
  float s = 0.f;
  for (int xx = max(0, x - R); xx <= min(W - 1, x + R); ++xx) s += src[xx];
  out[idx] = s;
}

}  // namespace

hipError_t launch_out(const OutLaunch& a, hipStream_t s) {
  switch (a.n) {
    case 1: return launch_out_n1(a, s);
    case 2: return launch_out_n2(a, s);
    case 3: return launch_out_n3(a, s);
    case 4: return launch_out_n4(a, s);
    case 5: return launch_out_n5(a, s);
    case 6: return launch_out_n6(a, s);
    case 7: return launch_out_n7(a, s);
    case 8: return launch_out_n8(a, s);
    case 9: return launch_out_n9(a, s);
    case 19: return launch_out_n19(a, s);
    default: return hipErrorNotSupported;
  }
}

hipError_t launch_key_fill(unsigned long long* keys, size_t count, hipStream_t s) {
  const unsigned blocks = static_cast<unsigned>((count + 255) / 256);
  hipLaunchKernelGGL(key_fill_kernel, dim3(blocks), dim3(256), 0, s, keys, count);
  return hipGetLastError();
}

hipError_t launch_key_finalize(const unsigned long long* keys, size_t count, float* best,
                               int32_t* labels, int merge, hipStream_t s) {
  const unsigned blocks = static_cast<unsigned>((count + 255) / 256);
  hipLaunchKernelGGL(key_finalize_kernel, dim3(blocks), dim3(256), 0, s, keys, count, best,
                     labels, merge);
  return hipGetLastError();
}

hipError_t launch_box_sum(const float* in, float* out, int C, int H, int W, int R, float* tmp,
                          hipStream_t s) {
  const unsigned b1 = static_cast<unsigned>((C * W + 255) / 256);
  hipLaunchKernelGGL(box_vertical_kernel, dim3(b1), dim3(256), 0, s, in, tmp, C, H, W, R);
  const size_t total = static_cast<size_t>(C) * H * W;
  const unsigned b2 = static_cast<unsigned>((total + 255) / 256);
  hipLaunchKernelGGL(box_horizontal_kernel, dim3(b2), dim3(256), 0, s, tmp, out, C, H, W, R);
  return hipGetLastError();
}

}  // namespace hgf
