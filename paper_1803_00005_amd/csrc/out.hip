// Winner-takes-all key handling and the standalone box sum.  The output
// kernel (a6 + a7) is in out.hpp, instantiated per channel count in
// generated units and dispatched from dispatch.hip.
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

// Standalone box sum in one pass, no temporary: a block takes 64 output
// columns of one channel over a band of rows; its threads keep the vertical
// running sums of the 64 + 2R state columns (float32: exact for the integer
// test images, whose sums stay below 2^24), publish them in LDS each row, and
// the first 64 threads sum 2R + 1 neighbours for their output column.
constexpr int kBoxCols = 64;
constexpr int kBoxBand = 64;
constexpr int kBoxThreads = 256;  // 64 output columns plus 2R state columns, R <= 95

__global__ __launch_bounds__(kBoxThreads) void box_sum_kernel(const float* __restrict__ in,
                                                              float* __restrict__ out, int H,
                                                              int W, int R) {
  __shared__ float vrow[kBoxThreads];
  const int strip = static_cast<int>(blockIdx.x);
  const int band = static_cast<int>(blockIdx.y);
  const int c = static_cast<int>(blockIdx.z);
  const int t = static_cast<int>(threadIdx.x);
  const int x0 = strip * kBoxCols;
  const int xs = x0 - R + t;  // this thread's state column
  const bool state = t < kBoxCols + 2 * R && xs >= 0 && xs < W;
  const int y0 = band * kBoxBand;
  const int y1 = min(H, y0 + kBoxBand);
  const float* __restrict__ src = in + static_cast<size_t>(c) * H * W;
  float* __restrict__ dst = out + static_cast<size_t>(c) * H * W;
  float v = 0.f;
  if (state)
    for (int y = max(0, y0 - R); y <= min(H - 1, y0 + R); ++y)
      v += src[static_cast<size_t>(y) * W + xs];
  for (int y = y0; y < y1; ++y) {
    if (y > y0 && state) {
      if (y + R < H) v += src[static_cast<size_t>(y + R) * W + xs];
      if (y - R - 1 >= 0) v -= src[static_cast<size_t>(y - R - 1) * W + xs];
    }
    vrow[t] = state ? v : 0.f;
    __syncthreads();
    const int x = x0 + t;
    if (t < kBoxCols && x < W) {
      float h = 0.f;
      for (int k = 0; k <= 2 * R; ++k) h += vrow[t + k];
      dst[static_cast<size_t>(y) * W + x] = h;
    }
    __syncthreads();
  }
}

}  // namespace

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

hipError_t launch_box_sum(const float* in, float* out, int C, int H, int W, int R,
                          hipStream_t s) {
  if (kBoxCols + 2 * R > kBoxThreads) return hipErrorInvalidValue;
  const dim3 grid(static_cast<unsigned>((W + kBoxCols - 1) / kBoxCols),
                  static_cast<unsigned>((H + kBoxBand - 1) / kBoxBand), static_cast<unsigned>(C));
  hipLaunchKernelGGL(box_sum_kernel, grid, dim3(kBoxThreads), 0, s, in, out, H, W, R);
  return hipGetLastError();
}

}  // namespace hgf
