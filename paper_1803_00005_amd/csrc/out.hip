// a6 + a7: coefficient box filter, output and winner-takes-all.
//
// Z(q) = (sum_i B(a_i)(q) G_i(q) + B(b)(q)) / N_q      (Eq. 11, Eq. 7)
// label(q) = argmin_l Z_l(q), lowest label on ties     (Sec. 1)
//
// Same strip mapping as the coefficient kernel: lanes are 64 labels of one
// pixel, waves split the n + 1 coefficient channels and keep float32
// vertical running sums of their channels over 64 state columns in
// registers; horizontal sums are float64 running sums in registers.  Each
// wave forms the partial dot product of its channels with the (wave-uniform)
// guidance at every output column; the partials meet in LDS and are summed in
// a fixed order, so Z does not depend on scheduling.  The winner-takes-all
// key (ordered cost bits << 32 | label) is reduced across the 64 lanes with
// shuffles and merged into a per-pixel 64-bit minimum; the minimum of keys
// is order independent, so label chunks may run concurrently.
#include "hgf_launch.hpp"

namespace hgf {
namespace {

constexpr int kOutMaxWaves = 10;

template <int R, int CPW, int SIN>
__global__ __launch_bounds__(640) void out_kernel(
    const float* __restrict__ ws, const float* __restrict__ g32, float* __restrict__ out,
    int out_ld, unsigned long long* __restrict__ keys, int label_base, int n, int H, int W,
    int label_count, int band_h, int strips, int bands) {
  constexpr int SOUT = SIN - 2 * R;
  constexpr int OC = SOUT < 10 ? SOUT : 10;
  __shared__ double part[kOutMaxWaves * OC * 64];

  const int NCH = n + 1;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int NW = __builtin_amdgcn_readfirstlane(blockDim.x >> 6);
  // work item of this block; integer division runs on the vector ALU, so the
  // results are moved back to scalar registers explicitly
  int bid = xcd_remap(static_cast<int>(blockIdx.x), static_cast<int>(gridDim.x));
  const int chunks = __builtin_amdgcn_readfirstlane(static_cast<int>(gridDim.x) / (strips * bands));
  const int chunk = __builtin_amdgcn_readfirstlane(bid % chunks);
  bid = __builtin_amdgcn_readfirstlane(bid / chunks);
  const int strip = __builtin_amdgcn_readfirstlane(bid % strips);
  const int band = __builtin_amdgcn_readfirstlane(bid / strips);
  const int x_out0 = strip * SOUT;
  const int xs = x_out0 - R;
  const int y0 = band * band_h;
  const int y1 = min(H, y0 + band_h);
  const int lab = chunk * 64 + lane;
  const bool lab_ok = lab < label_count;
  const size_t P = static_cast<size_t>(H) * W;
  const float* __restrict__ wsc = ws + static_cast<size_t>(chunk) * P * NCH * 64;

  float vs[CPW][SIN];
#pragma unroll
  for (int k = 0; k < CPW; ++k)
#pragma unroll
    for (int c = 0; c < SIN; ++c) vs[k][c] = 0.f;

  // Vertical update with row yy, kGrp columns of loads issued at a time;
  // columns outside the image read a clamped pixel with weight 0.
  auto acc_row = [&](int yy, bool add) {
    int xsl = __builtin_amdgcn_readfirstlane(xs);
    asm volatile("" : "+s"(xsl));
    xsl = __builtin_amdgcn_readfirstlane(xsl);
    // uniform row base + lane offset: loads use an SGPR base and one VGPR offset
    const float* __restrict__ row = wsc + static_cast<size_t>(yy) * W * NCH * 64;
    constexpr int GRP = CPW > 1 ? kGrp / 2 : kGrp;
#pragma unroll
    for (int c0 = 0; c0 < SIN; c0 += GRP) {
      float v[CPW][GRP];
#pragma unroll
      for (int c = 0; c < GRP; ++c) {
        const int xc = min(max(xsl + c0 + c, 0), W - 1);
#pragma unroll
        for (int k = 0; k < CPW; ++k) {
          const int ch = wv * CPW + k;
          const int chc = ch < NCH ? ch : NCH - 1;
          v[k][c] = row[(static_cast<uint32_t>(xc) * NCH + chc) * 64u + lane];
        }
      }
#pragma unroll
      for (int c = 0; c < GRP; ++c) {
        const int xr = xsl + c0 + c;
#pragma unroll
        for (int k = 0; k < CPW; ++k) {
          const int ch = wv * CPW + k;
          const bool ok = xr >= 0 && xr < W && ch < NCH;
          const float w = ok ? (add ? 1.f : -1.f) : 0.f;
          vs[k][c0 + c] = fmaf(w, v[k][c], vs[k][c0 + c]);
        }
      }
    }
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
    // Output columns in chunks of OC: the unrolled part touches only the
    // register state; the reduction over waves runs after it as a plain loop.
    constexpr int NCB = (SOUT + OC - 1) / OC;
    const size_t prow = static_cast<size_t>(y) * W + x_out0;
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
#pragma unroll
      for (int jj = 0; jj < OC; ++jj) {
        const int j = cb * OC + jj;
        if (j < SOUT) {
          if (j > 0) {
#pragma unroll
            for (int k = 0; k < CPW; ++k) {
              // fresh conversions each step (see the coefficient kernel)
              float a = vs[k][j + 2 * R], b = vs[k][j - 1];
              asm volatile("" : "+v"(a), "+v"(b));
              hs[k] += static_cast<double>(a) - static_cast<double>(b);
            }
          }
          // guidance at output column x_out0 + j (planar, consecutive in j;
          // columns past the image read padding and their partials are unused)
          double pj = 0.0;
#pragma unroll
          for (int k = 0; k < CPW; ++k) {
            const int ch = wv * CPW + k;
            const int chc = ch < NCH ? ch : NCH - 1;
            const float g = ldu(g32 + static_cast<size_t>(chc) * P + prow, j);
            pj = fma(hs[k], ch < NCH ? static_cast<double>(g) : 0.0, pj);
          }
          part[(wv * OC + jj) * 64 + lane] = pj;
        }
      }
      __syncthreads();
      const int cnt = min(OC, SOUT - cb * OC);
      for (int q = wv; q < cnt; q += NW) {
        const int x = x_out0 + cb * OC + q;
        if (x < W) {
          const size_t p = static_cast<size_t>(y) * W + x;
          double z = 0.0;
          for (int w = 0; w < NW; ++w) z += part[(w * OC + q) * 64 + lane];
          z /= static_cast<double>(window_count(x, y, W, H, R));
          const float zf = static_cast<float>(z);
          if (out != nullptr && lab_ok) out[p * out_ld + lab] = zf;
          if (keys != nullptr) {
            unsigned long long key = lab_ok ? wta_key(zf, label_base + lab) : ~0ull;
            key = wave_min_u64(key);
            if (lane == 0) atomicMin(&keys[p], key);
          }
        }
      }
      __syncthreads();
    }
  }
}

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

template <int R, int CPW>
hipError_t out_launch_t(const OutLaunch& a, hipStream_t s) {
  constexpr int SIN = out_strip_width(CPW);
  const int NCH = a.n + 1;
  const int NW = (NCH + CPW - 1) / CPW;
  const StripGrid& g = a.grid;
  const unsigned blocks = static_cast<unsigned>(g.strips * g.bands * g.chunks);
  hipLaunchKernelGGL((out_kernel<R, CPW, SIN>), dim3(blocks), dim3(NW * 64), 0, s, a.ws, a.g32, a.out,
                     a.out_ld, a.keys, a.label_base, a.n, a.H, a.W, a.label_count, g.band_h,
                     g.strips, g.bands);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_out(const OutLaunch& a, hipStream_t s) {
  const int NCH = a.n + 1;
  const bool two = NCH > kOutMaxWaves;
  if (NCH > 2 * kOutMaxWaves) return hipErrorNotSupported;
  switch (a.R) {
#define HGF_OUT_R(r) \
  case r:            \
    return two ? out_launch_t<r, 2>(a, s) : out_launch_t<r, 1>(a, s);
    HGF_OUT_R(1)
    HGF_OUT_R(2)
    HGF_OUT_R(4)
    HGF_OUT_R(7)
    HGF_OUT_R(9)
#undef HGF_OUT_R
    default:
      return hipErrorNotSupported;
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
