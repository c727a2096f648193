// a6 + a7: coefficient box filter, output and winner-takes-all.
//
// Z(q) = (sum_i B(a_i)(q) G_i(q) + B(b)(q)) / N_q      (Eq. 11, Eq. 7)
// label(q) = argmin_l Z_l(q), lowest label on ties     (Sec. 1)
//
// Same strip mapping as the coefficient kernel: lanes are 64 labels of one
// pixel, waves split the n + 1 coefficient channels and keep float32
// vertical running sums of their channels over the strip's state columns in
// registers; horizontal sums are float64 running sums in registers.  Each
// wave forms the partial dot product of its channels with the (wave-uniform)
// guidance at every output column; the partials meet in LDS and are summed in
// a fixed order, so Z does not depend on scheduling.  The winner-takes-all
// key (ordered cost bits << 32 | label) of the 64 lanes is formed from the
// lanes' minimum (DPP row minima, then the four row values) and the lowest
// lane holding it, and merged into a per-pixel 64-bit minimum; the minimum
// of keys is order independent, so label chunks may run concurrently.  When
// all labels are in one chunk the label itself is written instead.
//
// With one channel per wave a row step loads the entering and the leaving row
// of the vertical window together, a group of columns at a time, so each
// group costs one memory round trip.  Strips that lie inside the image take a
// path without column bounds handling; the two border strips clamp their
// addresses and weight out-of-image columns by zero.
#pragma once

#include "hgf_launch.hpp"

namespace hgf {
// LDS for the per-wave partial dot products (float64) of one column chunk:
// 12 KB per wave, at most 120 KB.  Blocks of few waves (few channels) then
// leave room for more blocks per CU, so every layout keeps about ten or more
// waves per CU resident.
constexpr int out_part_bytes(int nw) { return nw * 12 * 1024 < 120 * 1024 ? nw * 12 * 1024 : 120 * 1024; }

template <int NW, int SOUT>
constexpr int out_column_chunk() {
  int oc = out_part_bytes(NW) / (NW * 64 * 8);
  if (oc > SOUT) oc = SOUT;
  if (oc < 1) oc = 1;
  const int ncb = (SOUT + oc - 1) / oc;
  return (SOUT + ncb - 1) / ncb;  // balanced chunks
}

// One vertical window update of every state column: coefficient SA (0, +1)
// times row ya and SS (0, +1, -1) times row ys.
template <int SA, int SS, bool CHECK, int CPW, int NCH, int SIN, int GRP>
__device__ __forceinline__ void out_vrow(float (&vs)[CPW][SIN], const float* __restrict__ wsc,
                                         int ya, int ys, int xsl, int W, int wv, int lane) {
  const size_t stride = static_cast<size_t>(W) * NCH * 64;
  // (buffer loads with scalar column offsets measured slower here than
  // global loads with vector addresses)
  const float* __restrict__ ga = wsc + static_cast<size_t>(SA != 0 ? ya : 0) * stride;
  const float* __restrict__ gs = wsc + static_cast<size_t>(SS != 0 ? ys : 0) * stride;
#pragma unroll
  for (int c0 = 0; c0 < SIN; c0 += GRP) {
    float e[CPW][GRP];
    float l[CPW][GRP];
#pragma unroll
    for (int c = 0; c < GRP; ++c) {
      if (c0 + c < SIN) {
        const int xr = xsl + c0 + c;
        const int xc = CHECK ? min(max(xr, 0), W - 1) : xr;
#pragma unroll
        for (int k = 0; k < CPW; ++k) {
          const int ch = (NCH % CPW == 0) ? wv * CPW + k : min(wv * CPW + k, NCH - 1);
          const uint32_t off = (static_cast<uint32_t>(xc) * NCH + ch) * 64u + lane;
          if (SA != 0) e[k][c] = ga[off];
          if (SS != 0) l[k][c] = gs[off];
        }
      }
    }
#pragma unroll
    for (int c = 0; c < GRP; ++c) {
      if (c0 + c < SIN) {
        const int xr = xsl + c0 + c;
#pragma unroll
        for (int k = 0; k < CPW; ++k) {
          const bool chok = (NCH % CPW == 0) || (wv * CPW + k < NCH);
          float& v = vs[k][c0 + c];
          if (CHECK || NCH % CPW != 0) {
            const bool ok = chok && (!CHECK || (xr >= 0 && xr < W));
            const float w = ok ? 1.f : 0.f;
            if (SA != 0) v = fmaf(w, e[k][c], v);
            if (SS > 0) v = fmaf(w, l[k][c], v);
            if (SS < 0) v = fmaf(-w, l[k][c], v);
          } else {
            if (SA != 0) v += e[k][c];
            if (SS > 0) v += l[k][c];
            if (SS < 0) v -= l[k][c];
          }
        }
      }
    }
    // keep the next group's loads from being hoisted into this one (the
    // registers they would hold are needed by the running sums)
    __builtin_amdgcn_sched_barrier(0);
  }
}

template <int R, int CPW, int NG, int SIN, int GRP, bool PAIR, bool CHECK>
__device__ __forceinline__ void out_strip(const float* __restrict__ wsc,
                                          const float* __restrict__ g32, float* __restrict__ out,
                                          int out_ld, unsigned long long* __restrict__ keys,
                                          int32_t* __restrict__ labels, int label_base, int H, int W, int xs, int x_out0,
                                          int y0, int y1, bool up, int lab, bool lab_ok, int wv,
                                          int lane, double* __restrict__ part) {
  constexpr int NCH = NG + 1;
  constexpr int NW = (NCH + CPW - 1) / CPW;
  constexpr int SOUT = SIN - 2 * R;
  constexpr int OC = out_column_chunk<NW, SOUT>();
  constexpr int NCB = (SOUT + OC - 1) / OC;
  const size_t P = static_cast<size_t>(H) * W;

  float vs[CPW][SIN];
#pragma unroll
  for (int k = 0; k < CPW; ++k)
#pragma unroll
    for (int c = 0; c < SIN; ++c) vs[k][c] = 0.f;

  // The strip origin is laundered so that per-column offsets are recomputed
  // for each row rather than hoisted out of the row loop (they would spill).
  auto launder = [&]() {
    int xsl = __builtin_amdgcn_readfirstlane(xs);
    asm volatile("" : "+s"(xsl));
    return __builtin_amdgcn_readfirstlane(xsl);
  };

  // Even bands run upward from their last row, odd bands downward from their
  // first: the two blocks of a band boundary then start on nearly the same
  // 2R + 1 rows at the same time (and end on the same rows at their other
  // boundaries), so the start-up rows are shared through L2 rather than read
  // twice from HBM.
  const int ystart = up ? y1 - 1 : y0;
  // initial window: rows ystart - R .. ystart + R; with one channel per wave
  // two rows at a time in groups of 32 columns (small images are mostly
  // start-up, and each group is one memory round trip)
  {
    constexpr int GI = CPW == 1 ? 32 : GRP;
    const int ra = max(0, ystart - R), rb = min(H - 1, ystart + R);
    int yy = ra;
    for (; (PAIR || CPW == 1) && yy + 1 <= rb; yy += 2)
      out_vrow<1, 1, CHECK, CPW, NCH, SIN, GI>(vs, wsc, yy, yy + 1, launder(), W, wv, lane);
    for (; yy <= rb; ++yy) out_vrow<1, 0, CHECK, CPW, NCH, SIN, GRP>(vs, wsc, yy, 0, launder(), W, wv, lane);
  }
  const int dir = up ? -1 : 1;
  for (int t = 0; t < y1 - y0; ++t) {
    const int y = ystart + dir * t;
    if (t > 0) {
      // the row entering the window and the row leaving it
      const int ye = y + dir * R, yl = y - dir * (R + 1);
      const bool a = ye >= 0 && ye < H, s = yl >= 0 && yl < H;
      if (PAIR && a && s) {
        out_vrow<1, -1, CHECK, CPW, NCH, SIN, GRP>(vs, wsc, ye, yl, launder(), W, wv, lane);
      } else {
        if (a) out_vrow<1, 0, CHECK, CPW, NCH, SIN, GRP>(vs, wsc, ye, 0, launder(), W, wv, lane);
        if (s) out_vrow<0, -1, CHECK, CPW, NCH, SIN, GRP>(vs, wsc, 0, yl, launder(), W, wv, lane);
      }
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
              // fresh conversions each step: keeping converted values alive
              // for 2R + 1 steps would double the register footprint
              float a = vs[k][j + 2 * R], b = vs[k][j - 1];
              asm volatile("" : "+v"(a), "+v"(b));
              hs[k] += static_cast<double>(a) - static_cast<double>(b);
            }
          }
          // guidance at output column x_out0 + j (planar, consecutive in j;
          // columns past the image read the next row or the padding, and
          // their partials are never used)
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
#pragma unroll
          for (int w = 0; w < NW; ++w) z += part[(w * OC + q) * 64 + lane];
          z /= static_cast<double>(window_count(x, y, W, H, R));
          const float zf = static_cast<float>(z);
          if (out != nullptr && lab_ok) out[p * out_ld + lab] = zf;
          if (keys != nullptr || labels != nullptr) {
            // lowest ordered cost of the 64 labels, then the lowest lane
            // holding it (labels increase with the lane)
            const uint32_t u = lab_ok ? ordered_bits(zf) : 0xffffffffu;
            const uint32_t m = wave_min_u32(u);
            const int first = __builtin_ctzll(__ballot(u == m));
            // both halves are wave-uniform; say so, so the atomic is issued once
            const uint32_t hi = __builtin_amdgcn_readfirstlane(m);
            const uint32_t lo = __builtin_amdgcn_readfirstlane(label_base + (lab - lane) + first);
            const unsigned long long key = (static_cast<unsigned long long>(hi) << 32) | lo;
            if (lane == 0) {
              // all labels in this one chunk: the label is final
              if (labels != nullptr)
                labels[p] = static_cast<int32_t>(lo);
              else
                atomicMin(&keys[p], key);
            }
          }
        }
      }
      __syncthreads();
    }
  }
}

template <int R, int CPW, int NG, int SIN, int GRP, bool PAIR>
__global__ __launch_bounds__(640) void out_kernel(
    const float* __restrict__ ws, const float* __restrict__ g32, float* __restrict__ out,
    int out_ld, unsigned long long* __restrict__ keys, int32_t* __restrict__ labels,
    int label_base, int H, int W,
    int label_count, int band_h, int strips, int bands) {
  constexpr int NCH = NG + 1;
  constexpr int NW = (NCH + CPW - 1) / CPW;
  constexpr int SOUT = SIN - 2 * R;
  constexpr int OC = out_column_chunk<NW, SOUT>();
  __shared__ double part[NW * OC * 64];

  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // work item of this block; integer division runs on the vector ALU, so the
  // results are moved back to scalar registers explicitly
  // logical order: label chunk fastest, then the two bands of a band pair
  // (which share their start-up rows), then strip, then band pair; a last
  // unpaired band comes after all pairs.  Each XCD gets a contiguous range.
  int bid = xcd_remap(static_cast<int>(blockIdx.x), static_cast<int>(gridDim.x));
  const int chunks = __builtin_amdgcn_readfirstlane(static_cast<int>(gridDim.x) / (strips * bands));
  const int paired = (bands / 2) * 2;
  const int chunk = __builtin_amdgcn_readfirstlane(bid % chunks);
  int strip, band;
  if (bid < strips * paired * chunks) {
    bid = __builtin_amdgcn_readfirstlane(bid / chunks);
    const int par = bid & 1;
    bid >>= 1;
    strip = __builtin_amdgcn_readfirstlane(bid % strips);
    band = __builtin_amdgcn_readfirstlane((bid / strips) * 2 + par);
  } else {
    strip = __builtin_amdgcn_readfirstlane((bid - strips * paired * chunks) / chunks);
    band = paired;
  }
  const int x_out0 = strip * SOUT;
  const int xs = x_out0 - R;
  const int y0 = band * band_h;
  const int y1 = min(H, y0 + band_h);
  const int lab = chunk * 64 + lane;
  const bool lab_ok = lab < label_count;
  const size_t P = static_cast<size_t>(H) * W;
  const float* __restrict__ wsc = ws + static_cast<size_t>(chunk) * P * NCH * 64;
  if (xs >= 0 && xs + SIN <= W)
    out_strip<R, CPW, NG, SIN, GRP, PAIR, false>(wsc, g32, out, out_ld, keys, labels, label_base, H, W,
                                                 xs,
                                           x_out0, y0, y1, (band & 1) == 0, lab, lab_ok, wv, lane, part);
  else
    out_strip<R, CPW, NG, SIN, GRP, PAIR, true>(wsc, g32, out, out_ld, keys, labels, label_base, H, W,
                                                 xs,
                                          x_out0, y0, y1, (band & 1) == 0, lab, lab_ok, wv, lane, part);
}

template <int R, int NG>
hipError_t out_launch_t(const OutLaunch& a, hipStream_t s) {
  constexpr int CPW = out_channels_per_wave(NG);
  constexpr int SIN = out_strip_width(NG, R);
  constexpr int GRP = 8;
  // one channel per wave and eight or nine channels: the entering and the
  // leaving row are loaded together; otherwise one row at a time (there the
  // pair spills registers)
  constexpr bool PAIR = CPW == 1 && NG >= 8;
  constexpr int NW = (NG + 1 + CPW - 1) / CPW;
  const StripGrid& g = a.grid;
  const unsigned blocks = static_cast<unsigned>(g.strips * g.bands * g.chunks);
  hipLaunchKernelGGL((out_kernel<R, CPW, NG, SIN, GRP, PAIR>), dim3(blocks), dim3(NW * 64), 0, s, a.ws,
                     a.g32, a.out, a.out_ld, a.keys, a.labels, a.label_base, a.H, a.W, a.label_count,
                     g.band_h, g.strips, g.bands);
  return hipGetLastError();
}

// Every compiled radius of one channel count.
template <int NG>
hipError_t out_launch_n(const OutLaunch& a, hipStream_t s) {
  static_assert(kMinRadius == 0 && kMaxRadius == 9, "the radius list below");
  switch (a.R) {
    case 0: return out_launch_t<0, NG>(a, s);
    case 1: return out_launch_t<1, NG>(a, s);
    case 2: return out_launch_t<2, NG>(a, s);
    case 3: return out_launch_t<3, NG>(a, s);
    case 4: return out_launch_t<4, NG>(a, s);
    case 5: return out_launch_t<5, NG>(a, s);
    case 6: return out_launch_t<6, NG>(a, s);
    case 7: return out_launch_t<7, NG>(a, s);
    case 8: return out_launch_t<8, NG>(a, s);
    case 9: return out_launch_t<9, NG>(a, s);
    default: return hipErrorNotSupported;
  }
}

}  // namespace hgf
