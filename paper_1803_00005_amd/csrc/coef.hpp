// a4 + a5: per-label box sums of the guidance x cost products and the per-pixel
// coefficient solve, fused.
//
// For every label slice Y of the cost volume and every pixel p (Sec. 4.3,
// Eq. 9 with Prop. 2; the covariance form of Sec. 5.1, Eqs. 12-13):
//   U = B(Y),  T_i = B(G_i Y)                       (window sums, i = 1..n)
//   covariance:  c = (T - mu U) / N_p,  a = M_p c,  b = U / N_p - a . mu
//   ridge:       [b; a] = M_p [U; T]               (M_p of the (n+1) system)
// with M_p the per-pixel inverse computed once per image.  The coefficient
// images [b, a_1..a_n] go to a float32 workspace [chunk][P][n+1][64].  The
// covariance solve runs in float32 from float32 records or in float64 from
// float64 records (the solve mode); the ridge solve runs in float64.
//
// Mapping (gfx950, wave64): the 64 lanes of a wave are 64 labels of one
// pixel.  Everything per-pixel (M_p, mu_p, G(p), N_p) is wave-uniform: M_p and
// mu_p come from 16-byte broadcast reads of LDS, G(p) from broadcast reads of
// the staged guidance, so the n x n times n x 64 product runs as plain VALU
// FMAs.  A workgroup owns a strip of SIN state columns (SIN - 2R output
// columns) over a band of rows.  Its waves split the n + 1 product channels:
// each wave keeps float32 vertical running sums of its channels for all state
// columns in registers (add the row entering the window, subtract the row
// leaving it) and forms the horizontal window sums in registers with float64
// running sums; the window sums T, U of a row are transposed through LDS
// before the solves, which all waves of the block share.  The cost rows, the
// guidance rows and the solve records reach LDS by direct-to-LDS loads issued
// ahead of their use.  Bands restart the vertical sums, which bounds float32
// drift to band_h + 2R additions.
//
// Strips inside the image take a path without column bounds handling; the two
// border strips clamp their addresses and weight out-of-image columns by zero.
#pragma once

#include <type_traits>

#include "hgf_launch.hpp"

namespace hgf {
// LDS for the transposed window sums of one row chunk: with up to ten
// channels one chunk holds the whole row; above, smaller chunks measured
// faster (the solves of a chunk start sooner).
constexpr int coef_lds_bytes(int nch) { return nch <= 10 ? 120 * 1024 : 50 * 1024; }

// Waves per block: one per channel group, rounded up to a multiple of the
// four SIMDs of a CU from eight groups on, so that the solves (shared by all
// waves) spread evenly over the SIMDs; with at most four groups, eight waves,
// so that the solves of few channels do not run on four waves alone.  The
// extra waves skip the box sums.
constexpr int coef_block_waves(int nw) { return nw >= 8 ? (nw + 3) / 4 * 4 : (nw <= 4 ? 8 : nw); }

// LDS of a block besides the transposed window sums: the staged inverses of
// one row and two staged cost rows.
template <int SOUT, int SIN, int NG, int MODE>
constexpr int coef_fixed_lds_bytes();

template <int NCH, int SOUT, int SIN, int MODE>
constexpr int coef_column_chunk() {
  constexpr int avail = 160 * 1024 - coef_fixed_lds_bytes<SOUT, SIN, NCH - 1, MODE>();
  constexpr int budget = coef_lds_bytes(NCH) < avail ? coef_lds_bytes(NCH) : avail;
  int oc = budget / (NCH * 64 * 4);
  if (oc > SOUT) oc = SOUT;
  if (oc < 1) oc = 1;
  const int ncb = (SOUT + oc - 1) / oc;
  return (SOUT + ncb - 1) / ncb;  // balanced chunks
}

// Cost rows pass through LDS: a slot holds the SIN state columns of one row,
// 64 labels each, one 32-bit word per (column, label).  The copies are direct global-to-LDS loads
// (no registers), issued cooperatively by all waves of the block one row
// step ahead of their use, so the vertical update reads LDS instead of
// waiting on global memory.  A 16-bit cost (bfloat16 or float16) lands in
// the low half of its word.
template <bool CHECK, int SIN, int NWB, typename TIN>
__device__ __forceinline__ void stage_cost_row(const TIN* __restrict__ cost, int cost_ld, int yy,
                                               int xsl, int W, int labc, float* __restrict__ slot,
                                               int wv) {
  const TIN* __restrict__ row = cost + static_cast<size_t>(yy) * W * cost_ld;
  for (int c = wv; c < SIN; c += NWB) {
    const int xr = xsl + c;
    const int xc = CHECK ? min(max(xr, 0), W - 1) : xr;
    typedef const __attribute__((address_space(1))) void* gsrc_t;
    typedef __attribute__((address_space(3))) void* ldst_t;
    const gsrc_t src = (gsrc_t)(row + static_cast<size_t>(xc) * cost_ld + labc);
    if constexpr (sizeof(TIN) == 2)
      __builtin_amdgcn_global_load_lds(src, (ldst_t)(slot + c * 64), 2, 0, 0);
    else
      __builtin_amdgcn_global_load_lds(src, (ldst_t)(slot + c * 64), 4, 0, 0);
  }
}

// The guidance rows of the same row steps: slot [NCH][64] floats, channel ch
// holding columns xs .. xs + 63 of the row (one direct-to-LDS load per
// channel; columns past the image read the padding around the planar
// guidance or a neighbouring row, and get weight 0).
template <int NCH, int NWB>
__device__ __forceinline__ void stage_guide_row(const float* __restrict__ g32, size_t P, int yy,
                                                int xsl, int W, float* __restrict__ slot, int wv,
                                                int lane) {
  typedef const __attribute__((address_space(1))) void* gsrc_t;
  typedef __attribute__((address_space(3))) void* ldst_t;
  for (int ch = wv; ch < NCH; ch += NWB) {
    const float* src = g32 + static_cast<size_t>(ch) * P + static_cast<size_t>(yy) * W + xsl + lane;
    __builtin_amdgcn_global_load_lds((gsrc_t)src, (ldst_t)(slot + ch * 64), 4, 0, 0);
  }
}

template <typename TIN>
__device__ __forceinline__ float lds_cost(const float* __restrict__ slot, int i) {
  if constexpr (sizeof(TIN) == 2) {
    return cost_bits_to_float<TIN>(reinterpret_cast<const uint16_t*>(slot)[2 * i]);
  } else {
    return slot[i];
  }
}

// One vertical window update of every state column from staged rows: SA (0,
// +1) times the products G_ch Y of row ya (slot sa) and SS (0, +1, -1) times
// those of row ys (slot ss).
template <int SA, int SS, bool CHECK, int CPW, int NCH, int SIN, typename TIN>
__device__ __forceinline__ void coef_vrow_lds(float (&vs)[CPW][SIN], const float* __restrict__ sa,
                                              const float* __restrict__ ss,
                                              const float4* __restrict__ g4, int xsl, int W,
                                              int wv, int lane) {
  // columns per group: LDS latency is short, so a small group suffices and
  // keeps registers (and, with two channels, scalar registers for the
  // guidance values) free
  constexpr int G = 8 / CPW;
  static_assert(G % 4 == 0 || SIN % 4 == 0, "guidance reads are 16-byte groups");
  // the lane's word in a slot, held in one vector register: every read then
  // addresses it with an immediate column offset
  int il = lane;
  asm volatile("" : "+v"(il));
#pragma unroll
  for (int c0 = 0; c0 < SIN; c0 += G) {
    float ea[G], es[G];
#pragma unroll
    for (int c = 0; c < G; ++c) {
      if (c0 + c < SIN) {
        if (SA != 0) ea[c] = lds_cost<TIN>(sa, il + (c0 + c) * 64);
        if (SS != 0) es[c] = lds_cost<TIN>(ss, il + (c0 + c) * 64);
      }
    }
#pragma unroll
    for (int k = 0; k < CPW; ++k) {
      const int ch = wv * CPW + k;
      const int chc = (NCH % CPW == 0) ? ch : min(ch, NCH - 1);
      // guidance of this channel at the group's columns: 16-byte broadcast
      // reads from one vector-register base (slot 1 lies NCH * 16 units on)
      int gb = chc * 16;
      asm volatile("" : "+v"(gb));
      float gav[G], gsv[G];
#pragma unroll
      for (int c4 = 0; c4 < G; c4 += 4) {
        if (SA != 0) {
          const float4 q = g4[gb + (c0 + c4) / 4];
          gav[c4] = q.x; gav[c4 + 1] = q.y; gav[c4 + 2] = q.z; gav[c4 + 3] = q.w;
        }
        if (SS != 0) {
          const float4 q = g4[gb + NCH * 16 + (c0 + c4) / 4];
          gsv[c4] = q.x; gsv[c4 + 1] = q.y; gsv[c4 + 2] = q.z; gsv[c4 + 3] = q.w;
        }
      }
#pragma unroll
      for (int c = 0; c < G; ++c) {
        if (c0 + c < SIN) {
          const int xr = xsl + c0 + c;
          const bool ok = ((NCH % CPW == 0) || ch < NCH) && (!CHECK || (xr >= 0 && xr < W));
          float& v = vs[k][c0 + c];
          if (SA != 0) v = fmaf(ok ? gav[c] : 0.f, ea[c], v);
          if (SS != 0) v = fmaf(ok ? (SS > 0 ? gsv[c] : -gsv[c]) : 0.f, es[c], v);
        }
      }
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Copy `dwords` consecutive dwords from global memory into LDS without
// passing through registers (global_load_lds, asynchronous: the copy is
// complete after the issuing wave's vmcnt reaches zero, visible to the other
// waves after the next barrier).  Lanes past the end re-read the last dword
// into the padding of the LDS buffer, so no lane reads outside the source.
template <int NW>
__device__ __forceinline__ void stage_dwords(const uint32_t* __restrict__ src,
                                             uint32_t* __restrict__ dst, int dwords, int wv,
                                             int lane) {
  for (int base = wv * 64; base < dwords; base += NW * 64) {
    const int i = min(base + lane, dwords - 1);
    __builtin_amdgcn_global_load_lds(src + i, dst + base, 4, 0, 0);
  }
}

// Dwords of LDS for the stored inverses (covariance form: the solve records
// with the window means) of one row of a strip, rounded up to whole waves.
template <int SOUT, int NG, int MODE>
constexpr int coef_stage_dwords() {
  constexpr int m = SOUT * minv_stride(MODE, NG) * (minv_elem_bytes(MODE) / 4);
  return (m + 63) / 64 * 64;
}

template <int SOUT, int SIN, int NG, int MODE>
constexpr int coef_fixed_lds_bytes() {
  return coef_stage_dwords<SOUT, NG, MODE>() * 4 + 2 * SIN * 64 * 4 + 2 * (NG + 1) * 64 * 4;
}

// Reads element e of a float record at 16-byte unit `base` of an LDS array,
// one 16-byte load per group of four elements.  Used with compile-time
// indices in increasing order, so each load is issued once and its registers
// are freed after the group.  The base index is held in a vector register so
// that every load addresses it with an immediate offset.
struct RecordReader {
  const float4* __restrict__ lds4;
  int base;
  float4 cur;
  int k = -1;
  __device__ __forceinline__ RecordReader(const float4* a, int b) : lds4(a), base(b) {
    asm volatile("" : "+v"(base));
  }
  __device__ __forceinline__ float operator()(int e) {
    if (e / 4 != k) {
      k = e / 4;
      cur = lds4[base + k];
    }
    switch (e % 4) {
      case 0: return cur.x;
      case 1: return cur.y;
      case 2: return cur.z;
      default: return cur.w;
    }
  }
};

// The same for float64 records: one 16-byte load per pair of elements.
struct RecordReader64 {
  const double2* __restrict__ lds2;
  int base;
  double2 cur;
  int k = -1;
  __device__ __forceinline__ RecordReader64(const double2* a, int b) : lds2(a), base(b) {
    asm volatile("" : "+v"(base));
  }
  __device__ __forceinline__ double operator()(int e) {
    if (e / 2 != k) {
      k = e / 2;
      cur = lds2[base + k];
    }
    return (e % 2) == 0 ? cur.x : cur.y;
  }
};

template <int R, int CPW, int NG, int MODE, typename TIN, int SIN, bool CHECK>
__device__ __forceinline__ void coef_strip(const TIN* __restrict__ cost, int cost_ld,
                                           const float* __restrict__ g32,
                                           const void* __restrict__ minv_void,
                                           float* __restrict__ wsc, int H, int W, int xs,
                                           int x_out0, int y0, int y1, int labc, int wv, int lane,
                                           float* __restrict__ lds, uint32_t* __restrict__ stage,
                                           float* __restrict__ cbuf, float* __restrict__ gbuf) {
  constexpr int SOUT = SIN - 2 * R;
  constexpr int NCH = NG + 1;
  constexpr int NW = (NCH + CPW - 1) / CPW;
  constexpr int NWB = coef_block_waves(NW);
  constexpr bool RIDGE = MODE == kSolveRidge;
  constexpr int D = RIDGE ? NG + 1 : NG;
  using MT = typename std::conditional<MODE != kSolveCov32, double, float>::type;
  const MT* __restrict__ minv = static_cast<const MT*>(minv_void);
  // inverse elements read from LDS per scheduling block of the product
  constexpr int MBLK = MODE == kSolveCov32 ? 16 : 8;
  constexpr int OC = coef_column_chunk<NCH, SOUT, SIN, MODE>();
  constexpr int NCB = (SOUT + OC - 1) / OC;
  const size_t P = static_cast<size_t>(H) * W;

  float vs[CPW][SIN];
#pragma unroll
  for (int k = 0; k < CPW; ++k)
#pragma unroll
    for (int c = 0; c < SIN; ++c) vs[k][c] = 0.f;

  // The strip origin is laundered so that the per-column offsets are
  // recomputed for each row rather than hoisted out of the row loop (64 live
  // offsets would spill).
  auto launder = [&]() {
    int xsl = __builtin_amdgcn_readfirstlane(xs);
    asm volatile("" : "+s"(xsl));
    return __builtin_amdgcn_readfirstlane(xsl);
  };

  // this row's stored inverses (covariance form: solve records [SOUT][RW]),
  // staged in LDS at the start of the row step
  constexpr int RW = minv_stride(MODE, NG);
  const MT* __restrict__ sm = reinterpret_cast<const MT*>(stage);

  auto solve_store = [&](int x, int y, int q, int qx) {
    const size_t p = static_cast<size_t>(y) * W + x;
    float T[NCH];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) T[ch] = lds[(q * NCH + ch) * 64 + lane];
    const MT* __restrict__ mp = sm + qx * RW;
    float* __restrict__ o = wsc + p * NCH * 64 + lane;
    if constexpr (MODE == kSolveCov32) {
      // c = (T - mu U) / N, a = M c, b = U / N - a . mu, all float32: T is
      // float32 already and each fused multiply-add rounds once, so c and b
      // carry rounding errors of the order of T's own.
      const float invN = __builtin_amdgcn_rcpf(static_cast<float>(window_count(x, y, W, H, R)));
      const float U = T[0];
      const float4* __restrict__ st4 = reinterpret_cast<const float4*>(stage);
      RecordReader rd(st4, qx * (RW / 4));
      float c[NG];
      float av[NG];
#pragma unroll
      for (int i = 0; i < NG; ++i) {
        c[i] = fmaf(-rd(i), U, T[i + 1]) * invN;
        av[i] = 0.f;
      }
#pragma unroll
      for (int i = 0; i < NG; ++i) {
#pragma unroll
        for (int j = i; j < NG; ++j) {
          const int qq = packed_index(i, j, D);
          // bound the LDS reads in flight (each holds registers)
          if ((NG + qq) % MBLK == 0) __builtin_amdgcn_sched_barrier(0);
          const float m = rd(NG + qq);
          av[i] = fmaf(m, c[j], av[i]);
          if (j != i) av[j] = fmaf(m, c[i], av[j]);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
      RecordReader rm(st4, qx * (RW / 4));
      float b = U * invN;
#pragma unroll
      for (int i = 0; i < NG; ++i) b = fmaf(-av[i], rm(i), b);
      o[0] = b;
#pragma unroll
      for (int i = 0; i < NG; ++i) o[(i + 1) * 64] = av[i];
    } else if constexpr (MODE == kSolveCov64) {
      // the same in float64, from the float64 record: c = (T - mu U) / N,
      // a = M c, b = U / N - a . mu; only T itself is float32
      const double invN = 1.0 / static_cast<double>(window_count(x, y, W, H, R));
      const double U = static_cast<double>(T[0]);
      const double2* __restrict__ st2 = reinterpret_cast<const double2*>(stage);
      RecordReader64 rd(st2, qx * (RW / 2));
      double c[NG];
      double av[NG];
#pragma unroll
      for (int i = 0; i < NG; ++i) {
        c[i] = fma(-rd(i), U, static_cast<double>(T[i + 1])) * invN;
        av[i] = 0.0;
      }
#pragma unroll
      for (int i = 0; i < NG; ++i) {
#pragma unroll
        for (int j = i; j < NG; ++j) {
          const int qq = packed_index(i, j, D);
          if ((NG + qq) % MBLK == 0) __builtin_amdgcn_sched_barrier(0);
          const double m = rd(NG + qq);
          av[i] = fma(m, c[j], av[i]);
          if (j != i) av[j] = fma(m, c[i], av[j]);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
      RecordReader64 rm(st2, qx * (RW / 2));
      double b = U * invN;
#pragma unroll
      for (int i = 0; i < NG; ++i) b = fma(-av[i], rm(i), b);
      o[0] = static_cast<float>(b);
#pragma unroll
      for (int i = 0; i < NG; ++i) o[(i + 1) * 64] = static_cast<float>(av[i]);
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
#pragma unroll
        for (int j = i; j < D; ++j) {
          const int qq = packed_index(i, j, D);
          if (qq % MBLK == 0) __builtin_amdgcn_sched_barrier(0);
          const double m = static_cast<double>(mp[qq]);
          w[i] = fma(m, v[j], w[i]);
          if (j != i) w[j] = fma(m, v[i], w[j]);
        }
      }
#pragma unroll
      for (int i = 0; i < D; ++i) o[i * 64] = static_cast<float>(w[i]);
    }
  };

  // Stage the inverses and means of row y's output pixels into LDS.  Issued
  // before the row's vertical update so the copy overlaps it; the barrier
  // before the solves makes it visible (the previous row's solves are past
  // their closing barrier, so the buffer is free).
  auto stage_row = [&](int y) {
    const int cnt = min(SOUT, W - x_out0);
    const size_t p0 = static_cast<size_t>(y) * W + x_out0;
    stage_dwords<NWB>(reinterpret_cast<const uint32_t*>(minv + p0 * RW), stage,
                     cnt * RW * (minv_elem_bytes(MODE) / 4), wv, lane);
  };

  // waves past the channel groups (wv >= NW) only stage and solve
  const bool box_wave = NWB == NW || wv < NW;
  float* __restrict__ slot0 = cbuf;
  float* __restrict__ slot1 = cbuf + SIN * 64;
  float* __restrict__ gslot0 = gbuf;
  float* __restrict__ gslot1 = gbuf + NCH * 64;
  const float4* __restrict__ g40 = reinterpret_cast<const float4*>(gslot0);
  // cost and guidance of row yy into a cost slot and a guidance slot
  auto stage_to = [&](int yy, float* cs, float* gs) {
    stage_cost_row<CHECK, SIN, NWB, TIN>(cost, cost_ld, yy, launder(), W, labc, cs, wv);
    stage_guide_row<NCH, NWB>(g32, P, yy, launder(), W, gs, wv, lane);
  };
  auto stage_cost = [&](int yy, int sl) {
    stage_to(yy, sl ? slot1 : slot0, sl ? gslot1 : gslot0);
  };

  // Initial window of the band, rows y0 - R .. y0 + R.  The window-sum area
  // is free until the first row's horizontal sums, so it holds XS more staged
  // rows (their cost slots first, then their guidance slots, each guidance
  // slot NCH * 64 floats after the previous one like the two main slots):
  // 2 + XS rows per round, consumed in pairs.
  {
    constexpr int XS = (OC * NCH * 64) / (SIN * 64 + NCH * 64);
    constexpr int QR = 2 + XS;
    auto xcost = [&](int e) { return lds + e * SIN * 64; };
    auto xguide = [&](int e) { return lds + XS * SIN * 64 + e * NCH * 64; };
    const int ra = max(0, y0 - R), rb = min(H - 1, y0 + R);
    for (int y00 = ra; y00 <= rb; y00 += QR) {
      const int cnt = min(QR, rb - y00 + 1);
      stage_cost(y00, 0);
      if (cnt > 1) stage_cost(y00 + 1, 1);
      for (int e = 0; e + 2 < cnt; ++e) stage_to(y00 + 2 + e, xcost(e), xguide(e));
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (box_wave) {
        if (cnt > 1)
          coef_vrow_lds<1, 1, CHECK, CPW, NCH, SIN, TIN>(vs, slot0, slot1, g40, launder(),
                                                       W, wv, lane);
        else
          coef_vrow_lds<1, 0, CHECK, CPW, NCH, SIN, TIN>(vs, slot0, slot1, g40, launder(),
                                                       W, wv, lane);
        for (int e = 0; e + 2 < cnt; e += 2) {
          const float4* gx = reinterpret_cast<const float4*>(xguide(e));
          if (e + 3 < cnt)
            coef_vrow_lds<1, 1, CHECK, CPW, NCH, SIN, TIN>(vs, xcost(e), xcost(e + 1), gx,
                                                           launder(), W, wv, lane);
          else
            coef_vrow_lds<1, 0, CHECK, CPW, NCH, SIN, TIN>(vs, xcost(e), xcost(e), gx,
                                                           launder(), W, wv, lane);
        }
      }
      __syncthreads();
    }
  }
  for (int y = y0; y < y1; ++y) {
    stage_row(y);
    // rows y + R (slot 0) and y - R - 1 (slot 1) were staged during the
    // previous row step
    if (box_wave && y > y0) {
      const bool a = y + R < H, sb = y - R - 1 >= 0;
      if (a && sb)
        coef_vrow_lds<1, -1, CHECK, CPW, NCH, SIN, TIN>(vs, slot0, slot1, g40, launder(), W,
                                                        wv, lane);
      else if (a)
        coef_vrow_lds<1, 0, CHECK, CPW, NCH, SIN, TIN>(vs, slot0, slot1, g40, launder(),
                                                       W, wv, lane);
      else if (sb)
        coef_vrow_lds<0, -1, CHECK, CPW, NCH, SIN, TIN>(vs, slot0, slot1, g40, launder(),
                                                       W, wv, lane);
    }
    double hs[CPW];
#pragma unroll
    for (int k = 0; k < CPW; ++k) {
      hs[k] = 0.0;
#pragma unroll
      for (int c = 0; c <= 2 * R; ++c) hs[k] += static_cast<double>(vs[k][c]);
    }
    // Output columns in LDS-sized chunks: the unrolled part touches only the
    // register state (horizontal sums -> LDS); the solve runs after it as an
    // ordinary loop, so the state array stays in registers.
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
#pragma unroll
      for (int jj = 0; jj < OC; ++jj) {
        const int j = cb * OC + jj;
        if (box_wave && j < SOUT) {
          if (j > 0) {
#pragma unroll
            for (int k = 0; k < CPW; ++k) {
              // fresh conversions each step: keeping the converted values alive
              // for 2R+1 steps would double the register footprint of the strip
              float a = vs[k][j + 2 * R], b = vs[k][j - 1];
              asm volatile("" : "+v"(a), "+v"(b));
              hs[k] += static_cast<double>(a) - static_cast<double>(b);
            }
          }
#pragma unroll
          for (int k = 0; k < CPW; ++k) {
            const int ch = wv * CPW + k;
            if (ch < NCH) lds[(jj * NCH + ch) * 64 + lane] = static_cast<float>(hs[k]);
          }
        }
      }
      // the staged row must have landed before the barrier publishes it
      if (cb == 0) __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (cb == 0 && y + 1 < y1) {
        // every wave is past its vertical update: stage the next row step's
        // cost rows while the solves run
        if (y + 1 + R < H) stage_cost(y + 1 + R, 0);
        if (y - R >= 0) stage_cost(y - R, 1);
      }
      const int cnt = min(OC, SOUT - cb * OC);
      for (int q = wv; q < cnt; q += NWB) {
        const int x = x_out0 + cb * OC + q;
        if (x < W) solve_store(x, y, q, cb * OC + q);
      }
      // the staged cost rows must have landed before the row's last barrier
      if (cb == NCB - 1) __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
    }
  }
}

template <int R, int CPW, int NG, int MODE, typename TIN, int SIN>
__global__ __launch_bounds__(768) void coef_kernel(
    const TIN* __restrict__ cost, int cost_ld, const float* __restrict__ g32,
    const void* __restrict__ minv, float* __restrict__ ws,
    int H, int W, int label_count, int band_h, int strips, int bands) {
  constexpr int SOUT = SIN - 2 * R;
  constexpr int NCH = NG + 1;
  constexpr int OC = coef_column_chunk<NCH, SOUT, SIN, MODE>();
  __shared__ float lds[OC * NCH * 64];
  __shared__ float4 stage4[coef_stage_dwords<SOUT, NG, MODE>() / 4];
  __shared__ float cbuf[2 * SIN * 64];
  __shared__ float4 gbuf4[2 * NCH * 16];
  uint32_t* stage = reinterpret_cast<uint32_t*>(stage4);

  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // work item of this block; integer division runs on the vector ALU, so the
  // results are moved back to scalar registers explicitly
  // logical order: label chunk fastest, then strip, then band (one XCD gets a
  // contiguous range, so both label chunks of a strip share the L2 copy of M)
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
  // lanes past the last label read the last label's costs; their results are never used
  const int labc = min(lab, label_count - 1);
  const size_t P = static_cast<size_t>(H) * W;
  float* __restrict__ wsc = ws + static_cast<size_t>(chunk) * P * NCH * 64;
  if (xs >= 0 && xs + SIN <= W)
    coef_strip<R, CPW, NG, MODE, TIN, SIN, false>(cost, cost_ld, g32, minv, wsc, H, W, xs,
                                                   x_out0, y0, y1, labc, wv, lane, lds, stage,
                                                   cbuf, reinterpret_cast<float*>(gbuf4));
  else
    coef_strip<R, CPW, NG, MODE, TIN, SIN, true>(cost, cost_ld, g32, minv, wsc, H, W, xs,
                                                  x_out0, y0, y1, labc, wv, lane, lds, stage,
                                                   cbuf, reinterpret_cast<float*>(gbuf4));
}

template <int R, int NG, int MODE, typename TIN>
hipError_t coef_launch_t(const CoefLaunch& a, hipStream_t s) {
  constexpr int NCH = NG + 1;
  constexpr int CPW = NCH > 10 ? 2 : 1;
  constexpr int NWB = coef_block_waves((NCH + CPW - 1) / CPW);
  constexpr int SIN = coef_strip_width(NG, R);
  const StripGrid& g = a.grid;
  const unsigned blocks = static_cast<unsigned>(g.strips * g.bands * g.chunks);
  hipLaunchKernelGGL((coef_kernel<R, CPW, NG, MODE, TIN, SIN>), dim3(blocks), dim3(NWB * 64), 0,
                     s, static_cast<const TIN*>(a.cost), a.cost_ld, a.g32, a.minv, a.ws, a.H,
                     a.W, a.label_count, g.band_h, g.strips, g.bands);
  return hipGetLastError();
}

// Every solve mode and cost type of one (n, radius): the ridge form with
// float32 costs, the covariance form with float32, bfloat16 or float16 costs
// and a float32 or float64 solve.
template <int NG, int R>
hipError_t coef_launch_nr(const CoefLaunch& a, hipStream_t s) {
  if (a.mode == kSolveRidge) {
    if (a.cost_type != kCostF32) return hipErrorNotSupported;
    return coef_launch_t<R, NG, kSolveRidge, float>(a, s);
  }
  if (a.mode == kSolveCov64) {
    switch (a.cost_type) {
      case kCostF32: return coef_launch_t<R, NG, kSolveCov64, float>(a, s);
      case kCostBF16: return coef_launch_t<R, NG, kSolveCov64, bf16_t>(a, s);
      case kCostF16: return coef_launch_t<R, NG, kSolveCov64, f16_t>(a, s);
      default: return hipErrorNotSupported;
    }
  }
  if (a.mode != kSolveCov32) return hipErrorNotSupported;
  switch (a.cost_type) {
    case kCostF32: return coef_launch_t<R, NG, kSolveCov32, float>(a, s);
    case kCostBF16: return coef_launch_t<R, NG, kSolveCov32, bf16_t>(a, s);
    case kCostF16: return coef_launch_t<R, NG, kSolveCov32, f16_t>(a, s);
    default: return hipErrorNotSupported;
  }
}

}  // namespace hgf
