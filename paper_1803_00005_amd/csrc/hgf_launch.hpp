// Internal launch interface between the C ABI layer and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hgf_device.hpp"

namespace hgf {

// Per-launch geometry of a strip kernel: strips of (sin - 2R) output columns,
// bands of band_h output rows, label chunks of 64 lanes.
struct StripGrid {
  int strips;
  int bands;
  int band_h;
  int chunks;
};

// The band partition depends on the image, the strip width, the target block
// count and the label chunk count of the whole volume (chunks_total), never
// on how many of those chunks one launch takes (chunks): the float32 running
// sums restart at band boundaries, so this keeps the results independent of
// label chunking and launch groups.
StripGrid strip_grid(int H, int W, int R, int chunks, int target_blocks);
StripGrid strip_grid_w(int H, int W, int R, int sin, int chunks, int chunks_total,
                       int target_blocks);

// State columns per strip of the coefficient kernel: up to n = 9 one channel
// per wave and 64 columns; above, two channels per wave and a narrower strip
// so that ten waves fit the register file.  With at most three guidance
// channels and a radius of at most 4, 32 output columns (2r + 32 state
// columns): the smaller register and LDS footprint lets two blocks share a
// CU, which these short solves need more than the wider strip's smaller
// halo share (measured faster at r = 4, slower at r = 9).
constexpr int coef_strip_width(int n, int r) {
  return n + 1 > 10 ? 38 : (n + 1 == 10 ? 62 : (n + 1 <= 4 && r <= 4 ? 2 * r + 32 : 64));
}
// Output kernel: channels per wave (ten waves at most) and state columns per
// strip for n guidance channels (two channels per wave leave room for 48;
// with at most three guidance channels and a radius of at most 4, 2r + 32
// state columns as in the coefficient kernel, whose smaller register
// footprint keeps more waves resident).
constexpr int out_channels_per_wave(int n) { return n + 1 > 10 ? 2 : 1; }
constexpr int out_strip_width(int n, int r) {
  return out_channels_per_wave(n) > 1 ? 48 : (n + 1 <= 4 && r <= 4 ? 2 * r + 32 : 64);
}

// Radii with compiled strip kernels.
bool radius_supported(int R);
// (n, R) has compiled kernels (every solve mode and cost type).
bool config_supported(int n, int R);

// a1 + shift: guidance channel shifts (covariance form: each channel's mean
// over a fixed grid of at most 16 x 16 pixels, an exact reformulation since
// the window covariance does not see a constant offset; ridge form: 0).
hipError_t launch_guide_mean(const float* I, int H, int W, const MonoTable& t, double* shift,
                             bool centre, hipStream_t s);
// Rows (and columns) of the shift sample grid.
constexpr int kShiftRows = 16;
// a1: synthesized (shifted) guidance: float64 [P][n] and planar float32
// [n+1][P] with the constant channel G_0 = 1 first (g32 points at channel 0;
// the allocation has kGPad floats before and after).
hipError_t launch_guide_synth(const float* I, int H, int W, const MonoTable& t,
                              const double* shift, float* g32, double* g64,
                              hipStream_t s);
// a2: window sums of G_i and G_i G_j (i <= j), float64 [P][K], K = n + n(n+1)/2.
// For few channels the same kernel also computes a3 (the arguments of
// launch_invert) and sets *fused; S is then not written and launch_invert is
// not needed.
hipError_t launch_moments(const double* g64, int n, int H, int W, int R,
                          int target_blocks, double* S, double eps, int mode, double* mu,
                          void* minv, int* fused, hipStream_t s);
// a3: per-pixel window mean mu [P][n] (float64, covariance form) and the
// per-pixel inverse by the bordering recursion of Prop. 1, computed in
// float64 and stored as the solve mode says (SolveMode below).
hipError_t launch_invert(const double* S, int n, int H, int W, int R, double eps,
                         int mode, double* mu, void* minv, hipStream_t s);

// How the per-pixel inverse is stored and applied (the solve mode):
//   kSolveCov32  covariance form, float32 solve record per pixel: the window
//                mean mu_1..mu_n, then the packed upper triangle of M_p
//                (n(n+1)/2 entries, row by row), zero-padded to a multiple of
//                four floats (16-byte reads);
//   kSolveCov64  covariance form, the same record in float64, padded to an
//                even number of doubles;
//   kSolveRidge  ridge form, the packed upper triangle of the (n+1) x (n+1)
//                inverse in float64.
// M_p is computed in float64 in every mode.
enum SolveMode { kSolveCov32 = 0, kSolveCov64 = 1, kSolveRidge = 2 };

__host__ __device__ constexpr int cov_record_floats(int n) {
  return (n + n * (n + 1) / 2 + 3) / 4 * 4;
}
__host__ __device__ constexpr int cov_record_doubles(int n) {
  return (n + n * (n + 1) / 2 + 1) / 2 * 2;
}

// Elements per pixel of the stored inverse, and bytes per element.
__host__ __device__ constexpr int minv_stride(int mode, int n) {
  return mode == kSolveCov32 ? cov_record_floats(n)
                             : (mode == kSolveCov64 ? cov_record_doubles(n) : (n + 1) * (n + 2) / 2);
}
__host__ __device__ constexpr int minv_elem_bytes(int mode) { return mode == kSolveCov32 ? 4 : 8; }

// Cost element codes (hgf_dtype values of the cost volume).
enum CostType { kCostF32 = 0, kCostBF16 = 1, kCostF16 = 2 };

// Compiled set of the strip kernels.
constexpr int kMinRadius = 0;
constexpr int kMaxRadius = 9;

// Logical block index of hardware block `bid` of `nb`: consecutive hardware
// blocks are dispatched round-robin over the 8 XCDs, so this hands each XCD a
// contiguous range of logical work items (neighbouring strips and label
// chunks of one strip then share that XCD's L2).
__device__ __forceinline__ int xcd_remap(int bid, int nb) {
  const int full = nb & ~7;
  if (bid >= full) return bid;
  const int per = full >> 3;
  return (bid & 7) * per + (bid >> 3);
}

struct CoefLaunch {
  const void* cost;     // [H][W][cost_ld]
  int cost_type;        // CostType
  int cost_ld;
  const float* g32;     // planar [n+1][P], channel 0 = 1, padded
  const void* minv;     // [P][minv_stride(mode, n)] solve records
  float* ws;            // [chunks][P][n+1][64]
  int n, H, W, R, mode;
  int label_count;      // labels in this launch (chunks = ceil(label_count / 64))
  StripGrid grid;
};
// a4 + a5: per-label product box sums and coefficients a_l, b_l.
hipError_t launch_coef(const CoefLaunch& a, hipStream_t s);

struct OutLaunch {
  const float* ws;      // [chunks][P][n+1][64]
  const float* g32;     // planar [n+1][P], channel 0 = 1, padded
  float* out;           // [H][W][out_ld] or null
  int out_ld;
  unsigned long long* keys;  // [P] or null
  int32_t* labels;      // [P] or null: final labels, when every label is in this one chunk
  int label_base;       // absolute label of lane 0 of chunk 0
  int n, H, W, R;
  int label_count;
  StripGrid grid;
};
// a6 + a7: coefficient box filter, output and winner-takes-all keys.
hipError_t launch_out(const OutLaunch& a, hipStream_t s);

// a4 - a7 for a single label slice (L = 1) with lanes as pixels: separable
// box sums over planar images in the workspace, which needs room for
// 2 (n + 1) float32 images of P pixels.
struct SingleLaunch {
  const void* cost;     // [H][W][cost_ld], the label at offset 0
  int cost_type;        // CostType
  int cost_ld;
  const float* g32;     // planar [n+1][P], channel 0 = 1, padded
  const void* minv;     // solve records of the solve mode
  float* ws;            // >= 2 (n+1) P floats
  float* out;           // [H][W][out_ld] or null
  int out_ld;
  unsigned long long* keys;  // [P] or null
  int32_t* labels;      // [P] or null: final labels (the slice is the only label)
  int label;            // absolute label of the slice
  int n, H, W, R, mode;
};
hipError_t launch_single(const SingleLaunch& a, hipStream_t s);

// Fill `count` keys with ~0 (no hipMemsetAsync: safe under graph capture).
hipError_t launch_key_fill(unsigned long long* keys, size_t count, hipStream_t s);
// labels / best cost from keys; merge != 0 keeps the incoming (best, label)
// unless the key is strictly better.
hipError_t launch_key_finalize(const unsigned long long* keys, size_t count,
                               float* best, int32_t* labels, int merge,
                               hipStream_t s);

// Clipped box sum of C planar float32 images (radius up to 95), in one kernel.
constexpr int kBoxMaxRadius = 95;
hipError_t launch_box_sum(const float* in, float* out, int C, int H, int W, int R,
                          hipStream_t s);
hipError_t launch_spd_inverse(const double* a, double* minv, int D, int count,
                              hipStream_t s);

}  // namespace hgf
