// Device-side helpers shared by the HGF kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace hgf {

// Largest guidance channel count n the kernels are built for, and the largest
// per-pixel system (ridge form adds the constant channel: D = n + 1).
constexpr int kMaxN = 19;
constexpr int kMaxD = 20;

// State columns per strip of the moment kernel: one wavefront-width of
// columns (the coefficient and output kernels choose theirs per channel count
// and radius).
constexpr int kStrip = 64;

// Floats of padding before and after the planar float32 guidance [n+1][P]:
// the strip kernels read a row of a strip's columns as one block (64 columns
// from the strip origin, which lies at most R columns before the image), so
// columns outside the image read padding or a neighbouring row; their weight
// is selected to 0.
constexpr int kGPad = 64;

// Read-only loads through the constant address space.  When the address is
// wave-uniform the compiler emits scalar (SMEM) loads into SGPRs, so
// per-pixel data shared by the 64 label lanes (the guidance values of the
// output kernel) costs no vector load and enters the VALU as a scalar
// operand.
template <typename T>
__device__ __forceinline__ T ldu(const T* p, size_t i) {
  typedef const __attribute__((address_space(4))) T* const_ptr;
  return ((const_ptr)(p))[i];
}

// Exponent table of the polynomial guidance: channel k is
// prod_c I_c^{e[k][c]} (Sec. 4.2).
struct MonoTable {
  int32_t n;
  int32_t m;
  int8_t e[kMaxD][4];
};

// Number of in-image pixels of the clipped (2R+1)^2 window centred at (x, y).
__device__ __forceinline__ int window_count(int x, int y, int W, int H, int R) {
  const int nx = min(x + R, W - 1) - max(x - R, 0) + 1;
  const int ny = min(y + R, H - 1) - max(y - R, 0) + 1;
  return nx * ny;
}

// Index of (i, j), i <= j, in the row-major packed upper triangle of a D x D matrix.
__host__ __device__ constexpr int packed_index(int i, int j, int D) {
  return i * D - (i * (i - 1)) / 2 + (j - i);
}

__device__ __forceinline__ float bf16_to_float(uint16_t b) {
  return __uint_as_float(static_cast<uint32_t>(b) << 16);
}

// Cost element types: float32, bfloat16 (kept as its raw bits) and float16.
struct bf16_t {
  uint16_t bits;
};
using f16_t = _Float16;

// A cost element as float32 (exact for every type).
__device__ __forceinline__ float cost_to_float(float v) { return v; }
__device__ __forceinline__ float cost_to_float(bf16_t v) { return bf16_to_float(v.bits); }
__device__ __forceinline__ float cost_to_float(f16_t v) { return static_cast<float>(v); }

// The float32 value of a 16-bit cost element given by its bits.
template <typename T>
__device__ __forceinline__ float cost_bits_to_float(uint16_t b) {
  if constexpr (std::is_same<T, f16_t>::value)
    return static_cast<float>(__builtin_bit_cast(f16_t, b));
  else
    return bf16_to_float(b);
}

template <typename T>
__device__ __forceinline__ float load_cost(const T* p, size_t i) {
  return cost_to_float(p[i]);
}

// Order-preserving map of a float to uint32 (NaN canonicalised to +qNaN, which
// sorts above +inf): a < b  <=>  ordered(a) < ordered(b).
__device__ __forceinline__ uint32_t ordered_bits(float f) {
  uint32_t u = __float_as_uint(f);
  if (f != f) u = 0x7fc00000u;
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float ordered_to_float(uint32_t u) {
  const uint32_t b = (u & 0x80000000u) ? (u & 0x7fffffffu) : ~u;
  return __uint_as_float(b);
}

// (cost, label) key whose unsigned minimum is the lowest cost, lowest label on ties.
__device__ __forceinline__ unsigned long long wta_key(float z, int label) {
  return (static_cast<unsigned long long>(ordered_bits(z)) << 32) |
         static_cast<unsigned long long>(static_cast<uint32_t>(label));
}

// Minimum over the 64 lanes of a wave, the same value in every lane: DPP
// butterflies within each row of 16 lanes, then the four row minima.
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
  constexpr int kQuadSwap1 = 1 | (0 << 2) | (3 << 4) | (2 << 6);
  constexpr int kQuadSwap2 = 2 | (3 << 2) | (0 << 4) | (1 << 6);
  constexpr int kRowRor4 = 0x124;
  constexpr int kRowRor8 = 0x128;
  auto dpp = [](uint32_t x, auto ctrl) {
    return static_cast<uint32_t>(
        __builtin_amdgcn_mov_dpp(static_cast<int>(x), decltype(ctrl)::value, 0xf, 0xf, false));
  };
  v = min(v, dpp(v, std::integral_constant<int, kQuadSwap1>()));
  v = min(v, dpp(v, std::integral_constant<int, kQuadSwap2>()));
  v = min(v, dpp(v, std::integral_constant<int, kRowRor4>()));
  v = min(v, dpp(v, std::integral_constant<int, kRowRor8>()));
  const uint32_t a = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v), 0));
  const uint32_t b = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v), 16));
  const uint32_t c = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v), 32));
  const uint32_t d = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v), 48));
  return min(min(a, b), min(c, d));
}

}  // namespace hgf
