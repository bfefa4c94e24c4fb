// Device-side helpers shared by the TMFG kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tmfg {

constexpr int kWave = 64;

// Limits of the library. Vertex and face ids are packed as 16 bits, and the 2n - 4 face ids
// of n = 32768 vertices are the most that fit. A row of up to kMaxLdsSortN entries is sorted
// inside one workgroup's LDS (6 bytes per entry plus the digit counters); a longer one as two
// halves that are then merged. corr-tmfg keeps a 16-bit vertex per face in LDS, and batches
// sort every row in LDS, so both stop at n = 20480.
constexpr int kMaxN = 32768;
constexpr int kMaxLdsSortN = 20480;
constexpr int kMaxCorrN = 20480;
constexpr int kMaxBatchN = 20480;
constexpr int kLdsBytes = 160 * 1024;   // LDS of one gfx950 workgroup
constexpr int kMinN = 4;

// Host copies of one build's outputs (pinned, coherent host memory), which the loop fills
// and publishes when the build ends, for a reader outside the launch (servers). order null:
// none.
struct HostOut {
  int32_t* order;
  int32_t* edges;
  int32_t* steps;
  float* step_gain;
  int32_t* faces;
  int32_t* status;         // written last, with a system-scope release
};

// Error flags raised on the device; the loop kernel turns them into a tmfg_status.
enum : uint32_t {
  kFlagNonFinite = 1u << 0,
  kFlagAsymmetric = 1u << 1,
  kFlagDegenerate = 1u << 2,
  kFlagInternal = 1u << 3,
};

// Order-preserving map float -> uint32 (larger float -> larger integer). -0.0 and +0.0
// are made equal first (x + 0.0f is +0.0 for both under round-to-nearest).
__device__ __forceinline__ uint32_t ord_f32(float x) {
  uint32_t b = __float_as_uint(x + 0.0f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float unord_f32(uint32_t k) {
  uint32_t b = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
  return __uint_as_float(b);
}
__device__ __forceinline__ uint64_t ord_f64(double x) {
  uint64_t b = (uint64_t)__double_as_longlong(x + 0.0);
  return (b & 0x8000000000000000ull) ? ~b : (b | 0x8000000000000000ull);
}

// Wave-wide reductions (64 lanes) through cross-lane reads.
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    uint32_t lo = __shfl_xor((uint32_t)v, off, kWave);
    uint32_t hi = __shfl_xor((uint32_t)(v >> 32), off, kWave);
    uint64_t o = ((uint64_t)hi << 32) | lo;
    v = o > v ? o : v;
  }
  return v;
}
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    uint32_t o = __shfl_xor(v, off, kWave);
    v = o > v ? o : v;
  }
  return v;
}
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    uint32_t o = __shfl_xor(v, off, kWave);
    v = o < v ? o : v;
  }
  return v;
}
__device__ __forceinline__ int wave_sum_i32(int v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Tile t of the row-major enumeration of the upper triangle (bi <= bj) of an nb x nb grid.
// Block-row i starts at S(i) = i*nb - i*(i-1)/2.
__device__ __forceinline__ void upper_tri_coords(int t, int nb, int& bi, int& bj) {
  const double b = 2.0 * nb + 1.0;
  int i = (int)((b - sqrt(b * b - 8.0 * (double)t)) * 0.5);
  if (i < 0) i = 0;
  while (i > 0 && (int64_t)i * nb - (int64_t)i * (i - 1) / 2 > t) --i;
  while (i + 1 < nb && (int64_t)(i + 1) * nb - (int64_t)(i + 1) * i / 2 <= t) ++i;
  bi = i;
  bj = i + (int)(t - ((int64_t)i * nb - (int64_t)i * (i - 1) / 2));
}

__host__ __device__ __forceinline__ int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

}  // namespace tmfg
