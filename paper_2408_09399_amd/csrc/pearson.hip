// Pearson similarity of n series on gfx950: a standardisation pass, then W = Z Z^T as an
// FP32 MFMA GEMM (the one dense contraction of the path).
//
// The similarity matrix is the Pearson correlation of every pair of series (paper,
// Section 5, Datasets). With z_i = (x_i - mean_i) / ||x_i - mean_i||, W[i][j] = <z_i, z_j>.
#include "common.h"
#include "internal.h"

namespace tmfg {

// ---------------------------------------------------------------------------------------
// Standardisation of one series by one wave. Mean and centred norm are accumulated in
// float64; z is stored as float32 in a zero-padded (n_pad x L_pad) buffer so that the GEMM
// needs no bounds checks. A series with non-finite values, or with all values equal (no
// Pearson correlation exists), raises a flag.
// ---------------------------------------------------------------------------------------
__device__ void standardize_row(const float* __restrict__ X, int n, int L, float* __restrict__ Z, int L_pad,
                                uint32_t* __restrict__ flags, int row, int lane) {
  float* z = Z + (size_t)row * L_pad;
  if (row >= n) {
    for (int k = lane; k < L_pad; k += kWave) z[k] = 0.0f;
    return;
  }
  const float* x = X + (size_t)row * L;
  double s = 0.0;
  float mn = INFINITY, mx = -INFINITY;
  bool finite = true;
  for (int k = lane; k < L; k += kWave) {
    float v = x[k];
    finite &= (bool)isfinite(v);
    s += (double)v;
    mn = fminf(mn, v);
    mx = fmaxf(mx, v);
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    s += __shfl_xor(s, off, kWave);
    mn = fminf(mn, __shfl_xor(mn, off, kWave));
    mx = fmaxf(mx, __shfl_xor(mx, off, kWave));
  }
  const bool all_finite = __all(finite);
  if (!all_finite || !(mn < mx)) {
    if (lane == 0) atomicOr(flags, !all_finite ? kFlagNonFinite : kFlagDegenerate);
    for (int k = lane; k < L_pad; k += kWave) z[k] = 0.0f;
    return;
  }
  const double mean = s / (double)L;
  double q = 0.0;
  for (int k = lane; k < L; k += kWave) {
    double d = (double)x[k] - mean;
    q += d * d;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) q += __shfl_xor(q, off, kWave);
  const double inv = 1.0 / sqrt(q);
  for (int k = lane; k < L_pad; k += kWave) z[k] = k < L ? (float)(((double)x[k] - mean) * inv) : 0.0f;
}

__global__ __launch_bounds__(256) void standardize_kernel(const float* __restrict__ X, int n, int L,
                                                          float* __restrict__ Z, int n_pad, int L_pad,
                                                          uint32_t* __restrict__ flags) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n_pad) return;
  standardize_row(X, n, L, Z, L_pad, flags, row, threadIdx.x & 63);
}

// ---------------------------------------------------------------------------------------
// W = Z Z^T with v_mfma_f32_32x32x2_f32.
//
// Workgroup tile TB x TB: TB = 128 (4 waves) or TB = 64 (1 wave). Every wave computes a
// 64x64 block as 2x2 MFMA blocks of 32x32, with K staged through LDS 32 columns at a time.
// Only tiles with block-row <= block-column are computed; each is written to W[i][j] and
// mirrored to W[j][i], so W is bitwise symmetric. In a diagonal tile only entries with i < j
// are used (their mirrors fill j < i) and the diagonal is written as exactly 1.0f. Every
// entry is clamped to [-1, 1] and -0.0 is stored as +0.0.
//
// Summation order is a property of the wave's code alone: the K dimension is walked in
// steps of 4, each step issuing two MFMAs over the k pairs (k, k+2) and (k+1, k+3). The tile
// size only decides how many waves share a tile, so W's bits depend on neither the tile nor
// the launch shape.
//
// Operand layout for the 32x32x2 MFMA: lane l supplies A[l % 32][l / 32] and
// B[l / 32][l % 32]; the 16 accumulators of lane l hold D[8 (r / 4) + 4 (l / 32) + r % 4]
// [l % 32] for r = 0..15.
// ---------------------------------------------------------------------------------------
namespace {
constexpr int BK = 32, LDA = BK + 2;  // LDS row stride in floats (pad for banks)
typedef float f16x __attribute__((ext_vector_type(16)));
template <int TB>
struct GemmShape {
  static_assert(TB == 64 || TB == 128, "a tile is one wave's 64x64 block or 2x2 of them");
  static constexpr int kWavesPerDim = TB / 64;
  static constexpr int kThreads = kWavesPerDim * kWavesPerDim * kWave;
  static constexpr int kLdt = TB + 1;                                    // output staging stride
  static constexpr int kLoads = TB * (BK / 4) / kThreads;                // float4 per thread and operand
  static constexpr int kSmem = TB * kLdt > 2 * TB * LDA ? TB * kLdt : 2 * TB * LDA;   // floats
};
}  // namespace

__device__ __forceinline__ float fix_corr(float v) { return fminf(fmaxf(v, -1.0f), 1.0f) + 0.0f; }

template <int TB>
__device__ void gemm_tile(const float* __restrict__ Z, int n, int L_pad, float* __restrict__ W, int bi, int bj,
                          float* smem) {
  typedef GemmShape<TB> G;
  constexpr int NT = G::kThreads, LDT = G::kLdt;
  const int i0 = bi * TB, j0 = bj * TB;
  float* As = smem;
  float* Bs = smem + TB * LDA;

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wm = wave / G::kWavesPerDim, wn = wave % G::kWavesPerDim;
  const int li = lane & 31, lh = lane >> 5;

  f16x acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;

  const float* Za = Z + (size_t)i0 * L_pad;
  const float* Zb = Z + (size_t)j0 * L_pad;
  for (int k0 = 0; k0 < L_pad; k0 += BK) {
    float4 ra[G::kLoads], rb[G::kLoads];
#pragma unroll
    for (int r = 0; r < G::kLoads; ++r) {
      const int flat = r * NT + tid;
      const int row = flat >> 3, c4 = (flat & 7) * 4;
      ra[r] = *(const float4*)(Za + (size_t)row * L_pad + k0 + c4);
      rb[r] = *(const float4*)(Zb + (size_t)row * L_pad + k0 + c4);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < G::kLoads; ++r) {
      const int flat = r * NT + tid;
      const int row = flat >> 3, c4 = (flat & 7) * 4;
      float2* pa = (float2*)(As + row * LDA + c4);
      float2* pb = (float2*)(Bs + row * LDA + c4);
      pa[0] = make_float2(ra[r].x, ra[r].y);
      pa[1] = make_float2(ra[r].z, ra[r].w);
      pb[0] = make_float2(rb[r].x, rb[r].y);
      pb[1] = make_float2(rb[r].z, rb[r].w);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const float2 a0 = *(const float2*)(As + (wm * 64 + li) * LDA + kk + 2 * lh);
      const float2 a1 = *(const float2*)(As + (wm * 64 + 32 + li) * LDA + kk + 2 * lh);
      const float2 b0 = *(const float2*)(Bs + (wn * 64 + li) * LDA + kk + 2 * lh);
      const float2 b1 = *(const float2*)(Bs + (wn * 64 + 32 + li) * LDA + kk + 2 * lh);
      acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0.x, b0.x, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0.x, b1.x, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1.x, b0.x, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1.x, b1.x, acc[1][1], 0, 0, 0);
      acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0.y, b0.y, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0.y, b1.y, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1.y, b0.y, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1.y, b1.y, acc[1][1], 0, 0, 0);
    }
  }
  __syncthreads();
  // Stage the tile in LDS so both the direct and the mirrored stores coalesce.
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = wm * 64 + a * 32 + 8 * (r >> 2) + 4 * lh + (r & 3);
        const int col = wn * 64 + b * 32 + li;
        smem[row * LDT + col] = acc[a][b][r];
      }
  __syncthreads();
  const bool diag = (bi == bj);
  for (int flat = tid; flat < TB * TB; flat += NT) {
    const int r = flat / TB, c = flat % TB;
    const int gi = i0 + r, gj = j0 + c;
    if (gi < n && gj < n) {
      if (!diag || r < c) W[(size_t)gi * n + gj] = fix_corr(smem[r * LDT + c]);
      else if (r == c) W[(size_t)gi * n + gj] = 1.0f;
    }
    // mirrored store: row j0 + r, column i0 + c takes the entry computed at (i0 + c, j0 + r)
    const int mi = j0 + r, mj = i0 + c;
    if (mi < n && mj < n && (!diag || c < r)) W[(size_t)mi * n + mj] = fix_corr(smem[c * LDT + r]);
  }
}

__global__ __launch_bounds__(256, 2) void corr_gemm_kernel(const float* __restrict__ Z, int n, int L_pad,
                                                           int nb, int tiles, int tiles_per_xcd,
                                                           float* __restrict__ W) {
  // Blocks are handed to the 8 XCDs round-robin; give each XCD a contiguous run of tiles
  // (tiles in one block-row share their A operand, which then stays in that XCD's L2).
  const int xcd = blockIdx.x & 7;
  const int t = xcd * tiles_per_xcd + (blockIdx.x >> 3);
  if (t >= tiles) return;
  int bi, bj;
  upper_tri_coords(t, nb, bi, bj);
  __shared__ __attribute__((aligned(16))) float smem[GemmShape<128>::kSmem];
  gemm_tile<128>(Z, n, L_pad, W, bi, bj, smem);
}

// Batched forms: one launch over every instance's rows / tiles.
__global__ __launch_bounds__(256) void batch_standardize_kernel(const BatchJob* __restrict__ jobs,
                                                                const int* __restrict__ list,
                                                                const int* __restrict__ prefix, int nlist,
                                                                int total) {
  const int unit = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (unit >= total) return;
  const int i = find_unit(prefix, nlist, unit);
  const BatchJob& J = jobs[list[i]];
  standardize_row(J.X, J.n, J.L, J.Z, J.L_pad, J.flags, unit - prefix[i], threadIdx.x & 63);
}

template <int TB>
__global__ __launch_bounds__(GemmShape<TB>::kThreads, 2) void batch_gemm_kernel(const BatchJob* __restrict__ jobs,
                                                                            const int* __restrict__ list,
                                                                            const int* __restrict__ prefix, int nlist,
                                                                            int total, int per_xcd) {
  const int xcd = blockIdx.x & 7;
  const int t = xcd * per_xcd + (blockIdx.x >> 3);
  if (t >= total) return;
  const int i = find_unit(prefix, nlist, t);
  const BatchJob& J = jobs[list[i]];
  const int nb = (J.n + TB - 1) / TB;
  int bi, bj;
  upper_tri_coords(t - prefix[i], nb, bi, bj);
  __shared__ __attribute__((aligned(16))) float smem[GemmShape<TB>::kSmem];
  gemm_tile<TB>(J.Z, J.n, J.L_pad, J.Wdst, bi, bj, smem);
}

hipError_t launch_standardize(const float* X, int n, int L, float* Z, int n_pad, int L_pad, uint32_t* flags,
                              hipStream_t s) {
  dim3 grid((n_pad + 3) / 4);
  hipLaunchKernelGGL(standardize_kernel, grid, dim3(256), 0, s, X, n, L, Z, n_pad, L_pad, flags);
  return hipGetLastError();
}

hipError_t launch_corr_gemm(const float* Z, int n, int L_pad, float* W, hipStream_t s) {
  const int nb = (n + 127) / 128;
  const int tiles = nb * (nb + 1) / 2;
  const int per_xcd = (tiles + 7) / 8;
  hipLaunchKernelGGL(corr_gemm_kernel, dim3(8 * per_xcd), dim3(256), 0, s, Z, n, L_pad, nb, tiles, per_xcd, W);
  return hipGetLastError();
}

hipError_t launch_batch_standardize(const BatchJob* jobs, const int* list, const int* prefix, int nlist, int total,
                                    hipStream_t s) {
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(batch_standardize_kernel, dim3((total + 3) / 4), dim3(256), 0, s, jobs, list, prefix, nlist,
                     total);
  return hipGetLastError();
}

hipError_t launch_batch_gemm(const BatchJob* jobs, const int* list, const int* prefix, int nlist, int total,
                             int tile, hipStream_t s) {
  if (total <= 0) return hipSuccess;
  const int per_xcd = (total + 7) / 8;
  if (tile == 64)
    hipLaunchKernelGGL(batch_gemm_kernel<64>, dim3(8 * per_xcd), dim3(GemmShape<64>::kThreads), 0, s, jobs, list,
                       prefix, nlist, total, per_xcd);
  else if (tile == 128)
    hipLaunchKernelGGL(batch_gemm_kernel<128>, dim3(8 * per_xcd), dim3(GemmShape<128>::kThreads), 0, s, jobs, list,
                       prefix, nlist, total, per_xcd);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

int corr_tiles(int n, int tile) {
  const int nb = (n + tile - 1) / tile;
  return nb * (nb + 1) / 2;
}
int corr_row_pad() { return 128; }
int corr_k_pad() { return BK; }

}  // namespace tmfg
