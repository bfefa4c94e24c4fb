// Seed tetrahedron scores and the finite/symmetry validator.
//
// The four seed vertices are those with the largest total similarity across their row
// (Algorithm 1 and Algorithm 2, first comment). This library reads that as: the sum over
// u != v of W[v][u], accumulated in float64 strictly in index order of u, ranked by
// (score desc, id asc).
#include "common.h"
#include "internal.h"

namespace tmfg {

// One thread sums column v, which equals row v because W is bitwise symmetric; adjacent
// threads read adjacent addresses, so each row of W is read once, coalesced. Loads run a
// block ahead of the sequential float64 additions.
template <int U>
__device__ void seed_column(const float* __restrict__ W, int n, double* __restrict__ scores, int v) {
  const float* col = W + v;
  double acc = 0.0;
  float cur[U], nxt[U];
  int u = 0;
  const int full = n / U * U;
  if (full > 0) {
#pragma unroll
    for (int k = 0; k < U; ++k) cur[k] = col[(size_t)k * n];
  }
  for (; u < full; u += U) {
    const bool more = u + U < full;
    if (more) {
#pragma unroll
      for (int k = 0; k < U; ++k) nxt[k] = col[(size_t)(u + U + k) * n];
    }
#pragma unroll
    for (int k = 0; k < U; ++k) acc += (u + k == v) ? 0.0 : (double)cur[k];
    if (more) {
#pragma unroll
      for (int k = 0; k < U; ++k) cur[k] = nxt[k];
    }
  }
  for (; u < n; ++u) acc += (u == v) ? 0.0 : (double)col[(size_t)u * n];
  scores[v] = acc;
}

// Single builds with n a multiple of 4, tiled: a workgroup of 256 threads owns 64 rows, and
// all four waves stream those rows through LDS, kSeedCols columns at a time; the 16 threads
// of a row read its 256-byte span of a tile with one 16-byte load each, so a load
// instruction covers four rows' contiguous spans (8 lines, where one thread per row, each
// reading its own row, touches 64). Five register buffers hold four tiles in flight. Lane r of wave 0 then adds row
// v0 + r of the tile in index order: the sum is the sequential float64 chain of the
// definition, term by term. The chain is the pace, so a tile that holds no diagonal entry
// of the workgroup's rows (tile blockIdx.x holds them all) and no column past the row is
// added with no test per entry: the same additions in the same order.
constexpr int kSeedRows = 64, kSeedThreads = 256, kSeedCols = 64;
constexpr int kSeedQ = kSeedCols / 4;                          // quads of a row in a tile
constexpr int kSeedRowStep = kSeedThreads / kSeedQ;            // rows one pass of loads covers
static_assert(kSeedRows == kWave && kSeedRows == kSeedCols && kSeedRows / kSeedRowStep == 4,
              "the layout below");
#define SEED_ISSUE(t, X)                                                        \
  do {                                                                          \
    const int qq_ = (t) * kSeedQ + q;                                           \
    const int qc_ = qq_ < nq ? qq_ : nq - 1;                                    \
    X##0 = row0[qc_];                                                           \
    X##1 = row1[qc_];                                                           \
    X##2 = row2[qc_];                                                           \
    X##3 = row3[qc_];                                                           \
  } while (0)
#define SEED_STEP(t, XW, XL)                                                    \
  do {                                                                          \
    float4(*tb_)[kSeedQ + 1] = tile[(t) & 1];                                   \
    tb_[r0][q] = XW##0;                                                         \
    tb_[r0 + kSeedRowStep][q] = XW##1;                                          \
    tb_[r0 + 2 * kSeedRowStep][q] = XW##2;                                      \
    tb_[r0 + 3 * kSeedRowStep][q] = XW##3;                                      \
    SEED_ISSUE((t) + 4, XL);                                                    \
    __syncthreads();                                                            \
    if (tid < kSeedRows) {                                                      \
      if ((t) != (int)blockIdx.x && ((t) + 1) * kSeedCols <= n) {               \
        _Pragma("unroll") for (int k_ = 0; k_ < kSeedQ; ++k_) {                 \
          const float4 y_ = tb_[tid][k_];                                       \
          acc += (double)y_.x;                                                  \
          acc += (double)y_.y;                                                  \
          acc += (double)y_.z;                                                  \
          acc += (double)y_.w;                                                  \
        }                                                                       \
      } else {                                                                  \
        _Pragma("unroll") for (int k_ = 0; k_ < kSeedQ; ++k_) {                 \
          const float4 y_ = tb_[tid][k_];                                       \
          const int u_ = (t) * kSeedCols + 4 * k_;                              \
          const bool in_ = u_ < n;                                              \
          acc += (!in_ || u_ == v) ? 0.0 : (double)y_.x;                        \
          acc += (!in_ || u_ + 1 == v) ? 0.0 : (double)y_.y;                    \
          acc += (!in_ || u_ + 2 == v) ? 0.0 : (double)y_.z;                    \
          acc += (!in_ || u_ + 3 == v) ? 0.0 : (double)y_.w;                    \
        }                                                                       \
      }                                                                         \
    }                                                                           \
  } while (0)
__global__ __launch_bounds__(kSeedThreads) void seed_tiles_kernel(const float* __restrict__ W, int n,
                                                                  double* __restrict__ scores) {
  // padded rows: fewer bank conflicts; the buffer tile t goes to was last read two tiles
  // earlier, before the barrier of the previous tile
  __shared__ float4 tile[2][kSeedRows][kSeedQ + 1];
  const int tid = threadIdx.x;
  const int v0 = blockIdx.x * kSeedRows;
  const int nq = n / 4, nt = (n + kSeedCols - 1) / kSeedCols;
  const int q = tid % kSeedQ, r0 = tid / kSeedQ;
  // rows past n read row n - 1 and quads past the row its last quad (valid addresses; such
  // values are never added)
  auto row_of = [&](int r) {
    const int vr = v0 + r;
    return (const float4*)(W + (size_t)(vr < n ? vr : n - 1) * n);
  };
  const float4* row0 = row_of(r0);
  const float4* row1 = row_of(r0 + kSeedRowStep);
  const float4* row2 = row_of(r0 + 2 * kSeedRowStep);
  const float4* row3 = row_of(r0 + 3 * kSeedRowStep);
  const int v = v0 + tid;                                      // wave 0: the row this lane adds
  double acc = 0.0;
  float4 a0, a1, a2, a3, b0, b1, b2, b3, c0, c1, c2, c3, d0, d1, d2, d3, e0, e1, e2, e3;
  SEED_ISSUE(0, a);
  SEED_ISSUE(1, b);
  SEED_ISSUE(2, c);
  SEED_ISSUE(3, d);
  int t0 = 0;
  for (; t0 + 5 <= nt; t0 += 5) {
    SEED_STEP(t0, a, e);
    SEED_STEP(t0 + 1, b, a);
    SEED_STEP(t0 + 2, c, b);
    SEED_STEP(t0 + 3, d, c);
    SEED_STEP(t0 + 4, e, d);
  }
  // the last tiles (conditions uniform over the workgroup)
  if (t0 < nt) SEED_STEP(t0, a, e);
  if (t0 + 1 < nt) SEED_STEP(t0 + 1, b, a);
  if (t0 + 2 < nt) SEED_STEP(t0 + 2, c, b);
  if (t0 + 3 < nt) SEED_STEP(t0 + 3, d, c);
  if (tid < kSeedRows && v < n) scores[v] = acc;
}
#undef SEED_STEP
#undef SEED_ISSUE

// Other n: one thread per column (equal to the row: W is bitwise symmetric), adjacent
// threads on adjacent addresses.
__global__ __launch_bounds__(256) void seed_scores_kernel(const float* __restrict__ W, int n,
                                                          double* __restrict__ scores) {
  const int v = blockIdx.x * 256 + threadIdx.x;
  if (v < n) seed_column<32>(W, n, scores, v);
}

// Top-4 by (score desc, id asc), one 256-thread workgroup.
__global__ __launch_bounds__(256) void seed_top4_kernel(const double* __restrict__ scores, int n,
                                                        int32_t* __restrict__ seed4) {
  __shared__ uint64_t sk[4];
  __shared__ int sv[4];
  __shared__ int chosen[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int r = 0; r < 4; ++r) {
    uint64_t bk = 0;
    int bv = 0x7fffffff;
    for (int v = tid; v < n; v += 256) {
      bool skip = false;
      for (int q = 0; q < r; ++q) skip |= (chosen[q] == v);
      if (skip) continue;
      const uint64_t k = ord_f64(scores[v]);
      if (k > bk || (k == bk && v < bv)) {
        bk = k;
        bv = v;
      }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      const uint64_t ok = ((uint64_t)__shfl_xor((uint32_t)(bk >> 32), off, kWave) << 32) |
                          __shfl_xor((uint32_t)bk, off, kWave);
      const int ov = __shfl_xor(bv, off, kWave);
      if (ok > bk || (ok == bk && ov < bv)) {
        bk = ok;
        bv = ov;
      }
    }
    if (lane == 0) {
      sk[wave] = bk;
      sv[wave] = bv;
    }
    __syncthreads();
    if (tid == 0) {
      uint64_t k = sk[0];
      int v = sv[0];
      for (int w = 1; w < 4; ++w)
        if (sk[w] > k || (sk[w] == k && sv[w] < v)) {
          k = sk[w];
          v = sv[w];
        }
      chosen[r] = v;
      seed4[r] = v;
    }
    __syncthreads();
  }
}

// Flags non-finite entries and entries whose mirror has different bits. Each 32x32 tile
// (bi, bj) with bi <= bj is read directly and transposed through LDS.
__device__ void validate_tile(const float* __restrict__ W, int n, int bi, int bj, uint32_t* __restrict__ flags,
                              uint32_t (*t)[33]) {
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  uint32_t bad = 0;
  for (int r = ty; r < 32; r += 8) {
    const int gi = bj * 32 + r, gj = bi * 32 + tx;   // the mirror tile, row-major
    uint32_t bits = 0;
    if (gi < n && gj < n) {
      const float x = W[(size_t)gi * n + gj];
      bits = __float_as_uint(x);
      if (!isfinite(x)) bad |= kFlagNonFinite;
    }
    t[tx][r] = bits;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int gi = bi * 32 + r, gj = bj * 32 + tx;
    if (gi < n && gj < n) {
      const float x = W[(size_t)gi * n + gj];
      if (!isfinite(x)) bad |= kFlagNonFinite;
      if (__float_as_uint(x) != t[r][tx]) bad |= kFlagAsymmetric;
    }
  }
  if (bad) atomicOr(flags, bad);
}

__global__ __launch_bounds__(256) void validate_kernel(const float* __restrict__ W, int n,
                                                       uint32_t* __restrict__ flags) {
  __shared__ uint32_t t[32][33];
  int bi, bj;
  upper_tri_coords(blockIdx.x, (n + 31) / 32, bi, bj);
  validate_tile(W, n, bi, bj, flags, t);
}

// Batched forms.
__global__ __launch_bounds__(256) void batch_seed_kernel(const BatchJob* __restrict__ jobs,
                                                         const int* __restrict__ list,
                                                         const int* __restrict__ prefix, int nlist, int total) {
  const int unit = blockIdx.x * 256 + threadIdx.x;
  if (unit >= total) return;
  const int i = find_unit(prefix, nlist, unit);
  const BatchJob& J = jobs[list[i]];
  seed_column<32>(J.W, J.n, J.scores, unit - prefix[i]);
}

__global__ __launch_bounds__(256) void batch_validate_kernel(const BatchJob* __restrict__ jobs,
                                                             const int* __restrict__ list,
                                                             const int* __restrict__ prefix, int nlist,
                                                             int total) {
  __shared__ uint32_t t[32][33];
  const int unit = blockIdx.x;
  if (unit >= total) return;
  const int i = find_unit(prefix, nlist, unit);
  const BatchJob& J = jobs[list[i]];
  int bi, bj;
  upper_tri_coords(unit - prefix[i], (J.n + 31) / 32, bi, bj);
  validate_tile(J.W, J.n, bi, bj, J.flags, t);
}

hipError_t launch_seed_scores(const float* W, int n, double* scores, hipStream_t s) {
  if (n % 4 == 0)
    hipLaunchKernelGGL(seed_tiles_kernel, dim3((n + kSeedRows - 1) / kSeedRows), dim3(kSeedThreads), 0, s, W, n,
                       scores);
  else
    hipLaunchKernelGGL(seed_scores_kernel, dim3((n + 255) / 256), dim3(256), 0, s, W, n, scores);
  return hipGetLastError();
}

hipError_t launch_seed_top4(const double* scores, int n, int32_t* seed4, hipStream_t s) {
  hipLaunchKernelGGL(seed_top4_kernel, dim3(1), dim3(256), 0, s, scores, n, seed4);
  return hipGetLastError();
}

hipError_t launch_validate(const float* W, int n, uint32_t* flags, hipStream_t s) {
  hipLaunchKernelGGL(validate_kernel, dim3(validate_tiles(n)), dim3(256), 0, s, W, n, flags);
  return hipGetLastError();
}

hipError_t launch_batch_seed(const BatchJob* jobs, const int* list, const int* prefix, int nlist, int total,
                             hipStream_t s) {
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(batch_seed_kernel, dim3((total + 255) / 256), dim3(256), 0, s, jobs, list, prefix, nlist,
                     total);
  return hipGetLastError();
}

hipError_t launch_batch_validate(const BatchJob* jobs, const int* list, const int* prefix, int nlist, int total,
                                 hipStream_t s) {
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(batch_validate_kernel, dim3(total), dim3(256), 0, s, jobs, list, prefix, nlist, total);
  return hipGetLastError();
}

int validate_tiles(int n) {
  const int nb = (n + 31) / 32;
  return nb * (nb + 1) / 2;
}

}  // namespace tmfg
