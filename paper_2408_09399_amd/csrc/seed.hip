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

// Single builds with n a multiple of 4: one thread per row v, adding W[v][u] over u in index
// order (the definition itself, with no use of symmetry), one wave per 64 rows. Each lane
// reads its row front to back with 16-byte loads, kSeedDepth blocks of kSeedQuads loads in
// flight; a load serves one lane, so a wave's load touches 64 lines that the lanes' next
// loads reuse, and every row is read once, sequentially.
constexpr int kSeedBlock = 64, kSeedDepth = 4, kSeedQuads = 8;
static_assert(kSeedDepth * kSeedQuads <= 63, "the loads in flight fit the wave's load counter");
__global__ __launch_bounds__(kSeedBlock) void seed_rows_kernel(const float* __restrict__ W, int n,
                                                               double* __restrict__ scores) {
  const int v = blockIdx.x * kSeedBlock + threadIdx.x;
  if (v >= n) return;
  const float4* row = (const float4*)(W + (size_t)v * n);
  const int nq = n / 4;
  float4 buf[kSeedDepth][kSeedQuads];
  // blocks past the row read its last quad (a valid address; the values are never added);
  // loads are issued whatever the block, so every step has the same count in flight
  auto issue = [&](int b, float4 (&x)[kSeedQuads]) {
#pragma unroll
    for (int k = 0; k < kSeedQuads; ++k) {
      const int q = b * kSeedQuads + k;
      x[k] = row[q < nq ? q : nq - 1];
    }
  };
  double acc = 0.0;
  auto add = [&](int b, const float4 (&x)[kSeedQuads]) {
#pragma unroll
    for (int k = 0; k < kSeedQuads; ++k) {
      const int u = 4 * (b * kSeedQuads + k);
      const bool in = u < n;
      acc += (!in || u == v) ? 0.0 : (double)x[k].x;
      acc += (!in || u + 1 == v) ? 0.0 : (double)x[k].y;
      acc += (!in || u + 2 == v) ? 0.0 : (double)x[k].z;
      acc += (!in || u + 3 == v) ? 0.0 : (double)x[k].w;
    }
  };
  const int nb = (nq + kSeedQuads - 1) / kSeedQuads;
#pragma unroll
  for (int d = 0; d < kSeedDepth; ++d) issue(d, buf[d]);
  int b0 = 0;
  for (; b0 + kSeedDepth <= nb; b0 += kSeedDepth) {
#pragma unroll
    for (int d = 0; d < kSeedDepth; ++d) {
      add(b0 + d, buf[d]);
      issue(b0 + d + kSeedDepth, buf[d]);
    }
  }
#pragma unroll
  for (int d = 0; d < kSeedDepth; ++d)
    if (b0 + d < nb) add(b0 + d, buf[d]);
  scores[v] = acc;
}

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
    hipLaunchKernelGGL(seed_rows_kernel, dim3((n + kSeedBlock - 1) / kSeedBlock), dim3(kSeedBlock), 0, s, W, n,
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
