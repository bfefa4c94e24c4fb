// Per-vertex order of the other vertices by similarity (paper, Algorithm 1: one parallel
// sort of [(S[v,u], u)] for every vertex v, done once before any insertion).
//
// Order: W[v][u] descending, then u ascending; v itself is left out, so each row yields
// n-1 ids (16-bit). -0.0 and +0.0 compare equal.
//
// One workgroup sorts one row entirely in LDS:
//  1. the row is read once (coalesced) into registers as 32-bit keys k = ~ord(W[v][u]),
//     for which "larger similarity" is "smaller key";
//  2. 256 evenly spaced samples of the row are ranked against each other (rank by
//     counting) and become splitters; every element finds its splitter interval by binary
//     search and a linear sub-bucket inside it. The bucket index is a non-decreasing
//     function of the key, so buckets come out in key order and are about equally full
//     whatever the value distribution (Pearson rows crowd near 1);
//  3. a histogram, a scan and a scatter (LDS atomics) place each element in its bucket;
//     order inside a bucket is arbitrary at this point;
//  4. inside a bucket of at most kRankMax elements each element counts the elements that
//     precede it by (key, id), which is its exact position: the composite key is unique,
//     so the outcome is deterministic even though the scatter is not;
//  5. larger buckets (many exactly equal similarities) are bitonic-sorted by one wave each;
//  6. the ids are written out with 16-byte stores, and, when asked for, the similarities in
//     the same order (W[v][u] as float32, -0.0 written as +0.0).
#include "common.h"
#include "internal.h"

namespace tmfg {

namespace {
constexpr int kSamples = 256;
constexpr int kRankMax = 32;
constexpr int kMaxBig = kMaxN / (kRankMax + 1) + 1;
}  // namespace

// Bitonic sort of keys/ids[0..sz) in LDS by (key asc, id asc), one wave, no workgroup
// barrier. All comparators move the smaller element to the lower index; positions past sz
// act as +infinity and never move, so the network needs no padding storage.
__device__ void wave_bitonic(uint32_t* k, uint16_t* id, int sz, int lane) {
  int P = 1;
  while (P < sz) P <<= 1;
  for (int blk = 2; blk <= P; blk <<= 1) {
    for (int j = blk >> 1; j > 0; j >>= 1) {
      for (int i = lane; i < sz; i += kWave) {
        const int l = (j == (blk >> 1)) ? (i ^ (blk - 1)) : (i ^ j);
        if (l > i && l < sz) {
          const uint32_t ki = k[i], kl = k[l];
          const uint16_t ii = id[i], il = id[l];
          if (kl < ki || (kl == ki && il < ii)) {
            k[i] = kl;
            k[l] = ki;
            id[i] = il;
            id[l] = ii;
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
    }
  }
}

template <int BLOCK, int EPT>
__device__ void sort_row(const float* __restrict__ W, int n, uint16_t* __restrict__ idx, float* __restrict__ vals,
                         int64_t ldi, int sub_log2, int v, uint8_t* smem) {
  constexpr int NWAVE = BLOCK / kWave;
  __shared__ uint32_t red_lo[NWAVE], red_hi[NWAVE];
  __shared__ int nbig;
  __shared__ int big_list[kMaxBig];

  const int m = n - 1;
  const int m_al = (m + 7) & ~7;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int S = m < kSamples ? m : kSamples;
  const int SUB = 1 << sub_log2;
  const int NB = (S + 1) * SUB;

  uint32_t* keys = (uint32_t*)smem;             // m_al
  uint16_t* ids = (uint16_t*)(keys + m_al);     // m_al
  uint32_t* cnt = (uint32_t*)(ids + m_al);      // NB
  uint32_t* spl = cnt + NB;                     // S

  const float* row = W + (size_t)v * n;

  // 1. the row into registers
  uint32_t dk[EPT];
  uint32_t lmin = 0xffffffffu, lmax = 0u;
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int j = e * BLOCK + tid;
    if (j < n && j != v) {
      dk[e] = ~ord_f32(row[j]);
      lmin = min(lmin, dk[e]);
      lmax = max(lmax, dk[e]);
    }
  }
  lmin = wave_min_u32(lmin);
  lmax = wave_max_u32(lmax);
  if (lane == 0) {
    red_lo[wave] = lmin;
    red_hi[wave] = lmax;
  }
  for (int i = tid; i < NB; i += BLOCK) cnt[i] = 0;
  if (tid == 0) nbig = 0;
  // 2. samples: element position floor(i*m/S) of the row without v
  if (tid < S) {
    const int pos = (int)(((int64_t)tid * m) / S);
    const int j = pos < v ? pos : pos + 1;
    keys[tid] = ~ord_f32(row[j]);
  }
  __syncthreads();
  uint32_t kmin = red_lo[0], kmax = red_hi[0];
  for (int w = 1; w < NWAVE; ++w) {
    kmin = min(kmin, red_lo[w]);
    kmax = max(kmax, red_hi[w]);
  }
  if (tid < S) {
    const uint32_t s = keys[tid];
    int r = 0;
    for (int q = 0; q < S; ++q) {
      const uint32_t kq = keys[q];
      r += (kq < s) || (kq == s && q < tid);
    }
    spl[r] = s;
  }
  __syncthreads();

  // 3a. bucket of every element, histogram
  uint32_t bk[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int j = e * BLOCK + tid;
    if (j < n && j != v) {
      const uint32_t k = dk[e];
      int lo = 0, len = S;                       // first splitter > k
      while (len > 0) {
        const int half = len >> 1;
        if (spl[lo + half] <= k) {
          lo += half + 1;
          len -= half + 1;
        } else {
          len = half;
        }
      }
      const uint64_t blo = lo > 0 ? spl[lo - 1] : kmin;
      const uint64_t bhi = lo < S ? (uint64_t)spl[lo] : (uint64_t)kmax + 1;
      const uint32_t sub = (uint32_t)((((uint64_t)k - blo) << sub_log2) / (bhi - blo));
      bk[e] = (uint32_t)lo * SUB + sub;
      atomicAdd(&cnt[bk[e]], 1u);
    }
  }
  __syncthreads();

  // 3b. exclusive scan of the histogram (contiguous chunk per thread, then across threads)
  {
    const int per = (NB + BLOCK - 1) / BLOCK;
    const int b0 = tid * per;
    uint32_t local = 0;
    for (int i = 0; i < per; ++i)
      if (b0 + i < NB) local += cnt[b0 + i];
    // inclusive scan of 'local' across the workgroup
    uint32_t x = local;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const uint32_t y = __shfl_up(x, off, kWave);
      if (lane >= off) x += y;
    }
    if (lane == 63) red_lo[wave] = x;
    __syncthreads();
    uint32_t base = 0;
    for (int w = 0; w < wave; ++w) base += red_lo[w];
    uint32_t run = base + x - local;
    for (int i = 0; i < per; ++i)
      if (b0 + i < NB) {
        const uint32_t c = cnt[b0 + i];
        cnt[b0 + i] = run;
        run += c;
      }
  }
  __syncthreads();

  // 3c. scatter; afterwards cnt[b] is the end of bucket b
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int j = e * BLOCK + tid;
    if (j < n && j != v) {
      const uint32_t p = atomicAdd(&cnt[bk[e]], 1u);
      keys[p] = dk[e];
      ids[p] = (uint16_t)j;
    }
  }
  __syncthreads();

  // 4. exact position inside small buckets
  int fin[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    fin[e] = -1;
    const int j = e * BLOCK + tid;
    if (j < n && j != v) {
      const uint32_t b = bk[e];
      const int s = b ? (int)cnt[b - 1] : 0;
      const int en = (int)cnt[b];
      const uint32_t k = dk[e];
      if (en - s <= kRankMax) {
        int r = 0;
        for (int q = s; q < en; ++q) {
          const uint32_t kq = keys[q];
          r += (kq < k) || (kq == k && (int)ids[q] < j);
        }
        fin[e] = s + r;
      } else if ((int)ids[s] == j) {
        big_list[atomicAdd(&nbig, 1)] = (int)b;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < EPT; ++e)
    if (fin[e] >= 0) {
      ids[fin[e]] = (uint16_t)(e * BLOCK + tid);
      keys[fin[e]] = dk[e];
    }
  for (int i = m + tid; i < m_al; i += BLOCK) {
    ids[i] = 0xffff;
    keys[i] = 0xff800000u;              // -inf
  }
  __syncthreads();

  // 5. large buckets
  for (int q = wave; q < nbig; q += NWAVE) {
    const int b = big_list[q];
    const int s = b ? (int)cnt[b - 1] : 0;
    wave_bitonic(keys + s, ids + s, (int)cnt[b] - s, lane);
  }
  __syncthreads();

  // 6. write out
  uint4* dst = (uint4*)(idx + (size_t)v * ldi);
  const uint4* src = (const uint4*)ids;
  for (int i = tid; i < m_al / 8; i += BLOCK) dst[i] = src[i];
  if (vals) {
    float4* vdst = (float4*)(vals + (size_t)v * ldi);
    for (int i = tid; i < m_al / 4; i += BLOCK) {
      const uint4 k = ((const uint4*)keys)[i];
      vdst[i] = make_float4(unord_f32(~k.x), unord_f32(~k.y), unord_f32(~k.z), unord_f32(~k.w));
    }
  }
}

__host__ __device__ inline int sort_sub_log2(int n) {
  const int m = n - 1;
  const int S = m < kSamples ? m : kSamples;
  int s = 0;
  while (s < 5 && (int64_t)(S + 1) * (2 << s) * 2 <= m) ++s;
  return s;
}

template <int BLOCK, int EPT>
__global__ __launch_bounds__(BLOCK) void sort_rows_kernel(const float* __restrict__ W, int n,
                                                          uint16_t* __restrict__ idx, float* __restrict__ vals,
                                                          int64_t ldi, int sub_log2) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  sort_row<BLOCK, EPT>(W, n, idx, vals, ldi, sub_log2, blockIdx.x, smem);
}

template <int BLOCK, int EPT>
__global__ __launch_bounds__(BLOCK) void batch_sort_kernel(const BatchJob* __restrict__ jobs,
                                                           const int* __restrict__ list,
                                                           const int* __restrict__ prefix, int nlist, int total) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  const int unit = blockIdx.x;
  if (unit >= total) return;
  const int i = find_unit(prefix, nlist, unit);
  const BatchJob& J = jobs[list[i]];
  sort_row<BLOCK, EPT>(J.W, J.n, J.idx, J.vals, J.ldi, sort_sub_log2(J.n), unit - prefix[i], smem);
}

namespace {
size_t sort_lds_bytes(int n, int sub_log2) {
  const int m = n - 1;
  const int m_al = (m + 7) & ~7;
  const int S = m < kSamples ? m : kSamples;
  const int NB = (S + 1) << sub_log2;
  return (size_t)m_al * 6 + (size_t)NB * 4 + (size_t)S * 4;
}
template <int BLOCK, int EPT>
hipError_t launch_sort_t(const float* W, int n, uint16_t* idx, float* vals, int64_t ldi, hipStream_t s) {
  const int sl = sort_sub_log2(n);
  const size_t lds = sort_lds_bytes(n, sl);
  hipLaunchKernelGGL((sort_rows_kernel<BLOCK, EPT>), dim3(n), dim3(BLOCK), lds, s, W, n, idx, vals, ldi, sl);
  return hipGetLastError();
}
}  // namespace

int64_t sort_row_stride(int n) { return round_up(n - 1 > 0 ? n - 1 : 1, 8); }

template <int BLOCK, int EPT>
hipError_t launch_batch_sort_t(const BatchJob* jobs, const int* list, const int* prefix, int nlist, int total,
                               int n_max, hipStream_t s) {
  const size_t lds = sort_lds_bytes(n_max, sort_sub_log2(n_max));
  hipLaunchKernelGGL((batch_sort_kernel<BLOCK, EPT>), dim3(total), dim3(BLOCK), lds, s, jobs, list, prefix, nlist,
                     total);
  return hipGetLastError();
}

// Let every sort kernel use all of the LDS the static arrays leave free (set once).
template <int BLOCK, int EPT>
hipError_t sort_attr_t() {
  const void* ks[2] = {(const void*)sort_rows_kernel<BLOCK, EPT>, (const void*)batch_sort_kernel<BLOCK, EPT>};
  for (const void* k : ks) {
    hipFuncAttributes a;
    hipError_t e = hipFuncGetAttributes(&a, k);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(kLdsBytes - a.sharedSizeBytes));
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t sort_init_attributes() {
  hipError_t e;
  if ((e = sort_attr_t<256, 1>()) != hipSuccess) return e;
  if ((e = sort_attr_t<256, 4>()) != hipSuccess) return e;
  if ((e = sort_attr_t<512, 4>()) != hipSuccess) return e;
  if ((e = sort_attr_t<1024, 4>()) != hipSuccess) return e;
  if ((e = sort_attr_t<1024, 8>()) != hipSuccess) return e;
  if ((e = sort_attr_t<1024, 12>()) != hipSuccess) return e;
  if ((e = sort_attr_t<1024, 16>()) != hipSuccess) return e;
  return sort_attr_t<1024, 20>();
}

int sort_class(int n) {
  if (n <= 256) return 0;
  if (n <= 1024) return 1;
  if (n <= 2048) return 2;
  if (n <= 4096) return 3;
  if (n <= 8192) return 4;
  if (n <= 12288) return 5;
  if (n <= 16384) return 6;
  return 7;
}

hipError_t launch_batch_sort(const BatchJob* jobs, const int* list, const int* prefix, int nlist, int total,
                             int n_max, hipStream_t s) {
  if (total <= 0) return hipSuccess;
  switch (sort_class(n_max)) {
    case 0: return launch_batch_sort_t<256, 1>(jobs, list, prefix, nlist, total, n_max, s);
    case 1: return launch_batch_sort_t<256, 4>(jobs, list, prefix, nlist, total, n_max, s);
    case 2: return launch_batch_sort_t<512, 4>(jobs, list, prefix, nlist, total, n_max, s);
    case 3: return launch_batch_sort_t<1024, 4>(jobs, list, prefix, nlist, total, n_max, s);
    case 4: return launch_batch_sort_t<1024, 8>(jobs, list, prefix, nlist, total, n_max, s);
    case 5: return launch_batch_sort_t<1024, 12>(jobs, list, prefix, nlist, total, n_max, s);
    case 6: return launch_batch_sort_t<1024, 16>(jobs, list, prefix, nlist, total, n_max, s);
    default: return launch_batch_sort_t<1024, 20>(jobs, list, prefix, nlist, total, n_max, s);
  }
}

hipError_t launch_sort_rows(const float* W, int n, uint16_t* idx, float* vals, int64_t ldi, hipStream_t s) {
  if (n <= 256) return launch_sort_t<256, 1>(W, n, idx, vals, ldi, s);
  if (n <= 1024) return launch_sort_t<256, 4>(W, n, idx, vals, ldi, s);
  if (n <= 2048) return launch_sort_t<512, 4>(W, n, idx, vals, ldi, s);
  if (n <= 4096) return launch_sort_t<1024, 4>(W, n, idx, vals, ldi, s);
  if (n <= 8192) return launch_sort_t<1024, 8>(W, n, idx, vals, ldi, s);
  if (n <= 12288) return launch_sort_t<1024, 12>(W, n, idx, vals, ldi, s);
  if (n <= 16384) return launch_sort_t<1024, 16>(W, n, idx, vals, ldi, s);
  return launch_sort_t<1024, 20>(W, n, idx, vals, ldi, s);
}

}  // namespace tmfg
