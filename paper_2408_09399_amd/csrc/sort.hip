// Per-vertex order of the other vertices by similarity (paper, Algorithm 1: one parallel
// sort of [(S[v,u], u)] for every vertex v, done once before any insertion).
//
// Order: W[v][u] descending, then u ascending; v itself is left out, so each row yields
// n-1 ids (16-bit). -0.0 and +0.0 compare equal.
//
// One workgroup sorts one row at a time, entirely in LDS, by a stable least-significant-
// digit radix sort of 32-bit keys k = ~ord(W[v][u]) ("larger similarity" is "smaller key"),
// four passes of 8 bits. The row is loaded in ascending u, and every pass is stable, so
// equal keys come out in ascending u: the (value desc, id asc) order exactly, whatever the
// distribution of values, with no data-dependent work.
//
// Element slots: wave w holds positions [w*EPT*64, (w+1)*EPT*64), position w*EPT*64 +
// e*64 + lane in register e of that lane. One pass:
//  1. for each register e in order, lanes with the same digit are found with eight ballots;
//     they add their count to the wave's digit counter in LDS (all of them write the same
//     new value), and each gets its offset (counter before the add + its rank among them);
//  2. an exclusive scan over the counters in (digit, wave) order gives every (digit,
//     wave) its base;
//  3. every element is written to LDS at base + offset, then read back in position order.
// Slots past the row hold the key of -inf and id 0xffff; they sort last and fill the
// row's padding to a multiple of 8. Workgroups are persistent: each one loads the next row
// of its share into registers while it sorts the current one. Barriers wait on LDS only,
// so that prefetch stays in flight across them.
#include "common.h"
#include "internal.h"

namespace tmfg {

namespace {
constexpr int kPasses = 4;
constexpr int kDigits = 256;
constexpr int kHistStride = kDigits + 1;        // per-wave counters, padded against bank conflicts
constexpr uint32_t kPadKey = 0xff800000u;       // ~ord(-inf): above every finite key
// The two-run sort of rows longer than kMaxLdsSortN entries: kStageRows rows staged at a time,
// each half of a row sorted by one workgroup of kHalfBlock threads, kHalfEpt slots each.
constexpr int kStageRows = 1024;
constexpr int kHalfBlock = 1024, kHalfEpt = 16;
static_assert(kHalfBlock * kHalfEpt >= (kMaxN + 1) / 2, "a run of half a row fits one workgroup");

__device__ __forceinline__ void lds_barrier() {
  // LDS traffic only: a workgroup barrier that does not wait for global loads in flight
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

template <int BLOCK, int EPT>
struct RowSort {
  static constexpr int NW = BLOCK / kWave;
  static constexpr int CAP = BLOCK * EPT;        // slots per row
  static constexpr int WS = EPT * kWave;         // slots per wave
  static constexpr size_t lds_bytes() {
    return (size_t)CAP * 4 + (size_t)CAP * 2 + (size_t)NW * kHistStride * 4 + 64 * 4;
  }
};

// A run of one row to sort: the columns j in [c0, c0 + len + skip) other than v (skip is 1
// when v lies in that range), in ascending j. A whole row is c0 = 0, len = n - 1.
struct Run {
  int v, c0, len;
};
__device__ __forceinline__ int run_column(const Run& r, int p) {
  const int j = r.c0 + p;
  return (r.v >= r.c0 && j >= r.v) ? j + 1 : j;
}

// Global loads of one run into registers (raw similarities, position order).
template <int BLOCK, int EPT>
__device__ __forceinline__ void load_row(const float* __restrict__ W, int n, const Run& r, float (&raw)[EPT]) {
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const float* row = W + (size_t)r.v * n;
  // slots past the run read the row's last element (a valid address; the value is unused),
  // so that every load is unconditional
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int p = wave * RowSort<BLOCK, EPT>::WS + e * kWave + lane;
    const int j = run_column(r, p);
    raw[e] = row[j < n - 1 ? j : n - 1];
  }
}

// Keys and ids of one run from its similarities (position order).
template <int BLOCK, int EPT>
__device__ __forceinline__ void row_keys(const float (&raw)[EPT], const Run& r, uint32_t (&key)[EPT],
                                         uint32_t (&idp)[EPT]) {
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int p = wave * RowSort<BLOCK, EPT>::WS + e * kWave + lane;
    const int j = run_column(r, p);
    // branch-free select: slots past the run get the padding key and id
    const uint32_t in = 0u - (uint32_t)(p < r.len);
    key[e] = (~ord_f32(raw[e]) & in) | (kPadKey & ~in);
    idp[e] = ((uint32_t)j & in) | (0xffffu & ~in);
  }
}

// Sorts one run given as keys and ids (idp: id in the low 16 bits) and writes its ids (and
// values) to dst_idx / dst_vals, padded to a multiple of 8 entries (ids 0xffff, values -inf).
template <int BLOCK, int EPT>
__device__ __forceinline__ void sort_row_keys(uint32_t (&key)[EPT], uint32_t (&idp)[EPT], int len,
                                              uint16_t* __restrict__ dst_idx, float* __restrict__ dst_vals,
                                              uint8_t* smem) {
  using RS = RowSort<BLOCK, EPT>;
  constexpr int NW = RS::NW, CAP = RS::CAP, WS = RS::WS;
  const int m_al = (len + 7) & ~7;
  const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
  uint32_t* bkey = (uint32_t*)smem;                         // CAP
  uint16_t* bid = (uint16_t*)(bkey + CAP);                  // CAP
  uint32_t* hist = (uint32_t*)(bid + CAP);                  // NW x kHistStride
  uint32_t* wsum = hist + NW * kHistStride;                 // 64
  uint32_t* myh = hist + wave * kHistStride;
  const uint64_t below = (1ull << lane) - 1ull;
  // idp: low 16 bits the id, high 16 bits the element's offset in the current pass

  for (int pass = 0; pass < kPasses; ++pass) {
    const int shift = 8 * pass;
    for (int i = tid; i < NW * kHistStride; i += BLOCK) hist[i] = 0;
    lds_barrier();
    // 1. per-wave digit counts and each element's offset inside (digit, wave)
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const uint32_t d = (key[e] >> shift) & 0xffu;
      // lanes whose digit equals mine: for every bit, keep the lanes that agree with my bit
      // (ballot XOR my bit spread over 32 bits has a 1 exactly where a lane disagrees)
      uint32_t plo = ~0u, phi = ~0u;
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const uint32_t sb = (uint32_t)__builtin_amdgcn_sbfe((int32_t)d, b, 1);   // 0 or ~0
        const uint64_t bb = __ballot(sb != 0u);
        plo &= ~((uint32_t)bb ^ sb);
        phi &= ~((uint32_t)(bb >> 32) ^ sb);
      }
      const uint64_t peers = ((uint64_t)phi << 32) | plo;
      const uint32_t rank = (uint32_t)__popcll(peers & below);
      const uint32_t old = myh[d];
      myh[d] = old + (uint32_t)__popcll(peers);      // every peer writes the same value
      idp[e] = ((old + rank) << 16) | (idp[e] & 0xffffu);
      // materialise the offset now, so that the loaded counter and its address die here
      asm volatile("" : "+v"(idp[e]));
    }
    lds_barrier();
    // 2. exclusive scan in (digit, wave) order: thread t takes 4 consecutive counters
    {
      uint32_t c[4], s = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int g = 4 * tid + i;                 // g = d * NW + w
        c[i] = hist[(g % NW) * kHistStride + g / NW];
        s += c[i];
      }
      uint32_t x = s;
#pragma unroll
      for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t y = __shfl_up(x, off, kWave);
        if (lane >= off) x += y;
      }
      if (lane == kWave - 1) wsum[wave] = x;
      lds_barrier();
      uint32_t base = 0;
      for (int w = 0; w < wave; ++w) base += wsum[w];
      uint32_t run = base + x - s;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int g = 4 * tid + i;
        hist[(g % NW) * kHistStride + g / NW] = run;
        run += c[i];
      }
    }
    lds_barrier();
    // 3. scatter, then read back in position order (the digit address is recomputed
    //    rather than kept alive from step 1)
#pragma unroll
    for (int e = 0; e < EPT; ++e) asm volatile("" : "+v"(key[e]));
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const uint32_t pos = myh[(key[e] >> shift) & 0xffu] + (idp[e] >> 16);
      bkey[pos] = key[e];
      bid[pos] = (uint16_t)idp[e];
    }
    lds_barrier();
    if (pass + 1 < kPasses) {
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const int p = wave * WS + e * kWave + lane;
        key[e] = bkey[p];
        idp[e] = bid[p];
      }
      lds_barrier();      // every read of this pass's layout and counters is done
    }
  }

  // 4. write out: ids with 16-byte stores, values (-0.0 already +0.0) beside them
  uint4* dst = (uint4*)dst_idx;
  const uint4* src = (const uint4*)bid;
  for (int i = tid; i < m_al / 8; i += BLOCK) dst[i] = src[i];
  if (dst_vals) {
    float4* vdst = (float4*)dst_vals;
    for (int i = tid; i < m_al / 4; i += BLOCK) {
      const uint4 k = ((const uint4*)bkey)[i];
      vdst[i] = make_float4(unord_f32(~k.x), unord_f32(~k.y), unord_f32(~k.z), unord_f32(~k.w));
    }
  }
  lds_barrier();          // the next row may overwrite the buffers
}
}  // namespace

// Rows first, first + step, ... below n, each sorted in turn; the next row's similarities
// are loaded while the current one is sorted.
template <int BLOCK, int EPT>
__global__ __launch_bounds__(BLOCK) void sort_rows_kernel(const float* __restrict__ W, int n,
                                                          uint16_t* __restrict__ idx, float* __restrict__ vals,
                                                          int64_t ldi) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  float raw[EPT];
  uint32_t key[EPT], idp[EPT];
  int v = blockIdx.x;
  if (v < n) load_row<BLOCK, EPT>(W, n, Run{v, 0, n - 1}, raw);
  for (; v < n; v += gridDim.x) {
    row_keys<BLOCK, EPT>(raw, Run{v, 0, n - 1}, key, idp);
    if (v + (int)gridDim.x < n) load_row<BLOCK, EPT>(W, n, Run{v + (int)gridDim.x, 0, n - 1}, raw);
    sort_row_keys<BLOCK, EPT>(key, idp, n - 1, idx + (size_t)v * ldi, vals ? vals + (size_t)v * ldi : nullptr, smem);
  }
}

// Rows longer than one workgroup's LDS sorts at once (n - 1 > kMaxLdsSortN): each row of a
// block of `rows` rows from v0 is sorted as two runs, the columns [0, h) and [h, n) without
// v, each by the LDS radix sort above, into a staging area (run s of local row r at
// stage + (2r + s) * ldh); merge_halves_kernel then merges the two runs.
template <int BLOCK, int EPT>
__global__ __launch_bounds__(BLOCK) void sort_halves_kernel(const float* __restrict__ W, int n, int h, int v0,
                                                            int rows, uint16_t* __restrict__ st_idx,
                                                            float* __restrict__ st_vals, int64_t ldh) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  float raw[EPT];
  uint32_t key[EPT], idp[EPT];
  auto run_of = [&](int u) {
    const int v = v0 + (u >> 1), half = u & 1;
    const int c0 = half ? h : 0, c1 = half ? n : h;
    return Run{v, c0, (c1 - c0) - ((v >= c0 && v < c1) ? 1 : 0)};
  };
  const int units = 2 * rows;
  int u = blockIdx.x;
  if (u < units) load_row<BLOCK, EPT>(W, n, run_of(u), raw);
  for (; u < units; u += gridDim.x) {
    const Run r = run_of(u);
    row_keys<BLOCK, EPT>(raw, r, key, idp);
    if (u + (int)gridDim.x < units) load_row<BLOCK, EPT>(W, n, run_of(u + gridDim.x), raw);
    sort_row_keys<BLOCK, EPT>(key, idp, r.len, st_idx + (size_t)u * ldh, st_vals + (size_t)u * ldh, smem);
  }
}

// Merge of the two sorted runs of each staged row (one workgroup per row, grid-stride). Every
// id of the first run is below every id of the second, so on equal values the first run's
// entry goes first: the merged row is in (value desc, id asc) order. The runs' values are
// held in LDS; each thread finds where its share of the output starts by a binary search on
// the merge path, then merges its share sequentially.
constexpr int kMergeBlock = 1024;
__global__ __launch_bounds__(kMergeBlock) void merge_halves_kernel(const uint16_t* __restrict__ st_idx,
                                                                  const float* __restrict__ st_vals, int64_t ldh,
                                                                  int n, int h, int v0, int rows,
                                                                  uint16_t* __restrict__ idx, float* __restrict__ vals,
                                                                  int64_t ldi) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  float* sv = (float*)smem;                  // run A's values, then run B's
  const int m = n - 1, m_al = (m + 7) & ~7;
  const int tid = threadIdx.x;
  const int per = (m + kMergeBlock - 1) / kMergeBlock;
  for (int r = blockIdx.x; r < rows; r += gridDim.x) {
    const int v = v0 + r;
    const int a = h - (v < h ? 1 : 0), b = m - a;
    const uint16_t* ia = st_idx + (size_t)(2 * r) * ldh;
    const uint16_t* ib = st_idx + (size_t)(2 * r + 1) * ldh;
    const float* va = st_vals + (size_t)(2 * r) * ldh;
    const float* vb = st_vals + (size_t)(2 * r + 1) * ldh;
    for (int i = tid; i < a; i += kMergeBlock) sv[i] = va[i];
    for (int i = tid; i < b; i += kMergeBlock) sv[a + i] = vb[i];
    __syncthreads();
    const float* A = sv;
    const float* B = sv + a;
    const int d0 = tid * per < m ? tid * per : m;
    const int d1 = d0 + per < m ? d0 + per : m;
    // merge path: the number of A entries among the first d0 outputs (A[i] goes before B[j]
    // when A[i] >= B[j])
    int lo = d0 > b ? d0 - b : 0, hi = d0 < a ? d0 : a;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (A[mid] >= B[d0 - 1 - mid]) lo = mid + 1;
      else hi = mid;
    }
    int i = lo, j = d0 - lo;
    uint16_t* orow = idx + (size_t)v * ldi;
    float* ovals = vals ? vals + (size_t)v * ldi : nullptr;
    for (int d = d0; d < d1; ++d) {
      const bool take_a = i < a && (j >= b || A[i] >= B[j]);
      const float x = take_a ? A[i] : B[j];
      orow[d] = take_a ? ia[i] : ib[j];
      if (ovals) ovals[d] = x;
      i += take_a ? 1 : 0;
      j += take_a ? 0 : 1;
    }
    for (int d = m + tid; d < m_al; d += kMergeBlock) {
      orow[d] = 0xffff;
      if (ovals) ovals[d] = -INFINITY;
    }
    __syncthreads();                         // sv is reused by the next row
  }
}

// Batched form: work units are the rows of every listed job (prefix sums of n).
template <int BLOCK, int EPT>
__global__ __launch_bounds__(BLOCK) void batch_sort_kernel(const BatchJob* __restrict__ jobs,
                                                           const int* __restrict__ list,
                                                           const int* __restrict__ prefix, int nlist, int total) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  float raw[EPT];
  uint32_t key[EPT], idp[EPT];
  int u = blockIdx.x;
  const BatchJob* J = nullptr;
  int v = 0;
  if (u < total) {
    const int i = find_unit(prefix, nlist, u);
    J = &jobs[list[i]];
    v = u - prefix[i];
    load_row<BLOCK, EPT>(J->W, J->n, Run{v, 0, J->n - 1}, raw);
  }
  for (; u < total; u += gridDim.x) {
    const BatchJob* Jc = J;
    const int vc = v;
    row_keys<BLOCK, EPT>(raw, Run{vc, 0, Jc->n - 1}, key, idp);
    const int u2 = u + (int)gridDim.x;
    if (u2 < total) {
      const int i = find_unit(prefix, nlist, u2);
      J = &jobs[list[i]];
      v = u2 - prefix[i];
      load_row<BLOCK, EPT>(J->W, J->n, Run{v, 0, J->n - 1}, raw);
    }
    sort_row_keys<BLOCK, EPT>(key, idp, Jc->n - 1, Jc->idx + (size_t)vc * Jc->ldi,
                              Jc->vals ? Jc->vals + (size_t)vc * Jc->ldi : nullptr, smem);
  }
}

namespace {
// Launch configurations (BLOCK threads, EPT slots per thread): a row of n vertices fits a
// configuration when its n - 1 entries, padded to a multiple of 8, fit in BLOCK * EPT slots.
struct SortCfg {
  int block, ept;
};
constexpr SortCfg kCfgs[kSortConfigs] = {{256, 1},  {256, 4},  {512, 2},   {512, 4},   {256, 8},   {1024, 4},
                                         {512, 8},  {1024, 8}, {512, 16},  {1024, 12}, {1024, 16}, {1024, 20}};
// Size classes (by slot count) and the configuration each one uses by default.
constexpr int kClassCap[kSortClasses] = {256, 1024, 2048, 4096, 8192, 12288, 16384, 20480};
constexpr int kClassDefault[kSortClasses] = {0, 1, 3, 5, 7, 9, 10, 11};
int g_cus = 0;
int g_occ_rows[kSortConfigs], g_occ_batch[kSortConfigs];

template <int BLOCK, int EPT>
hipError_t sort_attr_t(int c) {
  const size_t lds = RowSort<BLOCK, EPT>::lds_bytes();
  const void* ks[2] = {(const void*)sort_rows_kernel<BLOCK, EPT>, (const void*)batch_sort_kernel<BLOCK, EPT>};
  int* occ[2] = {&g_occ_rows[c], &g_occ_batch[c]};
  for (int k = 0; k < 2; ++k) {
    hipFuncAttributes a;
    hipError_t e = hipFuncGetAttributes(&a, ks[k]);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute(ks[k], hipFuncAttributeMaxDynamicSharedMemorySize, (int)(kLdsBytes - a.sharedSizeBytes));
    if (e != hipSuccess) return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(occ[k], ks[k], BLOCK, lds);
    if (e != hipSuccess) return e;
    if (*occ[k] < 1) *occ[k] = 1;
  }
  return hipSuccess;
}

// Persistent grid: `rows_per_wg` = 0 fills the device once (resident workgroups); a positive
// value asks for about that many rows per workgroup instead (more, shorter-lived ones).
int grid_for(int rows, int occ, int rows_per_wg) {
  int g = (g_cus > 0 ? g_cus : 256) * occ;
  if (rows_per_wg > 0) g = (rows + rows_per_wg - 1) / rows_per_wg;
  return rows < g ? rows : (g < 1 ? 1 : g);
}

template <int BLOCK, int EPT>
hipError_t launch_sort_t(int c, const float* W, int n, uint16_t* idx, float* vals, int64_t ldi, hipStream_t s) {
  hipLaunchKernelGGL((sort_rows_kernel<BLOCK, EPT>), dim3(grid_for(n, g_occ_rows[c], 0)), dim3(BLOCK),
                     (RowSort<BLOCK, EPT>::lds_bytes()), s, W, n, idx, vals, ldi);
  return hipGetLastError();
}

template <int BLOCK, int EPT>
hipError_t launch_batch_sort_t(int c, const BatchJob* jobs, const int* list, const int* prefix, int nlist,
                               int total, int rows_per_wg, hipStream_t s) {
  hipLaunchKernelGGL((batch_sort_kernel<BLOCK, EPT>), dim3(grid_for(total, g_occ_batch[c], rows_per_wg)),
                     dim3(BLOCK), (RowSort<BLOCK, EPT>::lds_bytes()), s, jobs, list, prefix, nlist, total);
  return hipGetLastError();
}

#define TMFG_SORT_CFGS(X)                                                                                     \
  X(0, 256, 1) X(1, 256, 4) X(2, 512, 2) X(3, 512, 4) X(4, 256, 8) X(5, 1024, 4) X(6, 512, 8) X(7, 1024, 8) \
  X(8, 512, 16) X(9, 1024, 12) X(10, 1024, 16) X(11, 1024, 20)
}  // namespace

int64_t sort_row_stride(int n) { return round_up(n - 1 > 0 ? n - 1 : 1, 8); }

// Kernel attributes and occupancies, set once per process (on the current device).
hipError_t sort_init_attributes() {
  int dev = 0;
  hipError_t e;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&g_cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
#define X(i, b, t) \
  if ((e = sort_attr_t<b, t>(i)) != hipSuccess) return e;
  TMFG_SORT_CFGS(X)
#undef X
  const void* ks[2] = {(const void*)sort_halves_kernel<kHalfBlock, kHalfEpt>, (const void*)merge_halves_kernel};
  for (const void* k : ks) {
    hipFuncAttributes a;
    if ((e = hipFuncGetAttributes(&a, k)) != hipSuccess) return e;
    if ((e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)(kLdsBytes - a.sharedSizeBytes))) != hipSuccess)
      return e;
  }
  return hipSuccess;
}

// The smallest class whose slots hold a row of n - 1 entries padded to a multiple of 8.
int sort_class(int n) {
  const int m_al = (int)round_up(n - 1 > 0 ? n - 1 : 1, 8);
  for (int c = 0; c < kSortClasses; ++c)
    if (m_al <= kClassCap[c]) return c;
  return kSortClasses - 1;
}

int sort_default_config(int cls) { return kClassDefault[cls]; }

// Whether configuration `cfg` holds rows of class `cls` (and is no more than twice its size).
bool sort_config_fits(int cfg, int cls) {
  const int cap = kCfgs[cfg].block * kCfgs[cfg].ept;
  return cap >= kClassCap[cls] && cap <= 2 * kClassCap[cls];
}

hipError_t launch_batch_sort(const BatchJob* jobs, const int* list, const int* prefix, int nlist, int total,
                             int n_max, int cfg, int rows_per_wg, hipStream_t s) {
  if (total <= 0) return hipSuccess;
  if (cfg < 0) cfg = kClassDefault[sort_class(n_max)];
  switch (cfg) {
#define X(i, b, t) \
  case i: return launch_batch_sort_t<b, t>(i, jobs, list, prefix, nlist, total, rows_per_wg, s);
    TMFG_SORT_CFGS(X)
#undef X
  }
  return hipErrorInvalidValue;
}

// Staging of the two-run sort: two runs per row, each with this stride.
int64_t sort_stage_stride(int n) { return round_up((n + 1) / 2, 8); }
size_t sort_stage_bytes(int n) {
  if (n - 1 <= kMaxLdsSortN) return 0;
  const int rows = n < kStageRows ? n : kStageRows;
  return (size_t)rows * 2 * (size_t)sort_stage_stride(n) * (sizeof(uint16_t) + sizeof(float));
}

hipError_t launch_sort_rows(const float* W, int n, uint16_t* idx, float* vals, int64_t ldi, void* stage,
                            hipStream_t s) {
  if (n - 1 > kMaxLdsSortN) {
    if (!stage) return hipErrorInvalidValue;
    const int h = n / 2;
    const int64_t ldh = sort_stage_stride(n);
    const int rows_max = n < kStageRows ? n : kStageRows;
    uint16_t* st_idx = (uint16_t*)stage;
    float* st_vals = (float*)((uint8_t*)stage + (size_t)rows_max * 2 * ldh * sizeof(uint16_t));
    const size_t half_lds = RowSort<kHalfBlock, kHalfEpt>::lds_bytes();
    const size_t merge_lds = (size_t)(n - 1) * sizeof(float);
    const int cus = g_cus > 0 ? g_cus : 256;
    for (int v0 = 0; v0 < n; v0 += rows_max) {
      const int rows = n - v0 < rows_max ? n - v0 : rows_max;
      const int g1 = 2 * rows < cus ? 2 * rows : cus;
      hipLaunchKernelGGL((sort_halves_kernel<kHalfBlock, kHalfEpt>), dim3(g1), dim3(kHalfBlock), half_lds, s, W, n,
                         h, v0, rows, st_idx, st_vals, ldh);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
      const int g2 = rows < cus ? rows : cus;
      hipLaunchKernelGGL(merge_halves_kernel, dim3(g2), dim3(kMergeBlock), merge_lds, s, st_idx, st_vals, ldh, n, h,
                         v0, rows, idx, vals, ldi);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
  }
  const int cfg = kClassDefault[sort_class(n)];
  switch (cfg) {
#define X(i, b, t) \
  case i: return launch_sort_t<b, t>(i, W, n, idx, vals, ldi, s);
    TMFG_SORT_CFGS(X)
#undef X
  }
  return hipErrorInvalidValue;
}

}  // namespace tmfg
