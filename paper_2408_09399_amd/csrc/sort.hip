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

// Global loads of one row into registers (raw similarities, position order).
template <int BLOCK, int EPT>
__device__ __forceinline__ void load_row(const float* __restrict__ W, int n, int v, float (&raw)[EPT]) {
  const int m = n - 1;
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const float* row = W + (size_t)v * n;
  // slots past the row read the row's last element (a valid address; the value is unused),
  // so that every load is unconditional
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int p = wave * RowSort<BLOCK, EPT>::WS + e * kWave + lane;
    const int j = p < v ? p : p + 1;
    raw[e] = row[j < m ? j : m];
  }
}

// Keys and ids of one row from its similarities (position order).
template <int BLOCK, int EPT>
__device__ __forceinline__ void row_keys(const float (&raw)[EPT], int n, int v, uint32_t (&key)[EPT],
                                         uint32_t (&idp)[EPT]) {
  const int m = n - 1;
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int p = wave * RowSort<BLOCK, EPT>::WS + e * kWave + lane;
    const int j = p < v ? p : p + 1;
    // branch-free select: slots past the row get the padding key and id
    const uint32_t in = 0u - (uint32_t)(p < m);
    key[e] = (~ord_f32(raw[e]) & in) | (kPadKey & ~in);
    idp[e] = ((uint32_t)j & in) | (0xffffu & ~in);
  }
}

// Sorts one row given as keys and ids (idp: id in the low 16 bits) and writes ids (and
// values) out.
template <int BLOCK, int EPT>
__device__ __forceinline__ void sort_row_keys(uint32_t (&key)[EPT], uint32_t (&idp)[EPT], int n, int v, uint16_t* __restrict__ idx,
                              float* __restrict__ vals, int64_t ldi, uint8_t* smem) {
  using RS = RowSort<BLOCK, EPT>;
  constexpr int NW = RS::NW, CAP = RS::CAP, WS = RS::WS;
  const int m = n - 1;
  const int m_al = (m + 7) & ~7;
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
  uint4* dst = (uint4*)(idx + (size_t)v * ldi);
  const uint4* src = (const uint4*)bid;
  for (int i = tid; i < m_al / 8; i += BLOCK) dst[i] = src[i];
  if (vals) {
    float4* vdst = (float4*)(vals + (size_t)v * ldi);
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
  if (v < n) load_row<BLOCK, EPT>(W, n, v, raw);
  for (; v < n; v += gridDim.x) {
    row_keys<BLOCK, EPT>(raw, n, v, key, idp);
    if (v + (int)gridDim.x < n) load_row<BLOCK, EPT>(W, n, v + gridDim.x, raw);
    sort_row_keys<BLOCK, EPT>(key, idp, n, v, idx, vals, ldi, smem);
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
    load_row<BLOCK, EPT>(J->W, J->n, v, raw);
  }
  for (; u < total; u += gridDim.x) {
    const BatchJob* Jc = J;
    const int vc = v;
    row_keys<BLOCK, EPT>(raw, Jc->n, vc, key, idp);
    const int u2 = u + (int)gridDim.x;
    if (u2 < total) {
      const int i = find_unit(prefix, nlist, u2);
      J = &jobs[list[i]];
      v = u2 - prefix[i];
      load_row<BLOCK, EPT>(J->W, J->n, v, raw);
    }
    sort_row_keys<BLOCK, EPT>(key, idp, Jc->n, vc, Jc->idx, Jc->vals, Jc->ldi, smem);
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

hipError_t launch_sort_rows(const float* W, int n, uint16_t* idx, float* vals, int64_t ldi, hipStream_t s) {
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
