// Host-side launch wrappers of the TMFG kernels (internal to libtmfg).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace tmfg {

// Pearson similarity (standardise + FP32-MFMA GEMM).
hipError_t launch_standardize(const float* X, int n, int L, float* Z, int n_pad, int L_pad, uint32_t* flags,
                              hipStream_t s);
hipError_t launch_corr_gemm(const float* Z, int n, int L_pad, float* W, hipStream_t s);
int corr_row_pad();
int corr_k_pad();

// Finite and bitwise-symmetry check of a caller-supplied W.
hipError_t launch_validate(const float* W, int n, uint32_t* flags, hipStream_t s);

// Seed scores: float64 sums of each row without its diagonal, in index order.
hipError_t launch_seed_scores(const float* W, int n, double* scores, hipStream_t s);
// Top-4 of the scores (score desc, id asc) in rank order (one small workgroup).
hipError_t launch_seed_top4(const double* scores, int n, int32_t* seed4, hipStream_t s);

// Per-row order of the other vertices: (W[v][u] desc, u asc); u16 ids, and optionally the
// float32 similarities in the same order, both with row stride ldi.
// Rows of more than kMaxLdsSortN entries need a staging area of sort_stage_bytes(n) bytes.
hipError_t launch_sort_rows(const float* W, int n, uint16_t* idx, float* vals, int64_t ldi, void* stage,
                            hipStream_t s);
int64_t sort_row_stride(int n);
size_t sort_stage_bytes(int n);

// Exact best vertex of many faces by a full sweep of their three rows.
hipError_t launch_face_sweep(const float* W, int n, const int32_t* faces, int nfaces, const uint32_t* inserted,
                             int32_t* best_u, float* best_gain, hipStream_t s);

struct LoopParams {
  const float* W;
  int n;
  const uint16_t* idx;
  const float* vals;       // similarities in idx order (same row stride)
  int64_t ldi;
  const double* scores;
  uint4* frec;             // 2n-4 face records (scratch)
  const uint32_t* flags;   // error flags raised by earlier kernels of the same build
  int32_t* order;
  int32_t* edges;
  int32_t* steps;
  float* step_gain;
  int32_t* faces;
  int32_t* status;
  int32_t* stats;          // optional, 24 counters (see tmfg_plan_stats)
  bool paper;              // the paper's face rule (Algorithm 2) instead of the exact one
  int prefix;              // > 0: corr-tmfg (Algorithm 1) with this prefix size
  // Row compaction (single builds of the insertion loop; batches leave state null):
  int m;                   // entries per sorted row: n - 1, or n - s once compacted at s insertions
  int stop_at;             // save the loop's state and return once this many vertices are inserted
  int resume;              // continue from the saved state (the rows were compacted since)
  uint8_t* state;          // saved state, loop_state_bytes(n) bytes; null: no compaction
  int max_rounds;          // walk rounds before a walk gives up and its face is swept (exact either way)
  HostOut hout;            // optional (servers): host copies of the outputs, published at the end
};
constexpr int kWalkRounds = 64;   // the round limit of single builds and of untuned batches
constexpr int kMaxPrefix = 16;   // largest corr-tmfg prefix size

// Saved state of a single build between two segments of its loop (the lazy loop's or
// corr-tmfg's): this header, then, kStateHeader bytes in, an image of the loop's dynamic LDS.
struct LoopStateHeader {
  int live;                       // 1: a segment stopped at a checkpoint and the build goes on
  int ins, F, since_insert;       // vertices inserted, next face id, phases since the last insertion
  int compactions;                // checkpoints passed so far
  int m_old, m_new;               // entries per sorted row before and after the coming compaction
  int off_bits, off_ptr;          // byte offsets of the inserted bitmap and the row positions in the image
  unsigned long long ticks;       // loop time of the earlier segments
  unsigned long long cnt[20];     // the loop's counters
};
constexpr size_t kStateHeader = 256;
static_assert(sizeof(LoopStateHeader) <= kStateHeader, "the header fits its slot");

hipError_t launch_loop(const LoopParams& p, hipStream_t s);
size_t loop_lds_bytes(int n);
size_t corr_lds_bytes(int n);
size_t loop_state_bytes(int n);
// The loop of one build (the lazy loop, or corr-tmfg when p.prefix > 0) in segments: between
// two segments every sorted row drops its inserted entries (in place, order kept). idx and
// vals are p.idx and p.vals, writable.
hipError_t launch_loop_compacting(LoopParams p, uint16_t* idx, float* vals, hipStream_t s);
int loop_checkpoints(int n, int* s_out, int max);
hipError_t launch_corr(const LoopParams& p, hipStream_t s);

}  // namespace tmfg

namespace tmfg {

// One instance of a batch, as the batched kernels see it (device memory).
struct BatchJob {
  int n, L, n_pad, L_pad;
  int64_t ldi;
  const float* X;          // series, or null when W is given
  const float* W;          // the similarity matrix the build uses (caller's or scratch)
  float* Wdst;             // where the correlation kernels write W (null for a caller W)
  float* Z;
  uint16_t* idx;
  float* vals;
  double* scores;
  uint4* frec;
  uint32_t* flags;
  int32_t* order;
  int32_t* edges;
  int32_t* steps;
  float* step_gain;
  int32_t* faces;
  int32_t* status;
  HostOut hout;            // optional (servers): host copies of the outputs, published at the end
};

// Grouped launches over the instances of a batch. Each takes a device list of job indices
// and a device prefix array (prefix[i] = first unit of list[i], prefix[nlist] = total) of
// the phase's work units: rows, tiles or columns; blocks find their job by binary search.
hipError_t launch_batch_reset(BatchJob* jobs, int count, int* queue_head, bool clear_flags, hipStream_t s);
hipError_t launch_batch_standardize(const BatchJob* jobs, const int* list, const int* prefix, int nlist, int total,
                                    hipStream_t s);
// tile: 128 (four waves per tile) or 64 (one wave per tile); W's bits do not depend on it.
hipError_t launch_batch_gemm(const BatchJob* jobs, const int* list, const int* prefix, int nlist, int total,
                             int tile, hipStream_t s);
hipError_t launch_batch_validate(const BatchJob* jobs, const int* list, const int* prefix, int nlist, int total,
                                 hipStream_t s);
hipError_t launch_batch_seed(const BatchJob* jobs, const int* list, const int* prefix, int nlist, int total,
                             hipStream_t s);
// All instances in one sort launch share a size class (sort_class(n)); n_max is the
// largest n among them. cfg selects the launch configuration (-1: the class default; see
// sort_config_fits), rows_per_wg the persistent grid (0: one resident fill of the device).
constexpr int kSortClasses = 8;
constexpr int kSortConfigs = 12;
hipError_t launch_batch_sort(const BatchJob* jobs, const int* list, const int* prefix, int nlist, int total,
                             int n_max, int cfg, int rows_per_wg, hipStream_t s);
int sort_class(int n);
int sort_default_config(int cls);
bool sort_config_fits(int cfg, int cls);
// Persistent insertion loops: `grid` workgroups take instances from `order` (device array
// of job indices, largest first) through the counter at *queue_head.
hipError_t launch_batch_loop(const BatchJob* jobs, const int* order, int count, int* queue_head, int grid,
                             int n_max, bool paper, int max_rounds, hipStream_t s);
hipError_t launch_batch_corr(const BatchJob* jobs, const int* order, int count, int* queue_head, int grid,
                             int n_max, int prefix, hipStream_t s);
int corr_tiles(int n, int tile = 128);        // upper-triangular correlation tiles of n rows
hipError_t sort_init_attributes();            // LDS limits of the kernels (set once)
hipError_t loop_init_attributes();
hipError_t corr_init_attributes();
hipError_t init_attributes_once();            // both of the above, once per process
hipError_t batch_loop_occupancy(int* per_cu, int n_max, bool paper);   // loop workgroups per CU
hipError_t batch_corr_occupancy(int* per_cu, int n_max);
void record_hip_error(int e);                 // for tmfg_last_hip_error()
int validate_tiles(int n);                    // 32x32 validation tiles of an n x n matrix

// Binary search: the i in [0, nlist) with prefix[i] <= unit < prefix[i + 1].
__device__ __forceinline__ int find_unit(const int* prefix, int nlist, int unit) {
  int lo = 0, hi = nlist - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= unit) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

}  // namespace tmfg
