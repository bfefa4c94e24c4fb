// Host-side description of one set of grouped launches over many independent builds
// (internal to libtmfg). Used by the captured batches and by the request server.
#pragma once
#include "../../include/tmfg.h"
#include "internal.h"

#include <utility>
#include <vector>

namespace tmfg {

inline size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// One phase's work list inside BatchSpec::ints: job indices at o_list, unit prefixes at
// o_prefix (nlist + 1 entries, the last one is `total`).
struct GroupList {
  int nlist = 0, total = 0, n_max = 0;
  size_t o_list = 0, o_prefix = 0;
};

// The correlation GEMM runs in two groups, instances below kGemmSplitN and the others, each
// with its own tile (kGemmTiles[t]); the lists of both tiles are kept for each group.
constexpr int kGemmGroups = 2, kGemmSplitN = 1024;
constexpr int kGemmTiles[2] = {128, 64};

struct BatchSpec {
  int count = 0, n_max = 0;
  bool paper = false;                // every instance uses the paper's face rule
  int prefix = 0;                    // > 0: every instance uses corr-tmfg with this prefix
  std::vector<int> ints;             // every list, each padded to a multiple of 64 ints
  GroupList stdz, valid, seed, sort[8];
  GroupList gemm[kGemmGroups][2];    // [group][tile index]
  size_t o_order = 0;                // job indices by n descending: the loop's queue order
  std::vector<size_t> scratch;       // device scratch bytes of each job
};

// Checks one job's arguments and gives the scratch bytes it needs in a batch.
tmfg_status job_scratch_bytes(const tmfg_job& j, size_t* bytes);

// Work lists and scratch sizes of a set of jobs.
tmfg_status batch_describe(const tmfg_job* jobs, int count, uint32_t flags, BatchSpec& spec);

// Ints the lists of a batch of `count` jobs can take at most.
size_t batch_ints_capacity(int count);

// Device descriptor of a job whose scratch (job_scratch_bytes) starts at `scratch`.
void batch_job_desc(const tmfg_job& j, char* scratch, BatchJob& J);

// Where the descriptors and lists of one launch set live on the device.
struct BatchLaunch {
  BatchJob* d_jobs = nullptr;
  const int* d_ints = nullptr;
  int* d_queue = nullptr;
  int grid = 1;                                             // persistent loop workgroups
  int sort_cfg[kSortClasses] = {-1, -1, -1, -1, -1, -1, -1, -1};   // -1: the class default
  int sort_rows = 0;                                        // rows per sort workgroup (0: resident fill)
  int max_rounds = kWalkRounds;                             // walk rounds before the full-row sweep
  int gemm_tile[kGemmGroups] = {0, 0};                      // index into kGemmTiles of each GEMM group
  std::vector<std::pair<const float*, float*>> w_copies;    // caller W -> W_out
  std::vector<size_t> w_copy_bytes;
};

// Enqueues every phase of the batch on `s` (no allocation, no synchronisation).
hipError_t batch_enqueue(const BatchSpec& spec, const BatchLaunch& L, hipStream_t s);
// The row sorts of one size class alone, and the insertion loops alone (with the reset of
// the status flags and the queue they need); inputs of each must already be in place.
hipError_t batch_enqueue_sort(const BatchSpec& spec, const BatchLaunch& L, int cls, hipStream_t s);
// The correlation GEMM of one group alone (its standardised inputs must be in place).
hipError_t batch_enqueue_gemm(const BatchSpec& spec, const BatchLaunch& L, int group, hipStream_t s);
hipError_t batch_enqueue_loop(const BatchSpec& spec, const BatchLaunch& L, hipStream_t s);

// Persistent loop grid for `count` jobs of largest size n_max: the loop workgroups that
// fit on the device at once, at most one per job.
hipError_t batch_grid(int device, int count, int n_max, bool paper, int prefix, int* grid);

// The face rule that plan or batch flags select: false when they name an unknown rule, both
// rules, or a corr-tmfg prefix outside [1, kMaxPrefix] (or a prefix without that rule).
inline bool rule_from_flags(uint32_t flags, bool* paper, int* prefix) {
  const bool corr = (flags & TMFG_RULE_CORR) != 0;
  const int p = (int)((flags & TMFG_PREFIX_MASK) >> TMFG_PREFIX_SHIFT);
  *paper = (flags & TMFG_RULE_PAPER) != 0;
  *prefix = corr ? p : 0;
  if (corr) return !*paper && p >= 1 && p <= kMaxPrefix;
  return p == 0;
}
// Flag bits that select the face rule.
constexpr uint32_t kRuleFlags = TMFG_RULE_PAPER | TMFG_RULE_CORR | TMFG_PREFIX_MASK;

}  // namespace tmfg
