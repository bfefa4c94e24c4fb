// Batched TMFG builds: many independent instances of uneven n in one hipGraph replay.
//
// Every phase is one grouped launch over all instances (standardisation rows, correlation
// tiles, validation tiles, seed columns, row sorts per size class), and the insertion
// loops run in one persistent launch: about one workgroup per compute unit, each taking
// instances from a shared counter, largest n first, so the longest serial chains start
// at once and the small instances fill in behind them. The launch sequence is captured once
// into a graph and replayed by tmfg_batch_run. Instances share no scratch, and each one runs
// exactly the kernels of a single build, so its results are bitwise those of tmfg_build.
#include "../../include/tmfg.h"
#include "common.h"
#include "internal.h"
#include "batchplan.h"

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

namespace tmfg {

__global__ void batch_reset_kernel(BatchJob* jobs, int count, int* queue_head, int clear_flags) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (clear_flags && i < count) *jobs[i].flags = 0;
  if (i == 0) *queue_head = 0;
}

hipError_t launch_batch_reset(BatchJob* jobs, int count, int* queue_head, bool clear_flags, hipStream_t s) {
  hipLaunchKernelGGL(batch_reset_kernel, dim3((count + 255) / 256), dim3(256), 0, s, jobs, count, queue_head,
                     (int)clear_flags);
  return hipGetLastError();
}

hipError_t init_attributes_once() {
  static std::once_flag once;
  static hipError_t err = hipSuccess;
  std::call_once(once, [] {
    err = sort_init_attributes();
    if (err == hipSuccess) err = loop_init_attributes();
    if (err == hipSuccess) err = corr_init_attributes();
  });
  return err;
}

}  // namespace tmfg

namespace tmfg {

tmfg_status job_scratch_bytes(const tmfg_job& j, size_t* bytes) {
  if ((j.X == nullptr) == (j.W == nullptr)) return TMFG_E_INVALID;
  if (!j.order || !j.edges || !j.faces || !j.status) return TMFG_E_INVALID;
  if (j.n < kMinN || j.n > kMaxBatchN) return TMFG_E_SIZE;
  if (j.n > 4 && (!j.steps || !j.step_gain)) return TMFG_E_INVALID;
  if (j.X && j.L < 2) return TMFG_E_SIZE;
  const int n = j.n;
  const int64_t ldi = sort_row_stride(n);
  size_t b = align256(sizeof(uint32_t)) + align256((size_t)n * ldi * 2) + align256((size_t)n * ldi * 4) +
             align256((size_t)n * 8) + align256((size_t)(2 * n - 4) * 16);
  if (j.X) {
    const int n_pad = (int)round_up(n, corr_row_pad());
    const int L_pad = (int)round_up(j.L, corr_k_pad());
    b += align256((size_t)n_pad * L_pad * 4);
    if (!j.W_out) b += align256((size_t)n * n * 4);
  }
  *bytes = b;
  return TMFG_OK;
}

size_t batch_ints_capacity(int count) { return (size_t)12 * count + 16 + 30 * 64; }

tmfg_status batch_describe(const tmfg_job* jobs, int count, uint32_t flags, BatchSpec& spec) {
  spec = BatchSpec();
  spec.count = count;
  if (!rule_from_flags(flags, &spec.paper, &spec.prefix)) return TMFG_E_INVALID;
  spec.scratch.resize(count);
  for (int i = 0; i < count; ++i) {
    const tmfg_status st = job_scratch_bytes(jobs[i], &spec.scratch[i]);
    if (st != TMFG_OK) return st;
  }
  std::vector<int> lx, lw, la(count), pre_rows{0}, pre_vt{0}, pre_cols{0};
  std::vector<int> lg[kGemmGroups], pre_tiles[kGemmGroups][2];
  for (int g = 0; g < kGemmGroups; ++g)
    for (int t = 0; t < 2; ++t) pre_tiles[g][t].push_back(0);
  std::vector<int> lsort[8], pre_sort[8];
  int nmax_sort[8] = {0};
  for (int c = 0; c < 8; ++c) pre_sort[c].push_back(0);
  std::iota(la.begin(), la.end(), 0);
  for (int i = 0; i < count; ++i) {
    const tmfg_job& j = jobs[i];
    pre_cols.push_back(pre_cols.back() + j.n);
    if (j.X) {
      lx.push_back(i);
      pre_rows.push_back(pre_rows.back() + (int)round_up(j.n, corr_row_pad()));
      const int g = j.n < kGemmSplitN ? 0 : 1;
      lg[g].push_back(i);
      for (int t = 0; t < 2; ++t) pre_tiles[g][t].push_back(pre_tiles[g][t].back() + corr_tiles(j.n, kGemmTiles[t]));
    } else if (!(flags & TMFG_NO_VALIDATE)) {
      lw.push_back(i);
      pre_vt.push_back(pre_vt.back() + validate_tiles(j.n));
    }
    const int c = sort_class(j.n);
    lsort[c].push_back(i);
    pre_sort[c].push_back(pre_sort[c].back() + j.n);
    nmax_sort[c] = std::max(nmax_sort[c], j.n);
    spec.n_max = std::max(spec.n_max, j.n);
  }
  std::vector<int> order(count);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return jobs[x].n > jobs[y].n; });

  std::vector<int>& ints = spec.ints;
  auto put = [&](const std::vector<int>& v) {
    const size_t off = ints.size();
    ints.insert(ints.end(), v.begin(), v.end());
    while (ints.size() % 64) ints.push_back(0);
    return off;
  };
  auto list = [&](const std::vector<int>& l, const std::vector<int>& pre, int nmax) {
    GroupList g;
    g.nlist = (int)l.size();
    g.total = pre.back();
    g.n_max = nmax;
    g.o_list = put(l);
    g.o_prefix = put(pre);
    return g;
  };
  spec.stdz = list(lx, pre_rows, 0);
  for (int g = 0; g < kGemmGroups; ++g)
    for (int t = 0; t < 2; ++t) spec.gemm[g][t] = list(lg[g], pre_tiles[g][t], 0);
  spec.valid = list(lw, pre_vt, 0);
  spec.seed = list(la, pre_cols, 0);
  for (int c = 0; c < 8; ++c) spec.sort[c] = list(lsort[c], pre_sort[c], nmax_sort[c]);
  spec.o_order = put(order);
  return TMFG_OK;
}

void batch_job_desc(const tmfg_job& j, char* scratch, BatchJob& J) {
  char* cur = scratch;
  auto take = [&](size_t bytes) {
    char* p = cur;
    cur += align256(bytes);
    return p;
  };
  std::memset(&J, 0, sizeof(J));
  J.n = j.n;
  J.L = j.X ? j.L : 0;
  J.ldi = sort_row_stride(j.n);
  J.flags = (uint32_t*)take(4);
  J.idx = (uint16_t*)take((size_t)j.n * J.ldi * 2);
  J.vals = (float*)take((size_t)j.n * J.ldi * 4);
  J.scores = (double*)take((size_t)j.n * 8);
  J.frec = (uint4*)take((size_t)(2 * j.n - 4) * 16);
  if (j.X) {
    J.n_pad = (int)round_up(j.n, corr_row_pad());
    J.L_pad = (int)round_up(j.L, corr_k_pad());
    J.X = j.X;
    J.Z = (float*)take((size_t)J.n_pad * J.L_pad * 4);
    J.Wdst = j.W_out ? j.W_out : (float*)take((size_t)j.n * j.n * 4);
    J.W = J.Wdst;
  } else {
    J.W = j.W;
  }
  J.order = j.order;
  J.edges = j.edges;
  J.steps = j.steps;
  J.step_gain = j.step_gain;
  J.faces = j.faces;
  J.status = j.status;
}

hipError_t batch_enqueue(const BatchSpec& spec, const BatchLaunch& L, hipStream_t s) {
  const int* I = L.d_ints;
  auto lp = [&](const GroupList& g) { return I + g.o_list; };
  auto pp = [&](const GroupList& g) { return I + g.o_prefix; };
  hipError_t e;
  if ((e = launch_batch_reset(L.d_jobs, spec.count, L.d_queue, true, s)) != hipSuccess) return e;
  if ((e = launch_batch_standardize(L.d_jobs, lp(spec.stdz), pp(spec.stdz), spec.stdz.nlist, spec.stdz.total, s)) !=
      hipSuccess)
    return e;
  for (int g = 0; g < kGemmGroups; ++g)
    if ((e = batch_enqueue_gemm(spec, L, g, s)) != hipSuccess) return e;
  if ((e = launch_batch_validate(L.d_jobs, lp(spec.valid), pp(spec.valid), spec.valid.nlist, spec.valid.total, s)) !=
      hipSuccess)
    return e;
  for (size_t i = 0; i < L.w_copies.size(); ++i)
    if ((e = hipMemcpyAsync(L.w_copies[i].second, L.w_copies[i].first, L.w_copy_bytes[i], hipMemcpyDeviceToDevice,
                            s)) != hipSuccess)
      return e;
  if ((e = launch_batch_seed(L.d_jobs, lp(spec.seed), pp(spec.seed), spec.seed.nlist, spec.seed.total, s)) !=
      hipSuccess)
    return e;
  for (int c = 0; c < kSortClasses; ++c)
    if ((e = batch_enqueue_sort(spec, L, c, s)) != hipSuccess) return e;
  if (spec.prefix > 0)
    return launch_batch_corr(L.d_jobs, I + spec.o_order, spec.count, L.d_queue, L.grid, spec.n_max, spec.prefix, s);
  return launch_batch_loop(L.d_jobs, I + spec.o_order, spec.count, L.d_queue, L.grid, spec.n_max, spec.paper,
                           L.max_rounds, s);
}

hipError_t batch_enqueue_gemm(const BatchSpec& spec, const BatchLaunch& L, int group, hipStream_t s) {
  const GroupList& g = spec.gemm[group][L.gemm_tile[group]];
  if (g.nlist == 0) return hipSuccess;
  return launch_batch_gemm(L.d_jobs, L.d_ints + g.o_list, L.d_ints + g.o_prefix, g.nlist, g.total,
                           kGemmTiles[L.gemm_tile[group]], s);
}

hipError_t batch_enqueue_sort(const BatchSpec& spec, const BatchLaunch& L, int cls, hipStream_t s) {
  const GroupList& g = spec.sort[cls];
  if (g.nlist == 0) return hipSuccess;
  return launch_batch_sort(L.d_jobs, L.d_ints + g.o_list, L.d_ints + g.o_prefix, g.nlist, g.total, g.n_max,
                           L.sort_cfg[cls], L.sort_rows, s);
}

hipError_t batch_enqueue_loop(const BatchSpec& spec, const BatchLaunch& L, hipStream_t s) {
  hipError_t e;
  // the queue only: error flags raised by the earlier phases stay, and stop their instances
  if ((e = launch_batch_reset(L.d_jobs, spec.count, L.d_queue, false, s)) != hipSuccess) return e;
  if (spec.prefix > 0)
    return launch_batch_corr(L.d_jobs, L.d_ints + spec.o_order, spec.count, L.d_queue, L.grid, spec.n_max,
                             spec.prefix, s);
  return launch_batch_loop(L.d_jobs, L.d_ints + spec.o_order, spec.count, L.d_queue, L.grid, spec.n_max, spec.paper,
                           L.max_rounds, s);
}

hipError_t batch_grid(int device, int count, int n_max, bool paper, int prefix, int* grid) {
  int cus = 0, per_cu = 0;
  hipError_t e;
  if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device)) != hipSuccess) return e;
  if ((e = prefix > 0 ? batch_corr_occupancy(&per_cu, n_max) : batch_loop_occupancy(&per_cu, n_max, paper)) !=
      hipSuccess)
    return e;
  *grid = std::max(1, std::min(count, cus * std::max(per_cu, 1)));
  return hipSuccess;
}

}  // namespace tmfg

struct tmfg_batch_s {
  int device = 0;
  int count = 0;
  uint32_t flags = 0;
  void* arena = nullptr;
  size_t arena_bytes = 0;
  tmfg::BatchSpec spec;
  tmfg::BatchLaunch launch;
  hipStream_t capture_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<tmfg_job> jobs;   // the job set this batch was made for
  int tune_trials = 0;          // autotuning: configurations timed, and milliseconds spent
  float tune_ms = 0.0f;
  bool tune_cached = false;     // the tuned configuration came from the tuning cache
  int max_grid = 1;             // loop workgroups the device holds at once
};

namespace {

void batch_free(tmfg_batch b) {
  if (!b) return;
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  if (b->capture_stream) hipStreamDestroy(b->capture_stream);
  hipFree(b->arena);
  delete b;
}

tmfg_status fail(hipError_t e) {
  tmfg::record_hip_error((int)e);
  return e == hipErrorOutOfMemory ? TMFG_E_NOMEM : TMFG_E_HIP;
}

// Best of `reps` timed runs of `enq` on `st`, after one untimed run.
template <class F>
hipError_t time_best(hipStream_t st, hipEvent_t e0, hipEvent_t e1, int reps, F enq, float* ms) {
  hipError_t e;
  if ((e = enq()) != hipSuccess) return e;
  float best = 3.0e38f;
  for (int r = 0; r < reps; ++r) {
    if ((e = hipEventRecord(e0, st)) != hipSuccess || (e = enq()) != hipSuccess ||
        (e = hipEventRecord(e1, st)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess)
      return e;
    float t = 0.0f;
    if ((e = hipEventElapsedTime(&t, e0, e1)) != hipSuccess) return e;
    best = t < best ? t : best;
  }
  *ms = best;
  return hipSuccess;
}

// The launch configuration as tmfg_batch_config reports it ([10], [11], [15] aside).
void config_out(tmfg_batch b, int32_t out[16]) {
  for (int i = 0; i < 16; ++i) out[i] = 0;
  for (int c = 0; c < tmfg::kSortClasses; ++c) {
    const int cfg = b->launch.sort_cfg[c];
    out[c] = b->spec.sort[c].nlist == 0 ? -1 : (cfg >= 0 ? cfg : tmfg::sort_default_config(c));
  }
  out[8] = b->launch.sort_rows;
  out[9] = b->launch.grid;
  out[12] = b->launch.max_rounds;
  for (int g = 0; g < tmfg::kGemmGroups; ++g)
    out[13 + g] = b->spec.gemm[g][0].nlist == 0 ? 0 : tmfg::kGemmTiles[b->launch.gemm_tile[g]];
}

// Checks a configuration against the batch (entries of absent sort classes and GEMM groups
// are not looked at) and, when valid, applies it to the launch description.
bool config_apply(tmfg_batch b, const int32_t cfg[16], int max_grid) {
  tmfg::BatchLaunch L = b->launch;
  for (int c = 0; c < tmfg::kSortClasses; ++c) {
    if (b->spec.sort[c].nlist == 0) continue;
    if (cfg[c] < 0 || cfg[c] >= tmfg::kSortConfigs || !tmfg::sort_config_fits(cfg[c], c)) return false;
    L.sort_cfg[c] = cfg[c];
  }
  if (cfg[8] < 0 || cfg[9] < 1 || cfg[9] > max_grid || cfg[12] < 1 || cfg[12] > tmfg::kWalkRounds) return false;
  L.sort_rows = cfg[8];
  L.grid = cfg[9];
  L.max_rounds = cfg[12];
  for (int g = 0; g < tmfg::kGemmGroups; ++g) {
    if (b->spec.gemm[g][0].nlist == 0) continue;
    if (cfg[13 + g] == tmfg::kGemmTiles[0]) L.gemm_tile[g] = 0;
    else if (cfg[13 + g] == tmfg::kGemmTiles[1]) L.gemm_tile[g] = 1;
    else return false;
  }
  b->launch = L;
  return true;
}

// (Re)captures the batch's launches into its graph.
hipError_t capture(tmfg_batch b) {
  hipError_t e;
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  if (!b->capture_stream && (e = hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking)) != hipSuccess)
    return e;
  if ((e = hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess) return e;
  const hipError_t ee = tmfg::batch_enqueue(b->spec, b->launch, b->capture_stream);
  e = hipStreamEndCapture(b->capture_stream, &b->graph);
  if (ee != hipSuccess) return ee;
  if (e != hipSuccess) return e;
  return hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
}

// Tuned configurations, kept for the process and, when the environment variable
// TMFG_TUNE_CACHE names a file, across processes (one line per entry: key, tab, the 16
// configuration words). The key holds what the choice depends on: the device architecture
// and compute units, the HIP runtime version, the face rule and validation flags, and the
// batch's shape as the number of instances per (log2 n, log2 L) bucket, rounded to a power
// of two.
std::mutex g_tune_mu;
std::map<std::string, std::vector<int32_t>> g_tune_cache;
bool g_tune_loaded = false;

std::string tune_key(tmfg_batch b) {
  hipDeviceProp_t prop;
  int rt = 0;
  if (hipGetDeviceProperties(&prop, b->device) != hipSuccess || hipRuntimeGetVersion(&rt) != hipSuccess) return "";
  std::map<std::pair<int, int>, int> hist;
  for (const tmfg_job& j : b->jobs) {
    const int nb = 31 - __builtin_clz((unsigned)j.n);
    const int lb = j.X ? 31 - __builtin_clz((unsigned)std::max(j.L, 1)) : -1;
    ++hist[{nb, lb}];
  }
  std::string k = "tmfg-tune-1 ";
  k += prop.gcnArchName;
  k += " cu" + std::to_string(prop.multiProcessorCount) + " hip" + std::to_string(rt);
  k += " f" + std::to_string(b->flags & (TMFG_NO_VALIDATE | tmfg::kRuleFlags)) + " ";
  for (const auto& h : hist) {
    const int q = 32 - __builtin_clz((unsigned)h.second);   // count rounded to a power of two
    k += std::to_string(h.first.first) + "." + std::to_string(h.first.second) + ":" + std::to_string(q) + ",";
  }
  return k;
}

void tune_cache_load() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = std::getenv("TMFG_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  std::string line;
  for (int ch; (ch = std::fgetc(f)) != EOF;) {
    if (ch != '\n') {
      line.push_back((char)ch);
      continue;
    }
    const size_t tab = line.find('\t');
    if (tab != std::string::npos) {
      std::vector<int32_t> v;
      const char* p = line.c_str() + tab + 1;
      char* q = nullptr;
      for (int i = 0; i < 16; ++i, p = q) {
        const long x = std::strtol(p, &q, 10);
        if (q == p) break;
        v.push_back((int32_t)x);
      }
      if (v.size() == 16) g_tune_cache[line.substr(0, tab)] = v;
    }
    line.clear();
  }
  std::fclose(f);
}

bool tune_cache_get(const std::string& key, int32_t cfg[16]) {
  if (key.empty()) return false;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_cache_load();
  const auto it = g_tune_cache.find(key);
  if (it == g_tune_cache.end()) return false;
  std::copy(it->second.begin(), it->second.end(), cfg);
  return true;
}

void tune_cache_put(const std::string& key, const int32_t cfg[16]) {
  if (key.empty()) return;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_cache_load();
  g_tune_cache[key] = std::vector<int32_t>(cfg, cfg + 16);
  const char* path = std::getenv("TMFG_TUNE_CACHE");
  if (!path || !*path) return;
  // one write of the whole line, so that processes appending at once do not interleave
  std::string line = key + "\t";
  for (int i = 0; i < 16; ++i) line += (i ? " " : "") + std::to_string((int)cfg[i]);
  line += "\n";
  if (FILE* f = std::fopen(path, "a")) {
    std::fwrite(line.data(), 1, line.size(), f);
    std::fclose(f);
  }
}

// Autotuning on the batch's own inputs: one full run puts every phase's inputs in place,
// then each knob is timed on the phase it affects, one knob at a time, keeping a change only
// when it is at least 2% faster:
//   * the correlation GEMM's tile (128 or 64 rows) for instances below 1024 and for the rest;
//   * the launch configuration (threads x slots per thread) of each size class's row sort;
//   * the rows each sort workgroup takes (resident fill of the device, or 2, 4, 16 rows);
//   * the number of persistent loop workgroups (all that fit, three quarters, half);
//   * the walk rounds after which a face is swept instead (64, 16, 8; exact rule only).
// Results do not depend on any of these.
hipError_t autotune(tmfg_batch b) {
  tmfg::BatchLaunch& L = b->launch;
  const tmfg::BatchSpec& S = b->spec;
  hipStream_t st = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr, ea = nullptr, eb = nullptr;
  hipError_t e;
  if ((e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking)) != hipSuccess) return e;
  if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess ||
      (e = hipEventCreate(&ea)) != hipSuccess || (e = hipEventCreate(&eb)) != hipSuccess)
    goto done;
  if ((e = hipEventRecord(ea, st)) != hipSuccess) goto done;
  if ((e = tmfg::batch_enqueue(S, L, st)) != hipSuccess || (e = hipStreamSynchronize(st)) != hipSuccess) goto done;
  {
    auto sorts = [&]() -> hipError_t {
      for (int c = 0; c < tmfg::kSortClasses; ++c) {
        const hipError_t r = tmfg::batch_enqueue_sort(S, L, c, st);
        if (r != hipSuccess) return r;
      }
      return hipSuccess;
    };
    float best = 0.0f, t = 0.0f;
    for (int g = 0; g < tmfg::kGemmGroups; ++g) {
      if (S.gemm[g][0].nlist == 0) continue;
      L.gemm_tile[g] = 0;
      auto one = [&]() { return tmfg::batch_enqueue_gemm(S, L, g, st); };
      if ((e = time_best(st, e0, e1, 2, one, &best)) != hipSuccess) goto done;
      ++b->tune_trials;
      L.gemm_tile[g] = 1;
      if ((e = time_best(st, e0, e1, 2, one, &t)) != hipSuccess) goto done;
      ++b->tune_trials;
      if (!(t < 0.98f * best)) L.gemm_tile[g] = 0;
    }
    for (int c = 0; c < tmfg::kSortClasses; ++c) {
      if (S.sort[c].nlist == 0) continue;
      L.sort_cfg[c] = tmfg::sort_default_config(c);
      auto one = [&]() { return tmfg::batch_enqueue_sort(S, L, c, st); };
      if ((e = time_best(st, e0, e1, 2, one, &best)) != hipSuccess) goto done;
      ++b->tune_trials;
      for (int cfg = 0; cfg < tmfg::kSortConfigs; ++cfg) {
        if (cfg == tmfg::sort_default_config(c) || !tmfg::sort_config_fits(cfg, c)) continue;
        const int keep = L.sort_cfg[c];
        L.sort_cfg[c] = cfg;
        if ((e = time_best(st, e0, e1, 2, one, &t)) != hipSuccess) goto done;
        ++b->tune_trials;
        if (t < 0.98f * best) best = t;
        else L.sort_cfg[c] = keep;
      }
    }
    if ((e = time_best(st, e0, e1, 2, sorts, &best)) != hipSuccess) goto done;
    ++b->tune_trials;
    for (int rows : {2, 4, 16}) {
      const int keep = L.sort_rows;
      L.sort_rows = rows;
      if ((e = time_best(st, e0, e1, 2, sorts, &t)) != hipSuccess) goto done;
      ++b->tune_trials;
      if (t < 0.98f * best) best = t;
      else L.sort_rows = keep;
    }
    auto loops = [&]() { return tmfg::batch_enqueue_loop(S, L, st); };
    if ((e = time_best(st, e0, e1, 2, loops, &best)) != hipSuccess) goto done;
    ++b->tune_trials;
    const int full = L.grid;
    for (int g : {full * 3 / 4, full / 2}) {
      if (g < 1 || g == full) continue;
      const int keep = L.grid;
      L.grid = g;
      if ((e = time_best(st, e0, e1, 2, loops, &t)) != hipSuccess) goto done;
      ++b->tune_trials;
      if (t < 0.98f * best) best = t;
      else L.grid = keep;
    }
    for (int r : {16, 8}) {
      if (S.prefix > 0 || S.paper) break;      // only the exact rule walks
      const int keep = L.max_rounds;
      L.max_rounds = r;
      if ((e = time_best(st, e0, e1, 2, loops, &t)) != hipSuccess) goto done;
      ++b->tune_trials;
      if (t < 0.98f * best) best = t;
      else L.max_rounds = keep;
    }
  }
  if ((e = hipEventRecord(eb, st)) != hipSuccess || (e = hipEventSynchronize(eb)) != hipSuccess) goto done;
  e = hipEventElapsedTime(&b->tune_ms, ea, eb);
done:
  if (st) hipStreamSynchronize(st);
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  if (ea) hipEventDestroy(ea);
  if (eb) hipEventDestroy(eb);
  if (st) hipStreamDestroy(st);
  return e;
}

}  // namespace

extern "C" {

size_t tmfg_batch_footprint_bytes(const tmfg_job* jobs, int32_t count, uint32_t flags) {
  (void)flags;
  if (!jobs || count <= 0) return 0;
  size_t total = tmfg::align256((size_t)count * sizeof(tmfg::BatchJob)) + tmfg::align256(4) +
                 tmfg::align256(tmfg::batch_ints_capacity(count) * 4);
  for (int i = 0; i < count; ++i) {
    size_t b = 0;
    if (tmfg::job_scratch_bytes(jobs[i], &b) != TMFG_OK) return 0;
    total += b;
  }
  return total;
}

tmfg_status tmfg_batch_create(tmfg_batch* out, const tmfg_job* jobs, int32_t count, uint32_t flags) {
  if (!out) return TMFG_E_INVALID;
  *out = nullptr;
  if (!jobs || count <= 0) return TMFG_E_INVALID;
  if (flags & ~(uint32_t)(TMFG_NO_VALIDATE | TMFG_BATCH_NO_GRAPH | TMFG_BATCH_AUTOTUNE | tmfg::kRuleFlags))
    return TMFG_E_INVALID;
  tmfg::BatchSpec spec;
  const tmfg_status st = tmfg::batch_describe(jobs, count, flags, spec);
  if (st != TMFG_OK) return st;
  hipError_t e = tmfg::init_attributes_once();
  if (e != hipSuccess) return fail(e);
  tmfg_batch b = new (std::nothrow) tmfg_batch_s();
  if (!b) return TMFG_E_NOMEM;
  b->count = count;
  b->flags = flags;
  b->jobs.assign(jobs, jobs + count);
  b->spec = std::move(spec);
  if ((e = hipGetDevice(&b->device)) != hipSuccess) {
    batch_free(b);
    return fail(e);
  }

  // One arena: job descriptors, the integer lists, the queue counter, per-job scratch.
  const size_t jobs_bytes = tmfg::align256((size_t)count * sizeof(tmfg::BatchJob));
  const size_t ints_bytes = tmfg::align256(b->spec.ints.size() * 4);
  size_t total = jobs_bytes + ints_bytes + tmfg::align256(4);
  for (size_t x : b->spec.scratch) total += x;
  if ((e = hipMalloc(&b->arena, total)) != hipSuccess) {
    batch_free(b);
    return fail(e);
  }
  b->arena_bytes = total;
  char* base = (char*)b->arena;
  tmfg::BatchLaunch& L = b->launch;
  L.d_jobs = (tmfg::BatchJob*)base;
  int* d_ints = (int*)(base + jobs_bytes);
  L.d_ints = d_ints;
  L.d_queue = (int*)(base + jobs_bytes + ints_bytes);
  char* cur = base + jobs_bytes + ints_bytes + tmfg::align256(4);
  std::vector<tmfg::BatchJob> hj(count);
  for (int i = 0; i < count; ++i) {
    tmfg::batch_job_desc(jobs[i], cur, hj[i]);
    cur += b->spec.scratch[i];
    if (jobs[i].W && jobs[i].W_out && jobs[i].W_out != jobs[i].W) {
      L.w_copies.push_back({jobs[i].W, jobs[i].W_out});
      L.w_copy_bytes.push_back((size_t)jobs[i].n * jobs[i].n * 4);
    }
  }
  if ((e = hipMemcpy(L.d_jobs, hj.data(), sizeof(tmfg::BatchJob) * count, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(d_ints, b->spec.ints.data(), b->spec.ints.size() * 4, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = tmfg::batch_grid(b->device, count, b->spec.n_max, b->spec.paper, b->spec.prefix, &L.grid)) != hipSuccess) {
    batch_free(b);
    return fail(e);
  }

  b->max_grid = L.grid;
  if (flags & TMFG_BATCH_AUTOTUNE) {
    const std::string key = tune_key(b);
    int32_t cfg[16];
    if (tune_cache_get(key, cfg) && config_apply(b, cfg, b->max_grid)) {
      b->tune_cached = true;
    } else {
      if ((e = autotune(b)) != hipSuccess) {
        batch_free(b);
        return fail(e);
      }
      config_out(b, cfg);
      tune_cache_put(key, cfg);
    }
  }

  if (!(flags & TMFG_BATCH_NO_GRAPH) && (e = capture(b)) != hipSuccess) {
    batch_free(b);
    return fail(e);
  }
  *out = b;
  return TMFG_OK;
}

tmfg_status tmfg_batch_run(tmfg_batch batch, hipStream_t stream) {
  if (!batch) return TMFG_E_INVALID;
  hipError_t e = batch->exec ? hipGraphLaunch(batch->exec, stream) : tmfg::batch_enqueue(batch->spec, batch->launch, stream);
  if (e != hipSuccess) return fail(e);
  return TMFG_OK;
}

tmfg_status tmfg_batch_destroy(tmfg_batch batch) {
  if (!batch) return TMFG_OK;
  hipError_t e = hipDeviceSynchronize();
  batch_free(batch);
  if (e != hipSuccess) return fail(e);
  return TMFG_OK;
}

tmfg_status tmfg_batch_config(tmfg_batch batch, int32_t out[16]) {
  if (!batch || !out) return TMFG_E_INVALID;
  config_out(batch, out);
  out[10] = batch->tune_trials;
  out[11] = (int32_t)(batch->tune_ms + 0.5f);
  out[15] = batch->tune_cached ? 1 : 0;
  return TMFG_OK;
}

tmfg_status tmfg_batch_set_config(tmfg_batch batch, const int32_t cfg[16]) {
  if (!batch || !cfg) return TMFG_E_INVALID;
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return fail(e);
  const tmfg::BatchLaunch keep = batch->launch;
  if (!config_apply(batch, cfg, batch->max_grid)) return TMFG_E_INVALID;
  if (batch->exec && (e = capture(batch)) != hipSuccess) {
    batch->launch = keep;
    return fail(e);
  }
  return TMFG_OK;
}

bool tmfg_batch_matches(tmfg_batch batch, const tmfg_job* jobs, int32_t count) {
  return batch && batch->count == count && std::memcmp(batch->jobs.data(), jobs, sizeof(tmfg_job) * count) == 0;
}

}  // extern "C"
