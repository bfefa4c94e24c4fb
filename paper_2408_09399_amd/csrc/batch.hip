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

#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>
#include <vector>

namespace tmfg {

__global__ void batch_reset_kernel(BatchJob* jobs, int count, int* queue_head) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) *jobs[i].flags = 0;
  if (i == 0) *queue_head = 0;
}

hipError_t launch_batch_reset(BatchJob* jobs, int count, int* queue_head, hipStream_t s) {
  hipLaunchKernelGGL(batch_reset_kernel, dim3((count + 255) / 256), dim3(256), 0, s, jobs, count, queue_head);
  return hipGetLastError();
}

hipError_t init_attributes_once() {
  static std::once_flag once;
  static hipError_t err = hipSuccess;
  std::call_once(once, [] {
    err = sort_init_attributes();
    if (err == hipSuccess) err = loop_init_attributes();
  });
  return err;
}

}  // namespace tmfg

namespace {

struct List {
  int nlist = 0, total = 0, n_max = 0;
  const int* d_list = nullptr;
  const int* d_prefix = nullptr;
};

size_t al(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

struct tmfg_batch_s {
  int device = 0;
  int count = 0;
  uint32_t flags = 0;
  void* arena = nullptr;
  size_t arena_bytes = 0;
  tmfg::BatchJob* d_jobs = nullptr;
  int* d_queue = nullptr;
  const int* d_order = nullptr;
  int n_max = 0;
  int grid = 0;
  List stdz, gemm, valid, seed, sort[8];
  std::vector<std::pair<const float*, float*>> w_copies;   // caller W -> W_out
  std::vector<size_t> w_copy_bytes;
  hipStream_t capture_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<tmfg_job> jobs;   // the job set this batch was made for
};

namespace {

hipError_t enqueue(tmfg_batch b, hipStream_t s) {
  hipError_t e;
  if ((e = tmfg::launch_batch_reset(b->d_jobs, b->count, b->d_queue, s)) != hipSuccess) return e;
  if ((e = tmfg::launch_batch_standardize(b->d_jobs, b->stdz.d_list, b->stdz.d_prefix, b->stdz.nlist,
                                          b->stdz.total, s)) != hipSuccess)
    return e;
  if ((e = tmfg::launch_batch_gemm(b->d_jobs, b->gemm.d_list, b->gemm.d_prefix, b->gemm.nlist, b->gemm.total, s)) !=
      hipSuccess)
    return e;
  if ((e = tmfg::launch_batch_validate(b->d_jobs, b->valid.d_list, b->valid.d_prefix, b->valid.nlist,
                                       b->valid.total, s)) != hipSuccess)
    return e;
  for (size_t i = 0; i < b->w_copies.size(); ++i)
    if ((e = hipMemcpyAsync(b->w_copies[i].second, b->w_copies[i].first, b->w_copy_bytes[i],
                            hipMemcpyDeviceToDevice, s)) != hipSuccess)
      return e;
  if ((e = tmfg::launch_batch_seed(b->d_jobs, b->seed.d_list, b->seed.d_prefix, b->seed.nlist, b->seed.total, s)) !=
      hipSuccess)
    return e;
  for (int c = 0; c < 8; ++c) {
    const List& L = b->sort[c];
    if (L.nlist == 0) continue;
    if ((e = tmfg::launch_batch_sort(b->d_jobs, L.d_list, L.d_prefix, L.nlist, L.total, L.n_max, s)) != hipSuccess)
      return e;
  }
  return tmfg::launch_batch_loop(b->d_jobs, b->d_order, b->count, b->d_queue, b->grid, b->n_max, nullptr, s);
}

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

// Bytes of scratch one instance needs, and the check of its arguments.
tmfg_status job_scratch(const tmfg_job& j, size_t* bytes) {
  if ((j.X == nullptr) == (j.W == nullptr)) return TMFG_E_INVALID;
  if (!j.order || !j.edges || !j.faces || !j.status) return TMFG_E_INVALID;
  if (j.n < tmfg::kMinN || j.n > tmfg::kMaxN) return TMFG_E_SIZE;
  if (j.n > 4 && (!j.steps || !j.step_gain)) return TMFG_E_INVALID;
  if (j.X && j.L < 2) return TMFG_E_SIZE;
  const int n = j.n;
  const int64_t ldi = tmfg::sort_row_stride(n);
  size_t b = al(sizeof(uint32_t)) + al((size_t)n * ldi * 2) + al((size_t)n * ldi * 4) + al((size_t)n * 8) +
             al((size_t)(2 * n - 4) * 16);
  if (j.X) {
    const int n_pad = (int)tmfg::round_up(n, tmfg::corr_row_pad());
    const int L_pad = (int)tmfg::round_up(j.L, tmfg::corr_k_pad());
    b += al((size_t)n_pad * L_pad * 4);
    if (!j.W_out) b += al((size_t)n * n * 4);
  }
  *bytes = b;
  return TMFG_OK;
}

}  // namespace

extern "C" {

size_t tmfg_batch_footprint_bytes(const tmfg_job* jobs, int32_t count, uint32_t flags) {
  (void)flags;
  if (!jobs || count <= 0) return 0;
  size_t total = al((size_t)count * sizeof(tmfg::BatchJob)) + al(4) + al((size_t)(12 * count + 64) * 4);
  for (int i = 0; i < count; ++i) {
    size_t b = 0;
    if (job_scratch(jobs[i], &b) != TMFG_OK) return 0;
    total += b;
  }
  return total;
}

tmfg_status tmfg_batch_create(tmfg_batch* out, const tmfg_job* jobs, int32_t count, uint32_t flags) {
  if (!out) return TMFG_E_INVALID;
  *out = nullptr;
  if (!jobs || count <= 0) return TMFG_E_INVALID;
  if (flags & ~(uint32_t)(TMFG_NO_VALIDATE | TMFG_BATCH_NO_GRAPH)) return TMFG_E_INVALID;
  std::vector<size_t> scratch(count);
  for (int i = 0; i < count; ++i) {
    const tmfg_status st = job_scratch(jobs[i], &scratch[i]);
    if (st != TMFG_OK) return st;
  }
  hipError_t e = tmfg::init_attributes_once();
  if (e != hipSuccess) return fail(e);
  tmfg_batch b = new (std::nothrow) tmfg_batch_s();
  if (!b) return TMFG_E_NOMEM;
  b->count = count;
  b->flags = flags;
  b->jobs.assign(jobs, jobs + count);
  if ((e = hipGetDevice(&b->device)) != hipSuccess) {
    batch_free(b);
    return fail(e);
  }

  // Work lists of every phase (host side first).
  std::vector<int> lx, lw, la(count), pre_rows{0}, pre_tiles{0}, pre_vt{0}, pre_cols{0};
  std::vector<int> lsort[8], pre_sort[8];
  int nmax_sort[8] = {0};
  for (int c = 0; c < 8; ++c) pre_sort[c].push_back(0);
  std::iota(la.begin(), la.end(), 0);
  for (int i = 0; i < count; ++i) {
    const tmfg_job& j = jobs[i];
    pre_cols.push_back(pre_cols.back() + j.n);
    if (j.X) {
      lx.push_back(i);
      pre_rows.push_back(pre_rows.back() + (int)tmfg::round_up(j.n, tmfg::corr_row_pad()));
      pre_tiles.push_back(pre_tiles.back() + tmfg::corr_tiles(j.n));
    } else if (!(flags & TMFG_NO_VALIDATE)) {
      lw.push_back(i);
      pre_vt.push_back(pre_vt.back() + tmfg::validate_tiles(j.n));
    }
    const int c = tmfg::sort_class(j.n);
    lsort[c].push_back(i);
    pre_sort[c].push_back(pre_sort[c].back() + j.n);
    nmax_sort[c] = std::max(nmax_sort[c], j.n);
    b->n_max = std::max(b->n_max, j.n);
  }
  std::vector<int> order(count);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return jobs[x].n > jobs[y].n; });

  // One arena: job descriptors, the integer lists, the queue counter, per-job scratch.
  std::vector<int> ints;
  auto put = [&](const std::vector<int>& v) {
    const size_t off = ints.size();
    ints.insert(ints.end(), v.begin(), v.end());
    while (ints.size() % 64) ints.push_back(0);
    return off;
  };
  const size_t o_lx = put(lx), o_prow = put(pre_rows), o_ptile = put(pre_tiles), o_lw = put(lw), o_pvt = put(pre_vt),
               o_la = put(la), o_pcol = put(pre_cols), o_order = put(order);
  size_t o_ls[8], o_ps[8];
  for (int c = 0; c < 8; ++c) {
    o_ls[c] = put(lsort[c]);
    o_ps[c] = put(pre_sort[c]);
  }
  const size_t jobs_bytes = al((size_t)count * sizeof(tmfg::BatchJob));
  const size_t ints_bytes = al(ints.size() * 4);
  size_t total = jobs_bytes + ints_bytes + al(4);
  for (size_t x : scratch) total += x;
  if ((e = hipMalloc(&b->arena, total)) != hipSuccess) {
    batch_free(b);
    return fail(e);
  }
  b->arena_bytes = total;
  char* base = (char*)b->arena;
  b->d_jobs = (tmfg::BatchJob*)base;
  int* d_ints = (int*)(base + jobs_bytes);
  b->d_queue = (int*)(base + jobs_bytes + ints_bytes);
  char* cur = base + jobs_bytes + ints_bytes + al(4);
  auto take = [&](size_t bytes) {
    char* p = cur;
    cur += al(bytes);
    return p;
  };
  std::vector<tmfg::BatchJob> hj(count);
  for (int i = 0; i < count; ++i) {
    const tmfg_job& j = jobs[i];
    tmfg::BatchJob& J = hj[i];
    std::memset(&J, 0, sizeof(J));
    J.n = j.n;
    J.L = j.X ? j.L : 0;
    J.ldi = tmfg::sort_row_stride(j.n);
    J.flags = (uint32_t*)take(4);
    J.idx = (uint16_t*)take((size_t)j.n * J.ldi * 2);
    J.vals = (float*)take((size_t)j.n * J.ldi * 4);
    J.scores = (double*)take((size_t)j.n * 8);
    J.frec = (uint4*)take((size_t)(2 * j.n - 4) * 16);
    if (j.X) {
      J.n_pad = (int)tmfg::round_up(j.n, tmfg::corr_row_pad());
      J.L_pad = (int)tmfg::round_up(j.L, tmfg::corr_k_pad());
      J.X = j.X;
      J.Z = (float*)take((size_t)J.n_pad * J.L_pad * 4);
      J.Wdst = j.W_out ? j.W_out : (float*)take((size_t)j.n * j.n * 4);
      J.W = J.Wdst;
    } else {
      J.W = j.W;
      if (j.W_out) {
        b->w_copies.push_back({j.W, j.W_out});
        b->w_copy_bytes.push_back((size_t)j.n * j.n * 4);
      }
    }
    J.order = j.order;
    J.edges = j.edges;
    J.steps = j.steps;
    J.step_gain = j.step_gain;
    J.faces = j.faces;
    J.status = j.status;
  }
  if ((e = hipMemcpy(b->d_jobs, hj.data(), sizeof(tmfg::BatchJob) * count, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(d_ints, ints.data(), ints.size() * 4, hipMemcpyHostToDevice)) != hipSuccess) {
    batch_free(b);
    return fail(e);
  }
  auto list = [&](size_t ol, size_t op, int nlist, int tot, int nmax) {
    List L;
    L.nlist = nlist;
    L.total = tot;
    L.n_max = nmax;
    L.d_list = d_ints + ol;
    L.d_prefix = d_ints + op;
    return L;
  };
  b->stdz = list(o_lx, o_prow, (int)lx.size(), pre_rows.back(), 0);
  b->gemm = list(o_lx, o_ptile, (int)lx.size(), pre_tiles.back(), 0);
  b->valid = list(o_lw, o_pvt, (int)lw.size(), pre_vt.back(), 0);
  b->seed = list(o_la, o_pcol, count, pre_cols.back(), 0);
  for (int c = 0; c < 8; ++c) b->sort[c] = list(o_ls[c], o_ps[c], (int)lsort[c].size(), pre_sort[c].back(), nmax_sort[c]);
  b->d_order = d_ints + o_order;

  // Persistent loop grid: the workgroups that fit on the device at once, at most one per job.
  int cus = 0, per_cu = 0;
  if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device)) != hipSuccess ||
      (e = tmfg::batch_loop_occupancy(&per_cu, b->n_max)) != hipSuccess) {
    batch_free(b);
    return fail(e);
  }
  b->grid = std::max(1, std::min(count, cus * std::max(per_cu, 1)));

  if (!(flags & TMFG_BATCH_NO_GRAPH)) {
    if ((e = hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
      batch_free(b);
      return fail(e);
    }
    const hipError_t ee = enqueue(b, b->capture_stream);
    e = hipStreamEndCapture(b->capture_stream, &b->graph);
    if (ee != hipSuccess || e != hipSuccess) {
      batch_free(b);
      return fail(ee != hipSuccess ? ee : e);
    }
    if ((e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0)) != hipSuccess) {
      batch_free(b);
      return fail(e);
    }
  }
  *out = b;
  return TMFG_OK;
}

tmfg_status tmfg_batch_run(tmfg_batch batch, hipStream_t stream) {
  if (!batch) return TMFG_E_INVALID;
  hipError_t e = batch->exec ? hipGraphLaunch(batch->exec, stream) : enqueue(batch, stream);
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

bool tmfg_batch_matches(tmfg_batch batch, const tmfg_job* jobs, int32_t count) {
  return batch && batch->count == count && std::memcmp(batch->jobs.data(), jobs, sizeof(tmfg_job) * count) == 0;
}

}  // extern "C"
