// Request server: TMFG builds of series that arrive in host memory, with continuous
// batching.
//
// One scheduler thread owns the GPU side. Requests wait in arrival order; the head request
// is admitted when its device footprint (input, scratch, results) and its pinned host
// footprint (staged input, results) fit in the free ranges of two regions allocated once at
// creation, so serving never calls the HIP allocator. Whenever a stream slot is idle, the
// head request and the waiting requests of its size class (all waiting requests with
// TMFG_SERVER_FIFO), up to max_batch, go there as one batch: the grouped kernels of the
// batched form, launched directly, and an event. Several slots let a new batch start while
// the long serial chains of an earlier one still run.
//
// A request completes on its own, not with its batch: the loop workgroup that finishes an
// instance copies its outputs into the request's range of the pinned region (allocated
// coherent, so device writes reach host memory) and then stores its status there with a
// system-scope release. The scheduler reads the open requests' status words (atomic
// acquire loads, once per pass of its loop, which always sleeps between passes) and
// finishes each request whose build has ended: its results are already in pinned memory.
// A finished request frees its device range and its staged input at once, and its pinned
// results when the caller collects them.
#include "../../include/tmfg.h"
#include "arena.h"
#include "batchplan.h"
#include "common.h"
#include "internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

// The face-rule flags of a batch, from server flags: TMFG_SERVER_RULE_PAPER or the plan flags
// TMFG_RULE_PAPER / TMFG_RULE_CORR_PREFIX(p), which the server also takes.
static uint32_t server_rule_flags(uint32_t flags) {
  return ((flags & TMFG_SERVER_RULE_PAPER) ? (uint32_t)TMFG_RULE_PAPER : 0u) | (flags & tmfg::kRuleFlags);
}

namespace {

constexpr int kMaxSlots = 8;
constexpr int kMaxBatch = 4096;
constexpr size_t kAlign = 256;

// Size classes of the scheduler: n in [4, 256), [256, 1024), [1024, 4096), [4096, ...).
int size_class(int n) { return n < 256 ? 0 : n < 1024 ? 1 : n < 4096 ? 2 : 3; }

int64_t clock_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// Byte offsets of one request's outputs; the same layout in device and pinned memory.
struct ResultLayout {
  size_t order = 0, edges = 0, steps = 0, gain = 0, faces = 0, status = 0, bytes = 0;
  explicit ResultLayout(int n) {
    size_t o = 0;
    auto put = [&](size_t b) {
      const size_t at = o;
      o += tmfg::align256(b);
      return at;
    };
    order = put((size_t)n * 4);
    edges = put((size_t)(3 * n - 6) * 8);
    steps = put((size_t)std::max(n - 4, 1) * 16);
    gain = put((size_t)std::max(n - 4, 1) * 4);
    faces = put((size_t)(2 * n - 4) * 12);
    status = put(4);
    bytes = o;
  }
};

enum class State { Waiting, Running, Done };

struct Request {
  int n = 0, L = 0;
  std::vector<float> X;              // the caller's series until dispatch
  size_t x_bytes = 0, scratch = 0, res_bytes = 0;
  size_t dev_bytes = 0;              // input, results, scratch
  size_t dev_off = 0;
  size_t hx_off = 0, hr_off = 0;     // pinned: staged input (until done), results (until polled)
  State state = State::Waiting;
  int32_t status = TMFG_OK;
  int64_t arrival = 0, dispatch = 0, done = 0;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;         // the batch's kernels have finished
  char* d_desc = nullptr;            // device: descriptors, lists, queue counter
  char* h_desc = nullptr;            // pinned staging of descriptors and lists
  std::vector<Request*> reqs;
  bool busy = false;
};

}  // namespace

struct tmfg_server_s {
  tmfg_server_config cfg{};
  int device = 0;
  char* dev_base = nullptr;
  char* host_base = nullptr;
  tmfg::RangeAllocator dev_alloc, host_alloc;
  Slot slots[kMaxSlots];
  int nslots = 0;
  size_t jobs_bytes = 0, ints_cap = 0;

  std::mutex mu;
  std::condition_variable cv_work;   // a request arrived, memory was released, or stop
  std::condition_variable cv_done;   // requests finished
  bool kick = false, stop = false;
  std::deque<Request*> waiting;
  std::unordered_map<int64_t, std::unique_ptr<Request>> reqs;
  int64_t next_ticket = 1;
  std::thread worker;

  int64_t submitted = 0, completed = 0, dispatches = 0, dispatched = 0;
  int64_t min_arrival = INT64_MAX, last_done = 0;
  std::vector<double> lat_ms;
};

namespace {

tmfg_status fail(hipError_t e) {
  tmfg::record_hip_error((int)e);
  return e == hipErrorOutOfMemory ? TMFG_E_NOMEM : TMFG_E_HIP;
}

// Enqueues one batch on an idle slot. Called by the scheduler without the lock held; the
// slot's requests are not touched by any other thread while they run.
hipError_t dispatch(tmfg_server s, Slot& slot) {
  const int count = (int)slot.reqs.size();
  std::vector<tmfg_job> jobs(count);
  for (int i = 0; i < count; ++i) {
    Request* r = slot.reqs[i];
    char* d = s->dev_base + r->dev_off;
    std::memcpy(s->host_base + r->hx_off, r->X.data(), (size_t)r->n * r->L * 4);
    std::vector<float>().swap(r->X);
    const ResultLayout rl(r->n);
    char* res = d + r->x_bytes;
    tmfg_job& j = jobs[i];
    std::memset(&j, 0, sizeof(j));
    j.n = r->n;
    j.L = r->L;
    j.X = (const float*)d;
    j.order = (int32_t*)(res + rl.order);
    j.edges = (int32_t*)(res + rl.edges);
    j.steps = (int32_t*)(res + rl.steps);
    j.step_gain = (float*)(res + rl.gain);
    j.faces = (int32_t*)(res + rl.faces);
    j.status = (int32_t*)(res + rl.status);
  }
  tmfg::BatchSpec spec;
  if (tmfg::batch_describe(jobs.data(), count, server_rule_flags(s->cfg.flags), spec) != TMFG_OK ||
      spec.ints.size() > s->ints_cap)
    return hipErrorInvalidValue;
  tmfg::BatchJob* hj = (tmfg::BatchJob*)slot.h_desc;
  int* hi = (int*)(slot.h_desc + s->jobs_bytes);
  for (int i = 0; i < count; ++i) {
    Request* r = slot.reqs[i];
    tmfg::batch_job_desc(jobs[i], s->dev_base + r->dev_off + r->x_bytes + ResultLayout(r->n).bytes, hj[i]);
    // the host copies the loop fills at the end of the build; the status word is read by the
    // scheduler, so it holds TMFG_PENDING before any kernel of the batch is enqueued
    const ResultLayout rl(r->n);
    char* h = s->host_base + r->hr_off;
    hj[i].hout.order = (int32_t*)(h + rl.order);
    hj[i].hout.edges = (int32_t*)(h + rl.edges);
    hj[i].hout.steps = (int32_t*)(h + rl.steps);
    hj[i].hout.step_gain = (float*)(h + rl.gain);
    hj[i].hout.faces = (int32_t*)(h + rl.faces);
    hj[i].hout.status = (int32_t*)(h + rl.status);
    __atomic_store_n(hj[i].hout.status, (int32_t)TMFG_PENDING, __ATOMIC_RELEASE);
  }
  std::memcpy(hi, spec.ints.data(), spec.ints.size() * 4);
  tmfg::BatchLaunch L;
  L.d_jobs = (tmfg::BatchJob*)slot.d_desc;
  L.d_ints = (const int*)(slot.d_desc + s->jobs_bytes);
  L.d_queue = (int*)(slot.d_desc + s->jobs_bytes + tmfg::align256(s->ints_cap * 4));
  hipError_t e;
  if ((e = tmfg::batch_grid(s->device, count, spec.n_max, spec.paper, spec.prefix, &L.grid)) != hipSuccess) return e;
  const hipStream_t st = slot.stream;
  if ((e = hipMemcpyAsync(L.d_jobs, hj, sizeof(tmfg::BatchJob) * count, hipMemcpyHostToDevice, st)) != hipSuccess)
    return e;
  if ((e = hipMemcpyAsync((void*)L.d_ints, hi, spec.ints.size() * 4, hipMemcpyHostToDevice, st)) != hipSuccess)
    return e;
  for (Request* r : slot.reqs)
    if ((e = hipMemcpyAsync(s->dev_base + r->dev_off, s->host_base + r->hx_off, (size_t)r->n * r->L * 4,
                            hipMemcpyHostToDevice, st)) != hipSuccess)
      return e;
  if ((e = tmfg::batch_enqueue(spec, L, st)) != hipSuccess) return e;
  return hipEventRecord(slot.done, st);
}

// The published status of request r (pinned memory the device writes), or TMFG_PENDING.
int32_t published(tmfg_server s, const Request* r) {
  return __atomic_load_n((const int32_t*)(s->host_base + r->hr_off + ResultLayout(r->n).status), __ATOMIC_ACQUIRE);
}

// Marks one request finished (lock held): frees its device range and staged input.
void finish_request(tmfg_server s, Request* r, int32_t status, int64_t t) {
  r->status = status;
  r->done = t;
  r->state = State::Done;
  s->dev_alloc.release(r->dev_off, r->dev_bytes);
  s->host_alloc.release(r->hx_off, r->x_bytes);
  s->lat_ms.push_back((double)(t - r->arrival) * 1e-6);
  s->min_arrival = std::min(s->min_arrival, r->arrival);
  s->last_done = std::max(s->last_done, t);
  ++s->completed;
  s->cv_done.notify_all();
}

// Finishes the slot's requests whose builds have published their results and takes them off
// the slot (lock held): a finished request may be collected, and freed, by tmfg_server_poll as
// soon as the lock is released. Once the batch's kernels have ended (`all`), every request
// left is finished, one whose status was not published with `forced_status`, and the slot is
// free again.
void sweep_slot(tmfg_server s, Slot& slot, bool all, int32_t forced_status) {
  const int64_t t = clock_ns();
  for (auto it = slot.reqs.begin(); it != slot.reqs.end();) {
    Request* r = *it;
    const int32_t st = published(s, r);
    if (st != TMFG_PENDING || all) {
      finish_request(s, r, st != TMFG_PENDING ? st : forced_status, t);
      it = slot.reqs.erase(it);
    } else {
      ++it;
    }
  }
  if (all) slot.busy = false;
}

void scheduler(tmfg_server s) {
  hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    s->kick = false;
    bool busy = false;
    for (int k = 0; k < s->nslots; ++k) {
      Slot& slot = s->slots[k];
      if (!slot.busy) continue;
      const hipError_t q = hipEventQuery(slot.done);
      if (q == hipSuccess) {
        sweep_slot(s, slot, true, TMFG_E_INTERNAL);   // every build of a finished batch publishes
      } else if (q == hipErrorNotReady) {
        busy = true;
        sweep_slot(s, slot, false, TMFG_OK);
      } else {
        tmfg::record_hip_error((int)q);
        hipStreamSynchronize(slot.stream);
        sweep_slot(s, slot, true, TMFG_E_HIP);
      }
    }
    if (s->stop && !busy) break;
    for (int k = 0; k < s->nslots && !s->stop; ++k) {
      Slot& slot = s->slots[k];
      if (slot.busy || s->waiting.empty()) continue;
      // admit the oldest request, then (unless FIFO) later ones of its size class, while
      // both footprints fit; the first one that does not fit ends the batch
      const bool fifo = (s->cfg.flags & TMFG_SERVER_FIFO) != 0;
      const int cls = size_class(s->waiting.front()->n);
      for (auto it = s->waiting.begin(); it != s->waiting.end() && (int)slot.reqs.size() < s->cfg.max_batch;) {
        Request* r = *it;
        if (!fifo && size_class(r->n) != cls) {
          ++it;
          continue;
        }
        size_t doff, hx, hr;
        if (!s->dev_alloc.alloc(r->dev_bytes, &doff)) break;
        if (!s->host_alloc.alloc(r->x_bytes, &hx)) {
          s->dev_alloc.release(doff, r->dev_bytes);
          break;
        }
        if (!s->host_alloc.alloc(r->res_bytes, &hr)) {
          s->host_alloc.release(hx, r->x_bytes);
          s->dev_alloc.release(doff, r->dev_bytes);
          break;
        }
        r->dev_off = doff;
        r->hx_off = hx;
        r->hr_off = hr;
        r->state = State::Running;
        it = s->waiting.erase(it);
        slot.reqs.push_back(r);
      }
      if (slot.reqs.empty()) break;        // the head does not fit yet
      slot.busy = true;
      const int64_t t = clock_ns();
      for (Request* r : slot.reqs) r->dispatch = t;
      ++s->dispatches;
      s->dispatched += (int64_t)slot.reqs.size();
      lk.unlock();
      const hipError_t e = dispatch(s, slot);
      lk.lock();
      if (e != hipSuccess) {
        tmfg::record_hip_error((int)e);
        hipStreamSynchronize(slot.stream);
        sweep_slot(s, slot, true, TMFG_E_HIP);
      } else {
        busy = true;
      }
    }
    if (busy)
      s->cv_work.wait_for(lk, std::chrono::microseconds(20), [&] { return s->kick; });
    else
      s->cv_work.wait(lk, [&] { return s->kick || s->stop; });
  }
}

void server_free(tmfg_server s) {
  for (int k = 0; k < kMaxSlots; ++k) {
    Slot& slot = s->slots[k];
    if (slot.stream) hipStreamSynchronize(slot.stream);
    if (slot.done) hipEventDestroy(slot.done);
    if (slot.stream) hipStreamDestroy(slot.stream);
    hipFree(slot.d_desc);
    hipHostFree(slot.h_desc);
  }
  hipFree(s->dev_base);
  hipHostFree(s->host_base);
  delete s;
}

}  // namespace

extern "C" {

int64_t tmfg_server_now_ns(void) { return clock_ns(); }

tmfg_status tmfg_server_create(tmfg_server* out, const tmfg_server_config* cfg) {
  if (!out) return TMFG_E_INVALID;
  *out = nullptr;
  bool paper = false;
  int prefix = 0;
  if (!cfg || cfg->hbm_budget == 0 || cfg->host_budget == 0 || cfg->max_batch < 1 || cfg->max_batch > kMaxBatch ||
      cfg->n_streams < 1 || cfg->n_streams > kMaxSlots ||
      (cfg->flags & ~(uint32_t)(TMFG_SERVER_FIFO | TMFG_SERVER_RULE_PAPER | tmfg::kRuleFlags)) ||
      !tmfg::rule_from_flags(server_rule_flags(cfg->flags), &paper, &prefix))
    return TMFG_E_INVALID;
  if (cfg->n_max < tmfg::kMinN || cfg->n_max > tmfg::kMaxBatchN || cfg->L_max < 2) return TMFG_E_SIZE;
  hipError_t e = tmfg::init_attributes_once();
  if (e != hipSuccess) return fail(e);
  tmfg_server s = new (std::nothrow) tmfg_server_s();
  if (!s) return TMFG_E_NOMEM;
  s->cfg = *cfg;
  s->nslots = cfg->n_streams;
  s->jobs_bytes = tmfg::align256((size_t)cfg->max_batch * sizeof(tmfg::BatchJob));
  s->ints_cap = tmfg::batch_ints_capacity(cfg->max_batch);
  const size_t desc_bytes = s->jobs_bytes + tmfg::align256(s->ints_cap * 4) + kAlign;
  if ((e = hipGetDevice(&s->device)) != hipSuccess || (e = hipMalloc((void**)&s->dev_base, cfg->hbm_budget)) != hipSuccess ||
      // coherent: the loops' copies of finished builds' results reach host memory as they are written
      (e = hipHostMalloc((void**)&s->host_base, cfg->host_budget, hipHostMallocCoherent)) != hipSuccess) {
    server_free(s);
    return fail(e);
  }
  s->dev_alloc.reset(cfg->hbm_budget, kAlign);
  s->host_alloc.reset(cfg->host_budget, kAlign);
  for (int k = 0; k < s->nslots; ++k) {
    Slot& slot = s->slots[k];
    if ((e = hipStreamCreateWithFlags(&slot.stream, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&slot.done, hipEventDisableTiming)) != hipSuccess ||
        (e = hipMalloc((void**)&slot.d_desc, desc_bytes)) != hipSuccess ||
        (e = hipHostMalloc((void**)&slot.h_desc, desc_bytes, 0)) != hipSuccess) {
      server_free(s);
      return fail(e);
    }
  }
  s->worker = std::thread(scheduler, s);
  *out = s;
  return TMFG_OK;
}

tmfg_status tmfg_server_submit(tmfg_server s, const float* X_host, int32_t n, int32_t L, int64_t arrival_ns,
                               int64_t* ticket) {
  if (!s || !X_host || !ticket) return TMFG_E_INVALID;
  if (n < tmfg::kMinN || n > s->cfg.n_max || L < 2 || L > s->cfg.L_max) return TMFG_E_SIZE;
  std::unique_ptr<Request> r(new (std::nothrow) Request());
  if (!r) return TMFG_E_NOMEM;
  r->n = n;
  r->L = L;
  // scratch of the batched build of an X job that keeps no W
  tmfg_job probe;
  std::memset(&probe, 0, sizeof(probe));
  int32_t dummy[1];
  probe.n = n;
  probe.L = L;
  probe.X = X_host;
  probe.order = probe.edges = probe.steps = probe.faces = probe.status = dummy;
  probe.step_gain = (float*)dummy;
  const tmfg_status st = tmfg::job_scratch_bytes(probe, &r->scratch);
  if (st != TMFG_OK) return st;
  r->x_bytes = tmfg::align256((size_t)n * L * 4);
  r->res_bytes = ResultLayout(n).bytes;
  r->dev_bytes = r->x_bytes + r->res_bytes + r->scratch;
  if (s->dev_alloc.round(r->dev_bytes) > s->dev_alloc.capacity() ||
      s->host_alloc.round(r->x_bytes) + s->host_alloc.round(r->res_bytes) > s->host_alloc.capacity())
    return TMFG_E_SIZE;
  try {
    r->X.assign(X_host, X_host + (size_t)n * L);
  } catch (...) {
    return TMFG_E_NOMEM;
  }
  r->arrival = arrival_ns > 0 ? arrival_ns : clock_ns();
  std::lock_guard<std::mutex> g(s->mu);
  const int64_t t = s->next_ticket++;
  s->waiting.push_back(r.get());
  s->reqs.emplace(t, std::move(r));
  ++s->submitted;
  s->kick = true;
  s->cv_work.notify_one();
  *ticket = t;
  return TMFG_OK;
}

tmfg_status tmfg_server_poll(tmfg_server s, int64_t ticket, int32_t wait_ms, tmfg_server_result* out) {
  if (!s || !out) return TMFG_E_INVALID;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return TMFG_E_INVALID;
  Request* r = it->second.get();
  auto ready = [&] { return r->state == State::Done; };
  if (!ready()) {
    if (wait_ms == 0) return TMFG_PENDING;
    if (wait_ms < 0) s->cv_done.wait(lk, ready);
    else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), ready)) return TMFG_PENDING;
  }
  const int n = r->n;
  const ResultLayout rl(n);
  const char* h = s->host_base + r->hr_off;
  // outputs of a failed build are undefined, as for tmfg_build
  if (out->order) std::memcpy(out->order, h + rl.order, (size_t)n * 4);
  if (out->edges) std::memcpy(out->edges, h + rl.edges, (size_t)(3 * n - 6) * 8);
  if (out->steps && n > 4) std::memcpy(out->steps, h + rl.steps, (size_t)(n - 4) * 16);
  if (out->step_gain && n > 4) std::memcpy(out->step_gain, h + rl.gain, (size_t)(n - 4) * 4);
  if (out->faces) std::memcpy(out->faces, h + rl.faces, (size_t)(2 * n - 4) * 12);
  out->n = n;
  out->status = r->status;
  out->arrival_ns = r->arrival;
  out->dispatch_ns = r->dispatch;
  out->done_ns = r->done;
  s->host_alloc.release(r->hr_off, r->res_bytes);
  s->reqs.erase(it);
  s->kick = true;
  s->cv_work.notify_one();
  return TMFG_OK;
}

tmfg_status tmfg_server_stats(tmfg_server s, tmfg_server_report* rep, int32_t reset) {
  if (!s || !rep) return TMFG_E_INVALID;
  std::lock_guard<std::mutex> g(s->mu);
  std::memset(rep, 0, sizeof(*rep));
  rep->submitted = s->submitted;
  rep->completed = s->completed;
  rep->dispatches = s->dispatches;
  rep->waiting = (int64_t)s->waiting.size();
  if (!s->lat_ms.empty()) {
    std::vector<double> v(s->lat_ms);
    std::sort(v.begin(), v.end());
    const size_t N = v.size();
    auto rank = [&](double p) { return v[std::min(N - 1, (size_t)std::ceil(p * (double)N) - 1)]; };
    rep->p50_ms = rank(0.50);
    rep->p99_ms = rank(0.99);
    double sum = 0;
    for (double x : v) sum += x;
    rep->mean_ms = sum / (double)N;
    rep->max_ms = v.back();
    const double span = (double)(s->last_done - s->min_arrival) * 1e-9;
    rep->builds_per_s = span > 0 ? (double)N / span : 0.0;
  }
  rep->mean_batch = s->dispatches ? (double)s->dispatched / (double)s->dispatches : 0.0;
  if (reset) {
    s->submitted = s->completed = s->dispatches = s->dispatched = 0;
    s->min_arrival = INT64_MAX;
    s->last_done = 0;
    s->lat_ms.clear();
  }
  return TMFG_OK;
}

tmfg_status tmfg_server_destroy(tmfg_server s) {
  if (!s) return TMFG_OK;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
    s->kick = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  server_free(s);
  return TMFG_OK;
}

}  // extern "C"
