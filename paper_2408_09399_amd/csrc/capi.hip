// libtmfg C ABI: plans, scratch memory and the build pipeline.
#include <climits>
#include "../../include/tmfg.h"
#include "common.h"
#include "internal.h"
#include "batchplan.h"

#include <mutex>
#include <new>

namespace {

thread_local int g_last_hip = 0;

tmfg_status hip_fail(hipError_t e) {
  g_last_hip = (int)e;
  return TMFG_E_HIP;
}

}  // namespace

extern "C" bool tmfg_batch_matches(tmfg_batch batch, const tmfg_job* jobs, int32_t count);
void tmfg::record_hip_error(int e) { g_last_hip = e; }

namespace {
#define TMFG_HIP(call)                       \
  do {                                       \
    hipError_t e_ = (call);                  \
    if (e_ != hipSuccess) return hip_fail(e_); \
  } while (0)

constexpr int kPhaseEvents = 5;

__global__ void reset_flags_kernel(uint32_t* flags) { *flags = 0; }

// Turn device error flags into a status word (for stage entry points).
__global__ void flags_to_status_kernel(const uint32_t* flags, int32_t* status) {
  const uint32_t f = *flags;
  *status = (f & tmfg::kFlagNonFinite) ? TMFG_E_NONFINITE
          : (f & tmfg::kFlagAsymmetric) ? TMFG_E_ASYMMETRIC
          : (f & tmfg::kFlagDegenerate) ? TMFG_E_DEGENERATE
          : f ? TMFG_E_INTERNAL : TMFG_OK;
}

struct Sizes {
  int n, L;
  int n_pad, L_pad;
  int64_t ldi;
  size_t z_bytes, w_bytes, idx_bytes, vals_bytes, scores_bytes, frec_bytes;
};

Sizes sizes_for(int n, int L) {
  Sizes s;
  s.n = n;
  s.L = L;
  s.n_pad = (int)tmfg::round_up(n, tmfg::corr_row_pad());
  s.L_pad = (int)tmfg::round_up(L < 2 ? 2 : L, tmfg::corr_k_pad());
  s.ldi = tmfg::sort_row_stride(n);
  s.z_bytes = (size_t)s.n_pad * s.L_pad * sizeof(float);
  s.w_bytes = (size_t)n * n * sizeof(float);
  s.idx_bytes = (size_t)n * s.ldi * sizeof(uint16_t);
  s.vals_bytes = (size_t)n * s.ldi * sizeof(float);
  s.scores_bytes = (size_t)n * sizeof(double);
  s.frec_bytes = (size_t)(2 * n - 4) * 16;
  return s;
}

// The device scratch of one build: where each buffer sits in one region of `bytes`
// bytes, every buffer on a 256-byte boundary.
struct Scratch {
  float* Z;
  float* W;
  uint16_t* idx;
  float* vals;
  double* scores;
  uint4* frec;
  uint32_t* dflags;
  int32_t* stats;
  uint8_t* lstate;
  uint8_t* stage;     // the row sort's staging area (rows longer than one workgroup's LDS), or null
  size_t bytes;
};

Scratch carve(uint8_t* base, int n, int L) {
  const Sizes s = sizes_for(n, L);
  Scratch r{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    uint8_t* p = base ? base + off : nullptr;
    off += (size_t)tmfg::round_up((int64_t)(bytes < 256 ? 256 : bytes), 256);
    return p;
  };
  r.Z = (float*)take(s.z_bytes);
  r.W = (float*)take(s.w_bytes);
  r.idx = (uint16_t*)take(s.idx_bytes);
  r.vals = (float*)take(s.vals_bytes);
  r.scores = (double*)take(s.scores_bytes);
  r.frec = (uint4*)take(s.frec_bytes);
  r.dflags = (uint32_t*)take(4);
  r.stats = (int32_t*)take(128);
  r.lstate = take(tmfg::loop_state_bytes(n));
  const size_t stage = tmfg::sort_stage_bytes(n);
  r.stage = stage ? take(stage) : nullptr;
  r.bytes = off;
  return r;
}

}  // namespace

struct tmfg_plan_s {
  int device = 0;
  int n_max = 0, L_max = 0, max_jobs = 0;
  uint32_t flags = 0;
  uint8_t* region = nullptr;    // one allocation holding the scratch below
  Scratch sc{};                 // similarity, standardised series, sorted rows, face records,
                                // flags, counters, the insertion loop's state between segments
  hipEvent_t ev[kPhaseEvents] = {};
  bool timed = false;
  tmfg_batch batch = nullptr;   // the last batch built through tmfg_build_batch
  int wall_khz = 100000;   // device wall-clock counter rate
};

namespace {

void plan_free(tmfg_plan p) {
  if (!p) return;
  hipFree(p->region);
  for (auto& e : p->ev)
    if (e) hipEventDestroy(e);
  if (p->batch) tmfg_batch_destroy(p->batch);
  delete p;
}

tmfg_status alloc(void** ptr, size_t bytes) {
  hipError_t e = hipMalloc(ptr, bytes < 256 ? 256 : bytes);
  if (e == hipErrorOutOfMemory) {
    g_last_hip = (int)e;
    return TMFG_E_NOMEM;
  }
  if (e != hipSuccess) return hip_fail(e);
  return TMFG_OK;
}

bool valid_n(int n, int n_max) { return n >= tmfg::kMinN && n <= n_max && n <= tmfg::kMaxN; }

void record(tmfg_plan p, int i, hipStream_t s) {
  if (p && (p->flags & TMFG_TIMING)) hipEventRecord(p->ev[i], s);
}

// Argument checks of a build job against the limits n_max and L_max (no GPU work).
tmfg_status check_job(const tmfg_job* job, int n_max, int L_max) {
  if (!job) return TMFG_E_INVALID;
  const int n = job->n;
  if ((job->X == nullptr) == (job->W == nullptr)) return TMFG_E_INVALID;
  if (!job->order || !job->edges || !job->faces || !job->status) return TMFG_E_INVALID;
  if (!valid_n(n, n_max)) return TMFG_E_SIZE;
  if (n > 4 && (!job->steps || !job->step_gain)) return TMFG_E_INVALID;
  if (job->X && (job->L < 2 || job->L > L_max)) return TMFG_E_SIZE;
  return TMFG_OK;
}

// Enqueue one whole build on `stream` using the scratch `sc` (sized for at least this job).
// `timed` (may be null) is the plan whose phase events are recorded.
tmfg_status enqueue_build(const Scratch& sc, uint32_t flags, const tmfg_job* job, hipStream_t stream,
                          tmfg_plan timed) {
  const int n = job->n;
  record(timed, 0, stream);
  hipLaunchKernelGGL(reset_flags_kernel, dim3(1), dim3(1), 0, stream, sc.dflags);
  TMFG_HIP(hipGetLastError());
  const float* Wt;
  if (job->X) {
    const Sizes s = sizes_for(n, job->L);
    float* Wdst = job->W_out ? job->W_out : sc.W;
    TMFG_HIP(tmfg::launch_standardize(job->X, n, job->L, sc.Z, s.n_pad, s.L_pad, sc.dflags, stream));
    TMFG_HIP(tmfg::launch_corr_gemm(sc.Z, n, s.L_pad, Wdst, stream));
    Wt = Wdst;
  } else {
    if (!(flags & TMFG_NO_VALIDATE)) TMFG_HIP(tmfg::launch_validate(job->W, n, sc.dflags, stream));
    if (job->W_out && job->W_out != job->W)
      TMFG_HIP(hipMemcpyAsync(job->W_out, job->W, (size_t)n * n * sizeof(float), hipMemcpyDeviceToDevice, stream));
    Wt = job->W;
  }
  record(timed, 1, stream);
  TMFG_HIP(tmfg::launch_seed_scores(Wt, n, sc.scores, stream));
  record(timed, 2, stream);
  const int64_t ldi = tmfg::sort_row_stride(n);
  TMFG_HIP(tmfg::launch_sort_rows(Wt, n, sc.idx, sc.vals, ldi, sc.stage, stream));
  record(timed, 3, stream);
  tmfg::LoopParams P{};
  P.W = Wt;
  P.n = n;
  P.idx = sc.idx;
  P.vals = sc.vals;
  P.ldi = ldi;
  P.scores = sc.scores;
  P.frec = sc.frec;
  P.flags = sc.dflags;
  P.order = job->order;
  P.edges = job->edges;
  P.steps = job->steps;
  P.step_gain = job->step_gain;
  P.faces = job->faces;
  P.status = job->status;
  P.stats = (flags & TMFG_STATS) ? sc.stats : nullptr;   // the loop's counters, when asked for
  P.m = n - 1;
  P.stop_at = INT_MAX;
  P.state = sc.lstate;
  P.max_rounds = tmfg::kWalkRounds;
  tmfg::rule_from_flags(flags, &P.paper, &P.prefix);
  TMFG_HIP(tmfg::launch_loop_compacting(P, sc.idx, sc.vals, stream));
  record(timed, 4, stream);
  return TMFG_OK;
}

}  // namespace

extern "C" {

const char* tmfg_status_string(tmfg_status s) {
  switch (s) {
    case TMFG_OK: return "ok";
    case TMFG_E_INVALID: return "invalid argument";
    case TMFG_E_SIZE: return "size out of range";
    case TMFG_E_NONFINITE: return "non-finite input";
    case TMFG_E_ASYMMETRIC: return "similarity matrix not bitwise symmetric";
    case TMFG_E_DEGENERATE: return "series with zero variance";
    case TMFG_E_NOMEM: return "out of device memory";
    case TMFG_E_HIP: return "HIP runtime error";
    case TMFG_E_INTERNAL: return "internal error";
    case TMFG_PENDING: return "request pending";
  }
  return "unknown status";
}

int tmfg_last_hip_error(void) { return g_last_hip; }

size_t tmfg_footprint_bytes(int32_t n_max, int32_t L_max, uint32_t flags) {
  (void)flags;
  if (n_max < tmfg::kMinN) return 0;
  return carve(nullptr, n_max, L_max < 2 ? 2 : L_max).bytes;
}

tmfg_status tmfg_plan_create(tmfg_plan* plan, int32_t n_max, int32_t L_max, int32_t max_jobs, uint32_t flags) {
  if (!plan) return TMFG_E_INVALID;
  *plan = nullptr;
  bool paper = false;
  int prefix = 0;
  // TMFG_IDX32 (32-bit ids for n above 32768) is declared but not provided
  if ((flags & ~(uint32_t)(TMFG_NO_VALIDATE | TMFG_TIMING | TMFG_STATS | tmfg::kRuleFlags)) ||
      !tmfg::rule_from_flags(flags, &paper, &prefix))
    return TMFG_E_INVALID;
  if (n_max < tmfg::kMinN || n_max > tmfg::kMaxN || L_max < 2 || max_jobs < 0) return TMFG_E_SIZE;
  if (prefix > 0 && n_max > tmfg::kMaxCorrN) return TMFG_E_SIZE;
  hipError_t e = tmfg::init_attributes_once();
  if (e != hipSuccess) return hip_fail(e);
  tmfg_plan p = new (std::nothrow) tmfg_plan_s();
  if (!p) return TMFG_E_NOMEM;
  e = hipGetDevice(&p->device);
  if (e != hipSuccess) {
    delete p;
    return hip_fail(e);
  }
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, p->device) == hipSuccess && khz > 0)
    p->wall_khz = khz;
  p->n_max = n_max;
  p->L_max = L_max;
  p->max_jobs = max_jobs;
  p->flags = flags;
  const size_t bytes = carve(nullptr, n_max, L_max).bytes;
  tmfg_status st = alloc((void**)&p->region, bytes);
  if (st != TMFG_OK) {
    plan_free(p);
    return st;
  }
  p->sc = carve(p->region, n_max, L_max);
  for (auto& ev : p->ev) {
    e = hipEventCreate(&ev);
    if (e != hipSuccess) {
      plan_free(p);
      return hip_fail(e);
    }
  }
  *plan = p;
  return TMFG_OK;
}

tmfg_status tmfg_plan_destroy(tmfg_plan plan) {
  if (!plan) return TMFG_OK;
  hipError_t e = hipDeviceSynchronize();
  plan_free(plan);
  if (e != hipSuccess) return hip_fail(e);
  return TMFG_OK;
}

tmfg_status tmfg_build(tmfg_plan plan, const tmfg_job* job, hipStream_t stream) {
  if (!plan) return TMFG_E_INVALID;
  const tmfg_status st = check_job(job, plan->n_max, plan->L_max);
  if (st != TMFG_OK) return st;
  const tmfg_status e = enqueue_build(plan->sc, plan->flags, job, stream, plan);
  if (e != TMFG_OK) return e;
  plan->timed = (plan->flags & TMFG_TIMING) != 0;
  return TMFG_OK;
}

tmfg_status tmfg_build_batch(tmfg_plan plan, const tmfg_job* jobs, int32_t count, hipStream_t stream) {
  if (!plan || !jobs || count <= 0) return TMFG_E_INVALID;
  if (count > plan->max_jobs) return TMFG_E_SIZE;
  if (!tmfg_batch_matches(plan->batch, jobs, count)) {
    if (plan->batch) {
      tmfg_batch_destroy(plan->batch);
      plan->batch = nullptr;
    }
    const tmfg_status st =
        tmfg_batch_create(&plan->batch, jobs, count, plan->flags & (TMFG_NO_VALIDATE | tmfg::kRuleFlags));
    if (st != TMFG_OK) return st;
  }
  return tmfg_batch_run(plan->batch, stream);
}

tmfg_status tmfg_plan_phase_ms(tmfg_plan plan, float ms[5]) {
  if (!plan || !ms) return TMFG_E_INVALID;
  if (!plan->timed) return TMFG_E_INVALID;
  TMFG_HIP(hipEventSynchronize(plan->ev[4]));
  for (int i = 0; i < 4; ++i) TMFG_HIP(hipEventElapsedTime(&ms[i], plan->ev[i], plan->ev[i + 1]));
  TMFG_HIP(hipEventElapsedTime(&ms[4], plan->ev[0], plan->ev[4]));
  return TMFG_OK;
}

tmfg_status tmfg_plan_stats(tmfg_plan plan, int32_t out[32]) {
  if (!plan || !out || !(plan->flags & TMFG_STATS)) return TMFG_E_INVALID;
  TMFG_HIP(hipMemcpy(out, plan->sc.stats, 128, hipMemcpyDeviceToHost));
  for (int i = 5; i <= 10; ++i) out[i] = (int32_t)((int64_t)out[i] * 1000 / plan->wall_khz);
  for (int i = 16; i < 20; ++i) out[i] = (int32_t)((int64_t)out[i] * 1000 / plan->wall_khz);
  return TMFG_OK;
}

tmfg_status tmfg_correlation(tmfg_plan plan, const float* X, int32_t n, int32_t L, float* W, int32_t* status,
                             hipStream_t stream) {
  if (!plan || !X || !W || !status) return TMFG_E_INVALID;
  if (!valid_n(n, plan->n_max) || L < 2 || L > plan->L_max) return TMFG_E_SIZE;
  const Sizes s = sizes_for(n, L);
  hipLaunchKernelGGL(reset_flags_kernel, dim3(1), dim3(1), 0, stream, plan->sc.dflags);
  TMFG_HIP(hipGetLastError());
  TMFG_HIP(tmfg::launch_standardize(X, n, L, plan->sc.Z, s.n_pad, s.L_pad, plan->sc.dflags, stream));
  TMFG_HIP(tmfg::launch_corr_gemm(plan->sc.Z, n, s.L_pad, W, stream));
  hipLaunchKernelGGL(flags_to_status_kernel, dim3(1), dim3(1), 0, stream, plan->sc.dflags, status);
  TMFG_HIP(hipGetLastError());
  return TMFG_OK;
}

tmfg_status tmfg_sort_rows(tmfg_plan plan, const float* W, int32_t n, uint16_t* idx, float* vals, int64_t ld,
                           hipStream_t stream) {
  if (!plan || !W || !idx) return TMFG_E_INVALID;
  if (!valid_n(n, plan->n_max)) return TMFG_E_SIZE;
  if (ld % 8 != 0 || ld < tmfg::sort_row_stride(n) || ((uintptr_t)idx & 15u) || ((uintptr_t)vals & 15u))
    return TMFG_E_INVALID;
  TMFG_HIP(tmfg::launch_sort_rows(W, n, idx, vals, ld, plan->sc.stage, stream));
  return TMFG_OK;
}

tmfg_status tmfg_seed(tmfg_plan plan, const float* W, int32_t n, double* scores, int32_t* seed4,
                      hipStream_t stream) {
  if (!plan || !W || !scores || !seed4) return TMFG_E_INVALID;
  if (!valid_n(n, plan->n_max)) return TMFG_E_SIZE;
  TMFG_HIP(tmfg::launch_seed_scores(W, n, scores, stream));
  TMFG_HIP(tmfg::launch_seed_top4(scores, n, seed4, stream));
  return TMFG_OK;
}

tmfg_status tmfg_face_sweep(tmfg_plan plan, const float* W, int32_t n, const int32_t* faces, int32_t nfaces,
                            const uint32_t* inserted, int32_t* best_u, float* best_gain, hipStream_t stream) {
  if (!plan || !W || !faces || !inserted || !best_u || !best_gain) return TMFG_E_INVALID;
  if (!valid_n(n, plan->n_max)) return TMFG_E_SIZE;
  if (nfaces < 0) return TMFG_E_SIZE;
  TMFG_HIP(tmfg::launch_face_sweep(W, n, faces, nfaces, inserted, best_u, best_gain, stream));
  return TMFG_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------------------
// Builds that allocate nothing: the scratch is one fixed array per GPU. In host code the
// name `scratch` stands for a host-side shadow, not a device address; the device address
// comes from hipGetSymbolAddress, once per device, and only that address reaches GPU work.
// ---------------------------------------------------------------------------------------
static __device__ __align__(256) uint8_t scratch[TMFG_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint8_t* g_scratch_ptr[kMaxDevices];   // device address of `scratch` on each device, or null

tmfg_status scratch_on_current_device(uint8_t** out) {
  int dev = 0;
  TMFG_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return TMFG_E_INVALID;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    TMFG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return TMFG_E_INTERNAL;
    g_scratch_ptr[dev] = (uint8_t*)p;
  }
  *out = g_scratch_ptr[dev];
  return TMFG_OK;
}
}  // namespace

extern "C" {

tmfg_status tmfg_build_noalloc(const tmfg_job* job, uint32_t flags, hipStream_t stream) {
  bool paper = false;
  int prefix = 0;
  if ((flags & ~(uint32_t)(TMFG_NO_VALIDATE | tmfg::kRuleFlags)) || !tmfg::rule_from_flags(flags, &paper, &prefix))
    return TMFG_E_INVALID;
  const tmfg_status st = check_job(job, prefix > 0 ? tmfg::kMaxCorrN : tmfg::kMaxN, INT_MAX);
  if (st != TMFG_OK) return st;
  const int L = job->X ? job->L : 2;
  if (carve(nullptr, job->n, L).bytes > TMFG_NOALLOC_SCRATCH_BYTES) return TMFG_E_SIZE;
  hipError_t e = tmfg::init_attributes_once();
  if (e != hipSuccess) return hip_fail(e);
  uint8_t* base = nullptr;
  const tmfg_status sa = scratch_on_current_device(&base);
  if (sa != TMFG_OK) return sa;
  return enqueue_build(carve(base, job->n, L), flags, job, stream, nullptr);
}

}  // extern "C"
