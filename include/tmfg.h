/*
 * tmfg.h -- C ABI of libtmfg: triangular maximally filtered graph (TMFG) construction
 * on AMD Instinct MI355X (gfx950).
 *
 * The method is the TMFG of Raphael & Shun, "Faster Parallel Triangular Maximally
 * Filtered Graphs and Hierarchical Clustering" (arXiv 2408.09399): from an n x n
 * similarity matrix S (Section 2: S[i,j] is the weight of edge (i,j); Section 5: S is
 * the Pearson correlation of n time series) build a planar graph by starting from a
 * 4-clique and repeatedly joining one uninserted vertex to the three corners of one
 * triangular face, choosing the face/vertex pair whose three new edges have the largest
 * weight sum (the gain). Algorithms 1 and 2 give the set-up: four seed vertices of
 * largest row sum, one up-front sort of every row of S, then the insertion loop.
 *
 * Readings this library takes where the paper is silent:
 *   - seed score of v: sum over u != v of S[v][u], float64, added in index order of u;
 *     seed v1..v4 = the four largest by (score desc, id asc), in that order;
 *   - gain of face {a < b < c} and vertex u: float32 ((S[a][u] + S[b][u]) + S[c][u]);
 *   - each step takes the largest gain over all (live face, uninserted vertex) pairs; ties
 *     go to the lowest face id, then the lowest vertex id (this is the exact greedy rule of
 *     the sequential TMFG, Section 2). The paper's candidate rule (Algorithm 2) is
 *     available with TMFG_RULE_PAPER;
 *   - the split face f = {x < y < z} with new vertex u keeps id f as sorted(u,x,y);
 *     sorted(u,y,z) and sorted(u,x,z) take the next two ids;
 *   - the per-vertex sort orders u != v by (S[v][u] desc, u asc), -0.0 equal to +0.0.
 *
 * Conventions
 *   - All ids are 0-based int32. All data pointers are DEVICE pointers (hipMalloc or
 *     torch CUDA tensors on the plan's device) owned by the caller, unless stated.
 *   - Matrices are row-major, densely packed (row stride = number of columns).
 *   - Calls that take a stream only enqueue work on it and return at once; results are
 *     valid after the stream has been synchronised.
 *   - Argument errors are returned synchronously, before any GPU work is enqueued.
 *     Errors found on the device (non-finite input, asymmetric W, a constant series) are
 *     written as a tmfg_status to the caller's device status word; the other outputs of
 *     that call are then undefined. A failing HIP call returns TMFG_E_HIP; its raw
 *     hipError_t is available from tmfg_last_hip_error() on the same host thread.
 *   - A plan is not thread-safe: use one plan per host thread. Calls that share a plan
 *     must be ordered on one stream, since they share the plan's scratch memory.
 *   - Limits: 4 <= n <= 32768 for single builds (vertex and face ids are stored in 16 bits,
 *     and the 2n - 4 face ids of n = 32768 are the most that fit); 4 <= n <= 20480 for
 *     batches, servers and corr-tmfg (TMFG_RULE_CORR_PREFIX); 2 <= L. A row of up to 20480
 *     entries is sorted inside one workgroup's 160 KB LDS, a longer one as two halves that
 *     are then merged.
 */
#ifndef TMFG_H_
#define TMFG_H_

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TMFG_OK = 0,
  TMFG_E_INVALID = 1,     /* null pointer, both or neither of X and W, bad flags, misaligned buffer */
  TMFG_E_SIZE = 2,        /* n < 4, n > n_max (or above the limits below), L < 2, L > L_max */
  TMFG_E_NONFINITE = 3,   /* NaN or Inf in X or W (device-detected) */
  TMFG_E_ASYMMETRIC = 4,  /* W[i][j] and W[j][i] differ in their bits (device-detected) */
  TMFG_E_DEGENERATE = 5,  /* a series with all values equal: no Pearson correlation */
  TMFG_E_NOMEM = 6,       /* device allocation failed */
  TMFG_E_HIP = 7,         /* a HIP runtime call failed; see tmfg_last_hip_error() */
  TMFG_E_INTERNAL = 8,    /* an internal consistency check failed on the device */
  TMFG_PENDING = 9        /* server: the request has not finished yet */
} tmfg_status;

/* Plan and batch flags. */
enum {
  TMFG_NO_VALIDATE = 1u << 0,   /* skip the finite / bitwise-symmetry check of a caller W */
  TMFG_TIMING = 1u << 1,        /* record per-phase HIP events (tmfg_plan_phase_ms) */
  TMFG_BATCH_NO_GRAPH = 1u << 2, /* batch: launch the kernels directly instead of a graph */
  TMFG_BATCH_AUTOTUNE = 1u << 3, /* batch: pick launch configurations by timing them at creation */
  /* 32-bit vertex ids (n above 32768). Declared for the interface but not provided: ids and
     face ids are 16-bit throughout, and every call given this flag returns TMFG_E_INVALID. */
  TMFG_IDX32 = 1u << 4,
  /* Plans: record the insertion loop's counters and step timers (tmfg_plan_stats). They
     sit on the loop's critical path (counter updates after every face walk, clock reads
     between the steps of a phase) and cost about a tenth of the loop's time, so a plan made
     without this flag builds without them; results are the same bits either way. */
  TMFG_STATS = 1u << 5,
  /* The paper's candidate-limited face rule and heap schedule (Sections 4.1 and 4.2,
     Algorithm 2) instead of the exact greedy rule, for plans and batches. MaxCorrs[v] is
     the most similar uninserted vertex of v (the first uninserted entry of v's sorted row),
     evaluated when it is used; a face's pair is the MaxCorrs of its three corners with the
     largest gain (ties to the lowest vertex id); pairs are taken by (gain desc, face id
     asc), and a taken pair whose vertex is already inserted is recomputed and put back
     before the next pair is taken. The result is the one that heap order gives, bit for
     bit, not the exact greedy TMFG: its steps may take pairs of lower gain. */
  TMFG_RULE_PAPER = 1u << 8,
  /* corr-tmfg (Section 4.1, Algorithm 1) with a prefix size p, 1 <= p <= 16, for plans and
     batches: give TMFG_RULE_CORR_PREFIX(p). Faces hold pairs by the paper's candidate rule as
     with TMFG_RULE_PAPER, but each round takes the p pairs of largest (gain, then lowest face
     id), keeps for each vertex only the first of its pairs among them, applies the kept pairs
     in that order (the k-th kept pair's split takes the next two face ids in turn), and then
     recomputes, eagerly, every face whose pair vertex was inserted and every new face, against
     the uninserted set after the whole round. Exclusive with TMFG_RULE_PAPER. Up to n = 20480
     (each face's pair vertex is kept in LDS). */
  TMFG_RULE_CORR = 1u << 9
};
#define TMFG_PREFIX_SHIFT 16
#define TMFG_PREFIX_MASK (0xffu << TMFG_PREFIX_SHIFT)
#define TMFG_RULE_CORR_PREFIX(p) (TMFG_RULE_CORR | ((uint32_t)(p) << TMFG_PREFIX_SHIFT))

typedef struct tmfg_plan_s* tmfg_plan;
typedef struct tmfg_batch_s* tmfg_batch;

/* One TMFG construction. Exactly one of X and W is non-NULL. */
typedef struct {
  int32_t n;            /* number of vertices (series) */
  int32_t L;            /* series length; ignored when X is NULL */
  const float* X;       /* n x L series, or NULL */
  const float* W;       /* n x n similarity, finite and bitwise symmetric, or NULL */
  float* W_out;         /* optional n x n: the float32 similarity the build used (may be W
                           itself, which is then left as it is) */
  int32_t* order;       /* n: v1..v4 (seed rank order), then vertices in insertion order */
  int32_t* edges;       /* (3n-6) x 2: (v1,v2),(v1,v3),(v1,v4),(v2,v3),(v2,v4),(v3,v4),
                           then (u,x),(u,y),(u,z) for each step */
  int32_t* steps;       /* (n-4) x 4: face id f, corners x < y < z joined at each step
                           (may be NULL when n == 4) */
  float* step_gain;     /* n-4: float32 gain of each step (may be NULL when n == 4) */
  int32_t* faces;       /* (2n-4) x 3: final faces, ascending corner triples, by face id */
  int32_t* status;      /* 1: tmfg_status of the build, written last */
} tmfg_job;

/* Create a plan for builds with n <= n_max and L <= L_max on the current HIP device.
   Allocates the scratch (similarity matrix, standardised series, sorted ids, face
   records, the insertion loop's saved state, and for n_max > 20481 the row sort's staging
   area; see tmfg_footprint_bytes). A plan serves one build at a time: builds on one plan
   must be ordered (the same stream, or events), since each one rewrites all of the plan's
   scratch. max_jobs (>= 0) is the most jobs tmfg_build_batch accepts on this plan (0: the
   plan serves single builds only). Flags: TMFG_NO_VALIDATE, TMFG_TIMING, TMFG_STATS,
   TMFG_RULE_PAPER or TMFG_RULE_CORR_PREFIX(p) (n_max <= 20480); others, TMFG_IDX32 among
   them, give TMFG_E_INVALID. */
tmfg_status tmfg_plan_create(tmfg_plan* plan, int32_t n_max, int32_t L_max, int32_t max_jobs, uint32_t flags);

/* Release a plan and its scratch. Waits for the plan's outstanding work. NULL is a no-op. */
tmfg_status tmfg_plan_destroy(tmfg_plan plan);

/* Device bytes a plan for (n_max, L_max) holds. */
size_t tmfg_footprint_bytes(int32_t n_max, int32_t L_max, uint32_t flags);

/* Build one TMFG (Pearson similarity if X is given, the per-vertex sort, the seed and
   the n-4 insertions) asynchronously on `stream`. */
tmfg_status tmfg_build(tmfg_plan plan, const tmfg_job* job, hipStream_t stream);

/* Per-phase milliseconds of the plan's last build made with TMFG_TIMING: [0] similarity
   (or validation of a caller W), [1] seed scores, [2] row sort, [3] insertion loop
   (seed selection, initial faces and the n-4 steps), [4] total. Synchronises on the
   last event. */
tmfg_status tmfg_plan_phase_ms(tmfg_plan plan, float ms[5]);

/* Counters of the plan's last build (synchronous copy of 32 int32); TMFG_E_INVALID unless
   the plan was made with TMFG_STATS. [0] stale face
   recomputes, [1] walk rounds, [2] full-row sweeps, [3] selection phases, [4] walk
   batches, [5..9] microseconds spent in selection, chunk loading, walks, sweeps and
   publishing, [10] microseconds of the whole loop kernel, [11] similarities read from W
   by walks (those not carried by the sorted rows), [12] sum over selection phases of the
   deepest walk's rounds, [13] walks of 4 or more rounds, [14] walks of 16 or more rounds,
   [15] skip scans over fully inserted stretches, [16..19] microseconds one walk group
   spent loading and ranking list entries, reading candidate similarities, updating
   bounds, and skip-scanning (diagnostics: 0 unless the library is built with the walk
   timers on, kWalkDiag in loop.hip, which wait for every load and so slow the walks),
   [20] selection phases that found a stale maximum, [21] phases with more stale faces
   than one phase recomputes, [22] phases that loaded the most chunks one phase loads,
   [23] recomputed pairs that were not committed because a pair taken before them in heap
   order might change them (TMFG_RULE_PAPER), [24] row compactions, [25..31] reserved (0).
   From n = 512 on, a single build runs its loop in segments (every rule): it stops after
   n - n/4, n - n/8, ... insertions (under TMFG_RULE_CORR at the first round boundary at or
   past each count), as long as at least 128 vertices are left, and every sorted row drops
   its inserted entries (in place, order kept) before the loop resumes; results do not
   depend on it. Under TMFG_RULE_PAPER, [1] counts scans for the first uninserted entry of
   the corners' sorted rows instead of walk rounds. Under TMFG_RULE_CORR only these are
   kept: [0] faces recomputed because their pair vertex was inserted, [1] row scans,
   [2] extra passes (a round with more faces to recompute than one pass takes), [3] rounds,
   [5..9] microseconds in the scan for faces to recompute, their pairs, publishing,
   rebuilding chunk maxima and selection, [10] microseconds of the kernel, [24] row
   compactions; the others read 0. */
tmfg_status tmfg_plan_stats(tmfg_plan plan, int32_t out[32]);

/* ---- A build that allocates nothing ---------------------------------------------- */

/* For callers that cannot allocate device memory: code under HIP graph capture, tight
   serving loops, harnesses that forbid hipMalloc. Builds one TMFG as tmfg_build does (the
   same kernels, bit-identical results) with plan flags `flags` (TMFG_NO_VALIDATE,
   TMFG_RULE_PAPER or TMFG_RULE_CORR_PREFIX(p); TMFG_TIMING is refused with TMFG_E_INVALID),
   taking its scratch from one fixed device array inside the library instead of a plan:
   TMFG_NOALLOC_SCRATCH_BYTES bytes on each GPU it runs on, held from the library's loading
   on that GPU until the process ends. A job fits when tmfg_footprint_bytes(n, L, 0) is at
   most that size, with L = 2 when the job gives W (for example n <= 2048 for any L <= 2048,
   n <= 2530 at L = 256); a larger job gets TMFG_E_SIZE before any GPU work. The call
   allocates no memory; its first call on a device looks up the array's device address.
   All calls on one GPU share that GPU's array, which keeps the last call's contents (each
   build writes what it reads first). Calls that overlap on one GPU (different streams, or
   host threads without ordering) race and give undefined results: order them on one
   stream. Argument and error behaviour otherwise as tmfg_build. */
#define TMFG_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
tmfg_status tmfg_build_noalloc(const tmfg_job* job, uint32_t flags, hipStream_t stream);

/* ---- Batches: many independent builds in one graph replay ------------------------ */

/* Prepare `count` builds (the jobs' sizes and buffers are fixed from now on): allocates
   their scratch (tmfg_batch_footprint_bytes) and captures one hipGraph that runs every
   phase as one grouped launch over all instances, and the insertion loops as one
   persistent launch whose workgroups take instances largest first. Each instance gets the
   result tmfg_build would give it, bit for bit. Flags: TMFG_NO_VALIDATE,
   TMFG_BATCH_NO_GRAPH, TMFG_BATCH_AUTOTUNE, TMFG_RULE_PAPER, TMFG_RULE_CORR_PREFIX(p). */
tmfg_status tmfg_batch_create(tmfg_batch* batch, const tmfg_job* jobs, int32_t count, uint32_t flags);

/* Run (replay) the batch on `stream`; the inputs may change between runs, the buffers may
   not. Each job's *status receives its own tmfg_status. */
tmfg_status tmfg_batch_run(tmfg_batch batch, hipStream_t stream);

/* Release a batch (waits for the device). NULL is a no-op. */
tmfg_status tmfg_batch_destroy(tmfg_batch batch);

/* Launch configuration of a batch (with TMFG_BATCH_AUTOTUNE, the one the tuner chose by
   timing each knob on the batch's inputs at creation; those inputs must then be valid):
   [0..7] sort configuration index of each size class (-1: class absent), [8] rows per sort
   workgroup (0: one resident fill of the device), [9] persistent loop workgroups,
   [10] configurations timed, [11] milliseconds spent tuning, [12] walk rounds before a
   face is swept instead (64 untuned; 64, 16 or 8 tuned), [13] rows of the correlation
   GEMM's tile for instances with n < 1024 and [14] for the others (128 or 64; 0: no such
   instance, or no instance given as series), [15] 1 when the configuration came from the
   tuning cache instead of timing. The configuration never changes results.
   The tuner keeps its choices for the process and, when the environment variable
   TMFG_TUNE_CACHE names a writable file, in that file across processes, keyed by the
   device architecture and compute units, the HIP runtime version, the face rule and
   validation flags, and the batch's shape (instances per (log2 n, log2 L) bucket, counts
   rounded to a power of two); a later batch of the same key takes the stored choice. */
tmfg_status tmfg_batch_config(tmfg_batch batch, int32_t out[16]);

/* Apply a launch configuration in the layout of tmfg_batch_config ([10], [11], [15] are
   not read; entries of absent size classes and GEMM groups are not looked at). Each sort
   configuration must suit its class, [8] >= 0, 1 <= [9] <= the workgroups the device holds
   at once, 1 <= [12] <= 64, [13] and [14] 128 or 64. Waits for the device, then re-captures
   the batch's graph. TMFG_E_INVALID, with nothing changed, when a value is out of range;
   TMFG_E_HIP when the capture fails, with the previous configuration kept and the batch
   then launching its kernels directly. Results do not depend on the configuration. */
tmfg_status tmfg_batch_set_config(tmfg_batch batch, const int32_t cfg[16]);

/* Device bytes a batch over these jobs holds; 0 if a job is invalid. */
size_t tmfg_batch_footprint_bytes(const tmfg_job* jobs, int32_t count, uint32_t flags);

/* One-call form: builds (or reuses, when the job array is the same as the previous call's)
   a batch kept by the plan, and runs it on `stream`. The plan's n_max does not limit it;
   count above the plan's max_jobs gives TMFG_E_SIZE. */
tmfg_status tmfg_build_batch(tmfg_plan plan, const tmfg_job* jobs, int32_t count, hipStream_t stream);

/* ---- Serving: requests from host memory, continuous batching ---------------------- */
/* A server owns one device region (hbm_budget bytes) and one pinned host region
   (host_budget bytes), allocated at creation, and a scheduler thread. Requests wait in
   arrival order; each is admitted when its device footprint (input, scratch, results) and
   host footprint (staged input, results) fit in what is free. Whenever one of n_streams
   stream slots is idle, admitted requests (up to max_batch, grouped by size class unless
   TMFG_SERVER_FIFO) are dispatched there as one grouped batch (the kernels of
   tmfg_batch_run, launched directly), so a new batch starts while earlier ones still run.
   A request completes on its own, as soon as its build has finished, not with its batch:
   the workgroup that finishes a build copies its outputs into the request's range of the
   pinned region (allocated coherent) and then stores its status word there with a
   system-scope release; the scheduler reads the open requests' status words between its
   passes (every 20 us while work is in flight), finishes each published request and frees
   its device memory at once. A request's results stay in the pinned region until it is
   polled: requests that are never polled hold host memory and can stall admission. Every
   request gets the result tmfg_build gives it, bit for bit. submit, poll and stats may be
   called from any host thread.
   Each stream slot should have a hardware queue of its own. HIP gives a process
   GPU_MAX_HW_QUEUES queues (4 by default) and shares them among all of its streams, the
   caller's included; two slots on one queue run their dispatches one after the other,
   which raises latency under load. Keep n_streams within the queues the process's other
   streams leave free, or raise GPU_MAX_HW_QUEUES before the process first uses HIP. */
typedef struct tmfg_server_s* tmfg_server;

typedef struct {
  size_t hbm_budget;      /* device bytes for requests in flight */
  size_t host_budget;     /* pinned host bytes for staged inputs and unread results */
  int32_t max_batch;      /* requests one dispatch groups, at most (1..4096) */
  int32_t n_streams;      /* dispatches in flight at once (1..8), one stream each */
  int32_t n_max;          /* largest n accepted (4..20480) */
  int32_t L_max;          /* largest L accepted (>= 2) */
  uint32_t flags;         /* TMFG_SERVER_FIFO, a face rule (TMFG_SERVER_RULE_PAPER, or the plan
                             flags TMFG_RULE_PAPER or TMFG_RULE_CORR_PREFIX(p)), or 0 */
} tmfg_server_config;

/* Server flags. By default a dispatch takes the oldest waiting request and the waiting
   requests of the same size class (n in [4, 256), [256, 1024), [1024, 4096), [4096, ...)),
   so that small builds are not held up by the long serial chains of large ones; requests of
   other classes keep their order for the next idle slot. TMFG_SERVER_FIFO dispatches
   strictly in arrival order instead. TMFG_SERVER_RULE_PAPER builds every request with
   the paper's face rule (as TMFG_RULE_PAPER does for a plan). */
enum { TMFG_SERVER_FIFO = 1u << 0, TMFG_SERVER_RULE_PAPER = 1u << 1 };

/* Result of one request, filled by tmfg_server_poll. The array pointers are HOST buffers
   given by the caller (sizes as in tmfg_job for this n), or NULL to skip that output. */
typedef struct {
  int32_t* order;
  int32_t* edges;
  int32_t* steps;
  float* step_gain;
  int32_t* faces;
  int32_t n;              /* out */
  int32_t status;         /* out: tmfg_status of the build */
  int64_t arrival_ns;     /* out: server clock (tmfg_server_now_ns) */
  int64_t dispatch_ns;    /* out: when its batch was enqueued */
  int64_t done_ns;        /* out: when its results were in pinned memory */
} tmfg_server_result;

typedef struct {
  int64_t submitted, completed, dispatches, waiting;
  double p50_ms, p99_ms, mean_ms, max_ms;   /* latency done - arrival, completed requests */
  double builds_per_s;                      /* completed / (last done - first arrival) */
  double mean_batch;                        /* requests per dispatch */
} tmfg_server_report;

/* Allocates both regions, creates the stream slots and starts the scheduler thread on the
   current HIP device. */
tmfg_status tmfg_server_create(tmfg_server* server, const tmfg_server_config* config);

/* Queues one build of the n x L series at X_host (host memory, float32 row-major; copied
   before the call returns). arrival_ns is the request's arrival on the server clock, or 0
   for now. TMFG_E_SIZE if n or L is out of range or the request can never fit either
   budget. *ticket identifies the request in tmfg_server_poll. */
tmfg_status tmfg_server_submit(tmfg_server server, const float* X_host, int32_t n, int32_t L, int64_t arrival_ns,
                               int64_t* ticket);

/* Waits up to wait_ms milliseconds (negative: until done) for a request. Returns
   TMFG_PENDING if it has not finished; otherwise copies its results into `result`,
   returns TMFG_OK (the build's own status is result->status) and forgets the ticket.
   TMFG_E_INVALID for an unknown or already collected ticket. */
tmfg_status tmfg_server_poll(tmfg_server server, int64_t ticket, int32_t wait_ms, tmfg_server_result* result);

/* Counters and latency percentiles since creation or the last reset. */
tmfg_status tmfg_server_stats(tmfg_server server, tmfg_server_report* report, int32_t reset);

/* Stops the scheduler after the batches in flight finish, and frees both regions. NULL is
   a no-op. */
tmfg_status tmfg_server_destroy(tmfg_server server);

/* The server clock: monotonic nanoseconds. */
int64_t tmfg_server_now_ns(void);

/* ---- The stages of a build, callable on their own ------------------------------- */

/* Pearson similarity of n series of length L (paper, Section 5, Datasets):
   W[i][j] = <z_i, z_j> with z = (x - mean) / ||x - mean||, float32 via FP32 MFMA.
   W is bitwise symmetric with an exact 1.0f diagonal, clamped to [-1, 1], no -0.0.
   *status receives TMFG_OK, TMFG_E_NONFINITE or TMFG_E_DEGENERATE. */
tmfg_status tmfg_correlation(tmfg_plan plan, const float* X, int32_t n, int32_t L, float* W,
                             int32_t* status, hipStream_t stream);

/* Per-vertex order (Algorithm 1, sort of each row of S): idx[v*ld + k], k < n-1, is the
   k-th vertex u != v by (W[v][u] desc, u asc), as uint16; if vals is not NULL,
   vals[v*ld + k] = W[v][idx[v*ld + k]] as float32 (-0.0 written as +0.0). ld must be a
   multiple of 8 and at least n-1 rounded up to 8; idx and vals must be 16-byte aligned;
   entries n-1 up to the next multiple of 8 of each row are overwritten (idx 0xffff,
   vals -inf). Rows of more than 20480 entries are sorted in the plan's staging area as two
   halves (columns below n/2 and the rest), then merged. */
tmfg_status tmfg_sort_rows(tmfg_plan plan, const float* W, int32_t n, uint16_t* idx, float* vals,
                           int64_t ld, hipStream_t stream);

/* Seed (Algorithms 1 and 2, first comment): scores[v] = float64 sum of W[v][u] over
   u != v in index order; seed4 = the four largest by (score desc, id asc). W must be
   bitwise symmetric (column sums are used). */
tmfg_status tmfg_seed(tmfg_plan plan, const float* W, int32_t n, double* scores, int32_t* seed4,
                      hipStream_t stream);

/* Exact best vertex of each face (the per-face rule of Section 2 / Section 4.1's
   orig-tmfg): for face f with corners faces[3f..3f+2] (any order), best_u[f] = the
   vertex u with bit u clear in `inserted` (ceil(n/32) words, bit u of word u/32)
   maximising the float32 gain, lowest u on ties, and best_gain[f] its gain; -1 and
   -inf when every vertex is marked; -2 and NaN for a face with a corner outside [0, n),
   whose rows are not read. Reads three full rows of W per face. */
tmfg_status tmfg_face_sweep(tmfg_plan plan, const float* W, int32_t n, const int32_t* faces,
                            int32_t nfaces, const uint32_t* inserted, int32_t* best_u,
                            float* best_gain, hipStream_t stream);

/* ---- Clustering on the host ------------------------------------------------------ */

/* DBHT clustering of a finished TMFG (Section 2, Background: the directed bubble hierarchy
   tree; Section 5, Evaluation: the dendrogram cut into k clusters). Runs on the host; every
   pointer is HOST memory. Inputs: W (n x n, the float32 similarity the build used, bitwise
   symmetric) and the build's order, edges and steps, unchanged. k: clusters of the cut,
   1 <= k <= n. n_threads: host threads for the shortest paths (<= 0: all cores, at most 64).
   Outputs: labels[n] (clusters numbered by their smallest vertex), and optionally the
   dendrogram linkage[(n-1) x 4] (rows: smaller cluster id, larger id, distance, size; the
   vertices are clusters 0..n-1 and row m makes cluster n + m), group[n] (the converging
   bubble of each vertex) and bubble[n] (its bubble); bubble 0 is the seed clique and
   bubble s + 1 the clique of step s. Holds n x n doubles of shortest-path lengths while it
   runs (TMFG_E_NOMEM if that fails). TMFG_E_INVALID for a record with ids out of range.
   Readings where the paper leaves DBHT open:
   - edge length sqrt(2 (1 - W[i][j])) (0 if W > 1), Dijkstra path sums from the source,
     and the distance of a pair is the sum from its smaller id;
   - bubble s + 1's parent is the bubble that made the face step s split (the seed's faces:
     bubble 0), and that face is their separating triangle;
   - a tree edge points to the side, child (the vertices inserted in the child's subtree) or
     parent (the other vertices off the triangle), whose TMFG edges to the triangle have the
     strictly larger W sum (float64, triangle vertex ascending, then neighbour ascending);
     a tie points to the parent;
   - converging bubbles have no outgoing edge; a vertex's group is, of the converging bubbles
     reachable from the bubbles containing it, the one its TMFG edges weigh most (sum of W to
     the bubble's other vertices, ascending), ties to the lowest id; its bubble is, of the
     bubbles containing it that reach its group, the one of least summed path length to the
     bubble's four vertices, ties to the lowest id;
   - complete linkage (largest member-pair path length; the closest pair first, ties to the
     lowest (smaller id, larger id)) joins each (group, bubble) cell, then the cells of each
     group, then the groups, cells and groups in ascending bubble-id order; the cut undoes
     the last k - 1 merges of that sequence. */
tmfg_status tmfg_dbht(int32_t n, const float* W, const int32_t* order, const int32_t* edges,
                      const int32_t* steps, int32_t k, int32_t n_threads, int32_t* labels,
                      double* linkage, int32_t* group, int32_t* bubble);

/* ---- Diagnostics ------------------------------------------------------------------ */

const char* tmfg_status_string(tmfg_status s);
int tmfg_last_hip_error(void);

/* Latency of one dependent trip to memory from one wave, in nanoseconds: the floor of a
   chain of loads each of whose addresses is the value of the one before, as in the
   insertion loop (a list entry names the similarity read next). The call allocates a
   buffer of about `bytes` bytes (rounded down to a power of two of 128-byte lines, at
   least 64 lines, at most 16 GiB), links its lines into one cycle in a scattered order,
   and times `steps` (1..2^24) trips of one wave: with lanes == 1 every lane reads the same
   line (one line per trip), with lanes == 64 each lane follows its own stretch of the
   cycle (64 lines per trip, a gather). A buffer of at most 2 MiB (half of one L2) is read
   once untimed by the same wave, so the timed pass gives the L2 latency; a larger one is
   timed cold, and one of several GiB, of which each line is read at most once, gives the
   HBM latency. Synchronous, on the current device; frees what it allocates. */
tmfg_status tmfg_probe_load_latency(int64_t bytes, int32_t lanes, int32_t steps, double* ns_per_trip);

#ifdef __cplusplus
}
#endif

#endif /* TMFG_H_ */
