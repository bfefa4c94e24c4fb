// Host-side launch wrappers of the TMFG kernels (internal to libtmfg).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

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
hipError_t launch_sort_rows(const float* W, int n, uint16_t* idx, float* vals, int64_t ldi, hipStream_t s);
int64_t sort_row_stride(int n);

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
  int32_t* stats;          // optional, 16 counters (see tmfg_plan_stats)
};
hipError_t launch_loop(const LoopParams& p, hipStream_t s);
size_t loop_lds_bytes(int n);

}  // namespace tmfg
