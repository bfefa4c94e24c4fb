// Device helpers shared by the insertion loops (internal to libtmfg): the inserted-vertex
// bitmap, candidate keys, row and wave reductions, the seed choice, the paper's face pair,
// and the 16-byte face record.
#pragma once
#include "common.h"

namespace tmfg {
namespace {

constexpr int kGroup = 16;                       // lanes per face walk

__device__ __forceinline__ bool is_ins(const uint32_t* bits, int u) { return (bits[u >> 5] >> (u & 31)) & 1u; }

// 1 when list entry u at position p, lo <= p < hi, is an uninserted vertex (u >= n: no). The
// bitmap word is read whatever the position, and the tests are combined without short
// circuits, so that the reads of many entries are in flight together instead of one trip
// through the LDS each.
__device__ __forceinline__ uint32_t open_entry(const uint32_t* bits, int u, int n, int p, int lo, int hi) {
  const int uc = u < n ? u : 0;
  const uint32_t w = bits[uc >> 5];
  return (uint32_t)(p >= lo) & (uint32_t)(p < hi) & (uint32_t)(u < n) & ~(w >> (uc & 31)) & 1u;
}

// The same for the 8 ids of one 16-byte load (entry j at position q0 + j): bit j of the result.
// The eight bitmap words are read before any is used (a scheduling barrier keeps them
// together), so they cost one trip through the LDS instead of eight.
__device__ __forceinline__ uint32_t open_mask8(const uint32_t* bits, uint4 w8, int n, int q0, int lo, int hi) {
  const uint32_t wd[4] = {w8.x, w8.y, w8.z, w8.w};
  int u[8];
  uint32_t bw[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    u[j] = (int)((wd[j >> 1] >> (16 * (j & 1))) & 0xffffu);
    bw[j] = bits[(u[j] < n ? u[j] : 0) >> 5];
  }
  __builtin_amdgcn_sched_barrier(0);
  uint32_t mask = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int p = q0 + j;
    mask |= ((uint32_t)(p >= lo) & (uint32_t)(p < hi) & (uint32_t)(u[j] < n) & ~(bw[j] >> (u[j] & 31)) & 1u) << j;
  }
  return mask;
}

__device__ __forceinline__ uint64_t cand_key(float g, int u) {
  return ((uint64_t)ord_f32(g) << 32) | (uint32_t)(0xffff - u);
}

__device__ __forceinline__ void sort3(int& x, int& y, int& z) {
  int t;
  if (x > y) { t = x; x = y; y = t; }
  if (y > z) { t = y; y = z; z = t; }
  if (x > y) { t = x; x = y; y = t; }
}

// Reductions inside a 16-lane row (one walk group) with DPP lane permutations, which run at
// ALU latency instead of a trip through the LDS crossbar: pairs (quad_perm 1,0,3,2), quads
// (quad_perm 2,3,0,1), half rows (row_half_mirror) and the whole row (row_mirror); every
// lane of the row ends with the result. All lanes of the row must be active.
constexpr int kDppXor1 = 0xB1;
constexpr int kDppXor2 = 0x4E;
constexpr int kDppHalfMirror = 0x141;
constexpr int kDppMirror = 0x140;
static_assert(kGroup == 16, "a walk group is one DPP row");

template <int CTRL>
__device__ __forceinline__ uint32_t dpp32(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, 0xf, 0xf, false);
}
template <int CTRL>
__device__ __forceinline__ uint64_t dpp64(uint64_t v) {
  return ((uint64_t)dpp32<CTRL>((uint32_t)(v >> 32)) << 32) | dpp32<CTRL>((uint32_t)v);
}
__device__ __forceinline__ uint64_t max64(uint64_t a, uint64_t b) { return a > b ? a : b; }

// The same over groups of G = 4, 8 or 16 lanes (quads, half rows, rows). A 64-bit maximum
// is taken as two 32-bit ones: the high words, then the low words of the lanes whose high
// word is that maximum (0, the identity, elsewhere); each step is one DPP max.
template <int G>
__device__ __forceinline__ uint32_t group_max_u32(uint32_t x) {
  static_assert(G == 4 || G == 8 || G == 16, "a group is a quad, a half row or a row");
  x = max(x, dpp32<kDppXor1>(x));
  x = max(x, dpp32<kDppXor2>(x));
  if (G >= 8) x = max(x, dpp32<kDppHalfMirror>(x));
  if (G >= 16) x = max(x, dpp32<kDppMirror>(x));
  return x;
}
template <int G>
__device__ __forceinline__ uint64_t group_max_u64(uint64_t v) {
  const uint32_t vh = (uint32_t)(v >> 32);
  const uint32_t hi = group_max_u32<G>(vh);
  const uint32_t lo = group_max_u32<G>(vh == hi ? (uint32_t)v : 0u);
  return ((uint64_t)hi << 32) | lo;
}
template <int G>
__device__ __forceinline__ int group_min_i32(int x) {
  static_assert(G == 4 || G == 8 || G == 16, "a group is a quad, a half row or a row");
  x = min(x, (int)dpp32<kDppXor1>((uint32_t)x));
  x = min(x, (int)dpp32<kDppXor2>((uint32_t)x));
  if (G >= 8) x = min(x, (int)dpp32<kDppHalfMirror>((uint32_t)x));
  if (G >= 16) x = min(x, (int)dpp32<kDppMirror>((uint32_t)x));
  return x;
}
// The value of lane 15 of each 16-lane row, in every lane of the row (DPP row_newbcast:15,
// which the compiler's DPP builtin does not accept for this target). The compiler does not
// see the DPP read inside the asm, so the asm provides the two wait states a DPP read of a
// VGPR that a VALU instruction has just written needs.
__device__ __forceinline__ uint32_t row_last_u32(uint32_t x) {
  uint32_t r;
  asm("s_nop 1\n\tv_mov_b32_dpp %0, %1 row_newbcast:15 row_mask:0xf bank_mask:0xf" : "=v"(r) : "v"(x));
  return r;
}
// Inclusive prefix sum inside each 16-lane row (row_shr by 1, 2, 4, 8; lanes shifted in from
// outside the row contribute 0).
__device__ __forceinline__ uint32_t row_scan_u32(uint32_t x) {
  x += dpp32<0x111>(x);
  x += dpp32<0x112>(x);
  x += dpp32<0x114>(x);
  x += dpp32<0x118>(x);
  return x;
}
__device__ __forceinline__ int group_sum_i32(int x) {
  x += (int)dpp32<kDppXor1>((uint32_t)x);
  x += (int)dpp32<kDppXor2>((uint32_t)x);
  x += (int)dpp32<kDppHalfMirror>((uint32_t)x);
  x += (int)dpp32<kDppMirror>((uint32_t)x);
  return x;
}
__device__ __forceinline__ uint64_t group_max_u64(uint64_t v) { return group_max_u64<kGroup>(v); }
__device__ __forceinline__ int group_min_i32(int x) { return group_min_i32<kGroup>(x); }

// Wave-wide maximum: row maxima by DPP, then the four rows read out lane by lane; for 64
// bits, the high words first, then the low words of the lanes that hold the high maximum.
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t x) {
  x = group_max_u32<16>(x);
  uint32_t m = (uint32_t)__builtin_amdgcn_readlane((int)x, 0);
#pragma unroll
  for (int r = 1; r < 4; ++r) m = max(m, (uint32_t)__builtin_amdgcn_readlane((int)x, 16 * r));
  return m;
}
__device__ __forceinline__ int wave_min_i32(int x) {
  x = group_min_i32<16>(x);
  int m = __builtin_amdgcn_readlane(x, 0);
#pragma unroll
  for (int r = 1; r < 4; ++r) m = min(m, __builtin_amdgcn_readlane(x, 16 * r));
  return m;
}
__device__ __forceinline__ uint64_t wave_max_dpp(uint64_t v) {
  const uint32_t vh = (uint32_t)(v >> 32);
  const uint32_t hi = wave_max_u32(vh);
  const uint32_t lo = wave_max_u32(vh == hi ? (uint32_t)v : 0u);
  return ((uint64_t)hi << 32) | lo;
}

// Seed (Algorithm 1 and Algorithm 2, first comment): the four vertices of largest score,
// ties to the lower id, in rank order, into s_seed[0..3]. The whole workgroup of BLOCK
// threads takes part; s_part and s_vpart hold one entry per wave.
template <int BLOCK>
__device__ __forceinline__ void seed_top4(const double* scores, int n, int* s_seed, uint64_t* s_part, int* s_vpart) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int r = 0; r < 4; ++r) {
    uint64_t bk = 0;
    int bv = 0x7fffffff;
    for (int v = tid; v < n; v += BLOCK) {
      bool taken = false;
      for (int q = 0; q < r; ++q) taken |= (s_seed[q] == v);
      if (taken) continue;
      const uint64_t k = ord_f64(scores[v]);
      if (k > bk || (k == bk && v < bv)) {
        bk = k;
        bv = v;
      }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      const uint64_t ok = ((uint64_t)__shfl_xor((uint32_t)(bk >> 32), off, kWave) << 32) |
                          __shfl_xor((uint32_t)bk, off, kWave);
      const int ov = __shfl_xor(bv, off, kWave);
      if (ok > bk || (ok == bk && ov < bv)) {
        bk = ok;
        bv = ov;
      }
    }
    if (lane == 0) {
      s_part[wave] = bk;
      s_vpart[wave] = bv;
    }
    __syncthreads();
    if (tid == 0) {
      uint64_t k = s_part[0];
      int v = s_vpart[0];
      for (int w = 1; w < BLOCK / kWave; ++w)
        if (s_part[w] > k || (s_part[w] == k && s_vpart[w] < v)) {
          k = s_part[w];
          v = s_vpart[w];
        }
      s_seed[r] = v;
    }
    __syncthreads();
  }
}

// The paper's pair of one face (Section 4.1, Algorithm 2), by a group of G lanes (gl = lane
// within the group): the candidates are the MaxCorrs of the three corners, each the first
// uninserted entry of the corner's sorted row, found from the corner's cached position
// G * 8 * L entries at a time (L 16-byte loads of 8 ids per lane and corner, bitmap only);
// the pair is the candidate of largest gain, ties to the lowest id (a vertex that is MaxCorrs
// of two corners is evaluated twice, to the same key). Moves the corners' cached positions
// forward. 0 when no vertex is left. Rows hold m entries (n - 1, fewer once compacted).
template <int G = kGroup, int L = 1>
__device__ __forceinline__ uint64_t paper_face(const float* W, const uint16_t* idx, int n, int m, int ldi,
                                               const uint32_t* bits, uint16_t* ptr, int a, int b, int c, int gl,
                                               int* scans) {
  const int x3[3] = {a, b, c};
  int pos[3], cand[3];
  bool open[3];
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    // every entry before it is inserted; the group agrees on one value even if another
    // group moves the position meanwhile
    pos[t] = group_min_i32<G>((int)ptr[x3[t]]);
    cand[t] = -1;
    open[t] = pos[t] < m;
  }
  int trips = 0;
  while (open[0] || open[1] || open[2]) {
    uint4 sv[3][L];
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      const int qs = (pos[t] & ~7) + gl * 8 * L;
#pragma unroll
      for (int l = 0; l < L; ++l)
        sv[t][l] = *(const uint4*)(idx + (size_t)x3[t] * ldi + min(qs + 8 * l, ldi - 8));
    }
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      if (!open[t]) continue;
      const int qs = (pos[t] & ~7) + gl * 8 * L;
      int fp = 0x7fffffff;          // (position << 16) | id of the first uninserted entry
#pragma unroll
      for (int l = 0; l < L; ++l) {
        const uint32_t mk = open_mask8(bits, sv[t][l], n, qs + 8 * l, pos[t], m);
        const uint32_t wd[4] = {sv[t][l].x, sv[t][l].y, sv[t][l].z, sv[t][l].w};
        const int j = (int)__builtin_ctz(mk | 0x100u);
        int u = 0;                  // the id of entry j (selects over constant indices)
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) u = j == jj ? (int)((wd[jj >> 1] >> (16 * (jj & 1))) & 0xffffu) : u;
        fp = mk ? min(fp, ((qs + 8 * l + j) << 16) | u) : fp;
      }
      const int f = group_min_i32<G>(fp);
      if (f != 0x7fffffff) {
        pos[t] = f >> 16;
        cand[t] = f & 0xffff;
        open[t] = false;
      } else {
        pos[t] = min((pos[t] & ~7) + G * 8 * L, m);
        open[t] = pos[t] < m;
      }
    }
    ++trips;
  }
  if (gl == 0) {
#pragma unroll
    for (int t = 0; t < 3; ++t)
      if (pos[t] > (int)ptr[x3[t]]) ptr[x3[t]] = (uint16_t)pos[t];
  }
  // lane t < 3 evaluates the candidate of corner t, all three similarities from W
  const int t = gl < 3 ? gl : 0;
  const int u = t == 0 ? cand[0] : t == 1 ? cand[1] : cand[2];
  const int uc = u >= 0 ? u : 0;
  const float wa = W[(size_t)a * n + uc], wb = W[(size_t)b * n + uc], wc = W[(size_t)c * n + uc];
  const uint64_t k = (gl < 3 && u >= 0) ? cand_key((wa + wb) + wc, u) : 0;
  *scans += trips;
  return group_max_u64<G>(k);
}

// Copies a finished build's outputs (n vertices; none but the status when st is not TMFG_OK)
// to the host copies in h, then stores the status there with a system-scope release, so a
// host thread that reads the status while the launch still runs finds the outputs complete.
// The whole workgroup calls it, after its last output store.
__device__ __forceinline__ void publish_outputs(const HostOut& h, const int32_t* order, const int32_t* edges,
                                                const int32_t* steps, const float* step_gain, const int32_t* faces,
                                                int n, int32_t st) {
  // every wave's output stores are complete and visible across the device before any is read
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  if (st == 0) {
    const int nt = (int)blockDim.x, t = (int)threadIdx.x;
    for (int i = t; i < n; i += nt) h.order[i] = order[i];
    for (int i = t; i < 2 * (3 * n - 6); i += nt) h.edges[i] = edges[i];
    for (int i = t; i < 4 * (n - 4); i += nt) h.steps[i] = steps[i];
    for (int i = t; i < n - 4; i += nt) h.step_gain[i] = step_gain[i];
    for (int i = t; i < 3 * (2 * n - 4); i += nt) h.faces[i] = faces[i];
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");            // system scope
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(h.status, st, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

__device__ __forceinline__ uint64_t rec_key(const uint4& r) { return ((uint64_t)r.x << 32) | r.y; }
__device__ __forceinline__ int rec_face(const uint4& r) { return 0xffff - (int)(r.y >> 16); }
__device__ __forceinline__ int rec_vertex(const uint4& r) { return (int)(r.y & 0xffffu); }

// A face record: {ord(gain), (0xffff - face) << 16 | vertex, a | b << 16, c}. Its first two
// words, read as one 64-bit key, order records by (gain desc, face id asc); 0 means no pair.
__device__ __forceinline__ uint4 face_record(int f, int a, int b, int c, uint64_t best) {
  uint4 rec;
  rec.x = (uint32_t)(best >> 32);
  rec.y = best ? ((uint32_t)(0xffff - f) << 16) | (0xffffu - (uint32_t)(best & 0xffffu)) : 0u;
  rec.z = (uint32_t)a | ((uint32_t)b << 16);
  rec.w = (uint32_t)c;
  return rec;
}

}  // namespace
}  // namespace tmfg
