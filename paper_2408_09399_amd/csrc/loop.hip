// TMFG insertion loop: one persistent workgroup runs the whole serial chain of n-4
// insertions on the device.
//
// Method (paper, Section 2 and Section 4): start from the seed 4-clique and its 4 faces;
// repeatedly join the uninserted vertex u and face f of largest gain
//     gain(f, u) = (W[a][u] + W[b][u]) + W[c][u],   f = {a < b < c},   float32
// (ties: lowest face id, then lowest vertex id), emit edges (u,a), (u,b), (u,c), and replace
// f by {u,a,b} (keeps id f), {u,b,c} (id F), {u,a,c} (id F+1).
//
// Each face keeps a cached best pair. Removing vertices never raises a face's best gain,
// so a cached pair whose vertex is still uninserted is exact and one whose vertex has been
// inserted ("stale") is an upper bound. As in the paper's heap-based variant (Section 4.2)
// stale pairs are recomputed lazily, only when they could decide the next insertion. The
// global maximum is tracked with a two-level structure instead of a heap: face records in
// global memory (16 B each), and per 64-face chunk the maximum record in LDS; wave 0 scans
// the chunk maxima. If the top record is fresh it is inserted; otherwise every stale chunk
// maximum ranked above the best fresh one (up to one per wave) is recomputed in parallel.
//
// Best vertex of a face (one wave): the threshold walk over the three corners' sorted rows
// (the per-vertex sort of Algorithm 1). Each round reads the next 64 entries of each list,
// skipping inserted vertices (the first uninserted position per vertex is cached in LDS:
// the paper's MaxCorrs), and evaluates every uninserted candidate exactly. Any vertex not
// yet seen has W[x][u] <= the value at the last position read from x's list, for x = a, b,
// c, so its gain is at most T = (A + B) + C of those three values (float32 addition is
// monotone). The walk stops when the best gain seen is strictly above T, or a list is
// exhausted. A walk that needs more than kMaxRounds rounds is finished by a sweep of the
// three full rows by the whole workgroup. Both give the exact best pair.
#include "common.h"
#include "internal.h"

namespace tmfg {

namespace {
constexpr int kBlock = 1024;
constexpr int kWaves = kBlock / kWave;
constexpr int kMaxRounds = 8;

struct Work {
  int f;            // face id
  int a, b, c;      // corners, ascending
  uint64_t best;    // (ord(gain) << 32) | (0xffff - u), 0 when no candidate
  int sweep;        // 1 when the walk gave up and a full sweep is needed
};

__device__ __forceinline__ bool is_ins(const uint32_t* bits, int u) { return (bits[u >> 5] >> (u & 31)) & 1u; }

__device__ __forceinline__ uint64_t cand_key(float g, int u) {
  return ((uint64_t)ord_f32(g) << 32) | (uint32_t)(0xffff - u);
}

__device__ __forceinline__ void sort3(int& x, int& y, int& z) {
  int t;
  if (x > y) { t = x; x = y; y = t; }
  if (y > z) { t = y; y = z; z = t; }
  if (x > y) { t = x; x = y; y = t; }
}

// Threshold walk for one face by one wave. Returns false when it ran out of rounds.
__device__ bool walk_face(const LoopParams& P, const uint32_t* bits, uint16_t* ptr, int a, int b, int c,
                          uint64_t& best_out, int lane, int* rounds) {
  const int n = P.n, m = n - 1;
  const float* Wa = P.W + (size_t)a * n;
  const float* Wb = P.W + (size_t)b * n;
  const float* Wc = P.W + (size_t)c * n;
  const int x3[3] = {a, b, c};
  int p[3];
  bool skip[3];
  int np[3];
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    p[t] = ptr[x3[t]];
    skip[t] = true;
    np[t] = p[t];
  }
  uint64_t best = 0;
  bool done = false;
  int r = 0;
  for (; r < kMaxRounds && !done; ++r) {
    int id[3];
    bool ok[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      const int pos = p[t] + r * kWave + lane;
      id[t] = pos < m ? (int)P.idx[(size_t)x3[t] * P.ldi + pos] : -1;
      ok[t] = id[t] >= 0 && !is_ins(bits, id[t]);
    }
    // gains of uninserted candidates, plus the value at the last position of each list
    float g[3], last[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      g[t] = 0.0f;
      if (ok[t]) {
        const int u = id[t];
        g[t] = (Wa[u] + Wb[u]) + Wc[u];
      }
      const int u63 = __shfl(id[t], 63, kWave);
      last[t] = u63 >= 0 ? P.W[(size_t)x3[t] * n + u63] : -INFINITY;
    }
    uint64_t k = 0;
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      if (ok[t]) {
        const uint64_t kt = cand_key(g[t], id[t]);
        k = kt > k ? kt : k;
      }
      if (skip[t]) {
        const uint64_t msk = __ballot(ok[t]);
        if (msk) {
          skip[t] = false;
          np[t] = p[t] + r * kWave + (int)__builtin_ctzll(msk);
        } else {
          np[t] = min(p[t] + (r + 1) * kWave, m);
        }
      }
    }
    k = wave_max_u64(k);
    best = k > best ? k : best;
    const bool exhausted = p[0] + (r + 1) * kWave >= m || p[1] + (r + 1) * kWave >= m ||
                           p[2] + (r + 1) * kWave >= m;
    const float T = (last[0] + last[1]) + last[2];
    done = exhausted || (best != 0 && (uint32_t)(best >> 32) > ord_f32(T));
  }
  if (lane == 0) {
#pragma unroll
    for (int t = 0; t < 3; ++t)
      if (np[t] > p[t]) ptr[x3[t]] = (uint16_t)np[t];
  }
  *rounds += r;
  best_out = best;
  return done;
}

__device__ __forceinline__ uint64_t rec_key(const uint4& r) { return ((uint64_t)r.x << 32) | r.y; }

}  // namespace

// ---------------------------------------------------------------------------------------
// Bulk exact best vertex of many faces by sweeping their three rows (one workgroup per
// face). Reads 12n bytes of W plus the n-bit inserted set per face.
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void face_sweep_kernel(const float* __restrict__ W, int n,
                                                         const int32_t* __restrict__ faces, int nfaces,
                                                         const uint32_t* __restrict__ inserted,
                                                         int32_t* __restrict__ best_u,
                                                         float* __restrict__ best_gain) {
  __shared__ uint64_t part[4];
  const int f = blockIdx.x;
  if (f >= nfaces) return;
  int a = faces[3 * f], b = faces[3 * f + 1], c = faces[3 * f + 2];
  sort3(a, b, c);
  const float* Wa = W + (size_t)a * n;
  const float* Wb = W + (size_t)b * n;
  const float* Wc = W + (size_t)c * n;
  uint64_t best = 0;
  for (int u = threadIdx.x; u < n; u += 256) {
    const float wa = Wa[u], wb = Wb[u], wc = Wc[u];
    if (!((inserted[u >> 5] >> (u & 31)) & 1u)) {
      const uint64_t k = cand_key((wa + wb) + wc, u);
      best = k > best ? k : best;
    }
  }
  best = wave_max_u64(best);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t k = part[0];
    for (int w = 1; w < 4; ++w) k = part[w] > k ? part[w] : k;
    best_u[f] = k ? 0xffff - (int)(k & 0xffffffffu) : -1;
    best_gain[f] = k ? unord_f32((uint32_t)(k >> 32)) : -INFINITY;
  }
}

hipError_t launch_face_sweep(const float* W, int n, const int32_t* faces, int nfaces, const uint32_t* inserted,
                             int32_t* best_u, float* best_gain, hipStream_t s) {
  if (nfaces <= 0) return hipSuccess;
  hipLaunchKernelGGL(face_sweep_kernel, dim3(nfaces), dim3(256), 0, s, W, n, faces, nfaces, inserted, best_u,
                     best_gain);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// The insertion loop.
// ---------------------------------------------------------------------------------------
namespace {
struct LdsLayout {
  int nw, nchunk;
  size_t off_bits, off_ptr, off_cmax, total;
};
__host__ __device__ inline LdsLayout lds_layout(int n) {
  LdsLayout L;
  L.nw = (n + 31) / 32;
  const int nf = 2 * n - 4;
  L.nchunk = (nf + 63) / 64;
  L.off_cmax = 0;                                           // uint4[nchunk]
  L.off_bits = L.off_cmax + (size_t)L.nchunk * 16;          // uint32[nw]
  L.off_ptr = L.off_bits + (size_t)L.nw * 4;                // uint16[n]
  L.total = L.off_ptr + ((size_t)n * 2 + 15) / 16 * 16;
  return L;
}
}  // namespace

__global__ __launch_bounds__(kBlock) void tmfg_loop_kernel(LoopParams P) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  __shared__ Work work[kWaves];
  __shared__ int s_nwork, s_ins, s_F, s_stop, s_seed[4];
  __shared__ uint64_t s_part[kWaves];
  __shared__ int s_vpart[kWaves];

  const int n = P.n;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const LdsLayout LL = lds_layout(n);
  uint4* cmax = (uint4*)(smem + LL.off_cmax);
  uint32_t* bits = (uint32_t*)(smem + LL.off_bits);
  uint16_t* ptr = (uint16_t*)(smem + LL.off_ptr);
  const int nf = 2 * n - 4;

  // Errors raised by the kernels that produced W stop the build here.
  const uint32_t fl = *P.flags;
  if (fl) {
    if (tid == 0) {
      *P.status = (fl & kFlagNonFinite) ? 3 : (fl & kFlagAsymmetric) ? 4 : (fl & kFlagDegenerate) ? 5 : 8;
    }
    return;
  }

  for (int i = tid; i < nf; i += kBlock) P.frec[i] = make_uint4(0, 0, 0, 0);
  for (int i = tid; i < LL.nchunk; i += kBlock) cmax[i] = make_uint4(0, 0, 0, 0);
  for (int i = tid; i < LL.nw; i += kBlock) bits[i] = 0;
  for (int i = tid; i < n; i += kBlock) ptr[i] = 0;

  // Seed: top-4 by (score desc, id asc).
  for (int r = 0; r < 4; ++r) {
    uint64_t bk = 0;
    int bv = 0x7fffffff;
    for (int v = tid; v < n; v += kBlock) {
      bool taken = false;
      for (int q = 0; q < r; ++q) taken |= (s_seed[q] == v);
      if (taken) continue;
      const uint64_t k = ord_f64(P.scores[v]);
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
      for (int w = 1; w < kWaves; ++w)
        if (s_part[w] > k || (s_part[w] == k && s_vpart[w] < v)) {
          k = s_part[w];
          v = s_vpart[w];
        }
      s_seed[r] = v;
    }
    __syncthreads();
  }
  if (tid == 0) {
    const int v1 = s_seed[0], v2 = s_seed[1], v3 = s_seed[2], v4 = s_seed[3];
    P.order[0] = v1; P.order[1] = v2; P.order[2] = v3; P.order[3] = v4;
    const int e[12] = {v1, v2, v1, v3, v1, v4, v2, v3, v2, v4, v3, v4};
    for (int i = 0; i < 12; ++i) P.edges[i] = e[i];
    for (int q = 0; q < 4; ++q) bits[s_seed[q] >> 5] |= 1u << (s_seed[q] & 31);
    const int tri[4][3] = {{v1, v2, v3}, {v1, v2, v4}, {v1, v3, v4}, {v2, v3, v4}};
    for (int f = 0; f < 4; ++f) {
      int x = tri[f][0], y = tri[f][1], z = tri[f][2];
      sort3(x, y, z);
      work[f].f = f; work[f].a = x; work[f].b = y; work[f].c = z;
      work[f].best = 0; work[f].sweep = 0;
    }
    s_nwork = 4;
    s_ins = 4;
    s_F = 4;
    s_stop = 0;
  }
  __syncthreads();

  int walk_rounds = 0, stale_recomputes = 0, sweeps = 0, phases = 0, since_insert = 0;
  for (;;) {
    const int nwork = s_nwork;
    const bool have_cand = s_ins < n;
    // Phase B: best pair of every face in the work list, one wave per face.
    if (wave < nwork) {
      Work& w = work[wave];
      uint64_t best = 0;
      bool ok = true;
      if (have_cand) ok = walk_face(P, bits, ptr, w.a, w.b, w.c, best, lane, &walk_rounds);
      if (lane == 0) {
        w.best = best;
        w.sweep = ok ? 0 : 1;
      }
    }
    __syncthreads();
    // Phase B2: faces whose walk gave up are swept by the whole workgroup, one at a time.
    for (int q = 0; q < nwork; ++q) {
      if (!work[q].sweep) continue;
      const int a = work[q].a, b = work[q].b, c = work[q].c;
      const float* Wa = P.W + (size_t)a * n;
      const float* Wb = P.W + (size_t)b * n;
      const float* Wc = P.W + (size_t)c * n;
      uint64_t best = 0;
      for (int u = tid; u < n; u += kBlock) {
        if (!is_ins(bits, u)) {
          const uint64_t k = cand_key((Wa[u] + Wb[u]) + Wc[u], u);
          best = k > best ? k : best;
        }
      }
      best = wave_max_u64(best);
      if (lane == 0) s_part[wave] = best;
      __syncthreads();
      if (tid == 0) {
        uint64_t k = s_part[0];
        for (int w = 1; w < kWaves; ++w) k = s_part[w] > k ? s_part[w] : k;
        work[q].best = k;
        work[q].sweep = 0;
        ++sweeps;
      }
      __syncthreads();
    }
    // Phase B3: publish the new face records.
    if (tid < nwork) {
      const Work& w = work[tid];
      const uint64_t k = w.best;                          // low 16 bits: 0xffff - u
      uint4 rec;
      rec.x = (uint32_t)(k >> 32);
      // key word: face id (inverted, so a lower id ranks higher) and the vertex; a face
      // with no candidate left (after the last insertion) gets an all-zero key
      rec.y = k ? ((uint32_t)(0xffff - w.f) << 16) | (0xffffu - (uint32_t)(k & 0xffffu)) : 0u;
      rec.z = (uint32_t)w.a | ((uint32_t)w.b << 16);
      rec.w = (uint32_t)w.c;
      P.frec[w.f] = rec;
    }
    __threadfence_block();
    __syncthreads();
    // Phase C: refresh the chunk maxima of the chunks touched this phase.
    if (wave < nwork) {
      const int ch = work[wave].f >> 6;
      bool first = true;
      for (int q = 0; q < wave; ++q) first &= (work[q].f >> 6) != ch;
      if (first) {
        const int f = ch * 64 + lane;
        const uint4 r = f < nf ? P.frec[f] : make_uint4(0, 0, 0, 0);
        const uint64_t k = rec_key(r);
        const uint64_t mx = wave_max_u64(k);
        const uint64_t msk = __ballot(k == mx);
        if (lane == (int)__builtin_ctzll(msk)) cmax[ch] = r;
      }
    }
    __syncthreads();
    if (s_ins >= n || s_stop) break;
    // Phase A: select (wave 0).
    ++phases;
    if (wave == 0) {
      uint64_t k1 = 0, kf = 0;
      for (int ch = lane; ch < LL.nchunk; ch += kWave) {
        const uint4 r = cmax[ch];
        const uint64_t k = rec_key(r);
        if (!k) continue;
        k1 = k > k1 ? k : k1;
        const int u = (int)(r.y & 0xffffu);
        if (!is_ins(bits, u)) kf = k > kf ? k : kf;
      }
      k1 = wave_max_u64(k1);
      kf = wave_max_u64(kf);
      const int f1 = 0xffff - (int)((uint32_t)k1 >> 16);
      if (k1 != 0 && k1 == kf) {
        // Fresh maximum: insert.
        if (lane == 0) {
          const uint4 r = cmax[f1 >> 6];
          const int u = (int)(r.y & 0xffffu);
          const int x = (int)(r.z & 0xffffu), y = (int)(r.z >> 16), z = (int)r.w;
          const int ins = s_ins, st = ins - 4, F = s_F;
          P.order[ins] = u;
          int32_t* e = P.edges + 2 * (6 + 3 * st);
          e[0] = u; e[1] = x; e[2] = u; e[3] = y; e[4] = u; e[5] = z;
          int32_t* sp = P.steps + 4 * st;
          sp[0] = f1; sp[1] = x; sp[2] = y; sp[3] = z;
          P.step_gain[st] = unord_f32(r.x);
          bits[u >> 5] |= 1u << (u & 31);
          int t0 = u, t1 = x, t2 = y;
          sort3(t0, t1, t2);
          work[0] = Work{f1, t0, t1, t2, 0, 0};
          t0 = u; t1 = y; t2 = z;
          sort3(t0, t1, t2);
          work[1] = Work{F, t0, t1, t2, 0, 0};
          t0 = u; t1 = x; t2 = z;
          sort3(t0, t1, t2);
          work[2] = Work{F + 1, t0, t1, t2, 0, 0};
          s_nwork = 3;
          s_ins = ins + 1;
          s_F = F + 2;
        }
        since_insert = 0;
      } else if (k1 == 0) {
        if (lane == 0) {
          *P.status = 8;
          s_stop = 1;
          s_nwork = 0;
        }
      } else {
        // Stale maximum: recompute every stale chunk maximum ranked above the best fresh
        // record (the top one first), up to one per wave.
        if (++since_insert > nf + 8) {
          if (lane == 0) {
            *P.status = 8;
            s_stop = 1;
            s_nwork = 0;
          }
        } else {
          if (lane == 0) {
            const uint4 r = cmax[f1 >> 6];
            work[0] = Work{f1, (int)(r.z & 0xffffu), (int)(r.z >> 16), (int)r.w, 0, 0};
          }
          int cnt = 1;
          for (int ch0 = 0; ch0 < LL.nchunk; ch0 += kWave) {
            const int ch = ch0 + lane;
            bool pick = false;
            uint4 r = make_uint4(0, 0, 0, 0);
            if (ch < LL.nchunk) {
              r = cmax[ch];
              const uint64_t k = rec_key(r);
              const int u = (int)(r.y & 0xffffu);
              pick = k > kf && k != k1 && is_ins(bits, u);
            }
            const uint64_t msk = __ballot(pick);
            if (pick) {
              const int slot = cnt + (int)__popcll(msk & ((1ull << lane) - 1));
              if (slot < kWaves) {
                const int f = 0xffff - (int)(r.y >> 16);
                work[slot] = Work{f, (int)(r.z & 0xffffu), (int)(r.z >> 16), (int)r.w, 0, 0};
              }
            }
            cnt += (int)__popcll(msk);
          }
          if (lane == 0) s_nwork = cnt < kWaves ? cnt : kWaves;
          stale_recomputes += cnt < kWaves ? cnt : kWaves;
        }
      }
    }
    __syncthreads();
  }

  // Final faces, ascending triples in face-id order.
  __syncthreads();
  for (int f = tid; f < nf; f += kBlock) {
    const uint4 r = P.frec[f];
    P.faces[3 * f] = (int)(r.z & 0xffffu);
    P.faces[3 * f + 1] = (int)(r.z >> 16);
    P.faces[3 * f + 2] = (int)r.w;
  }
  if (lane == 0) s_vpart[wave] = walk_rounds;
  __syncthreads();
  if (tid == 0) {
    if (!s_stop) *P.status = 0;
    if (P.stats) {
      int wr = 0;
      for (int w = 0; w < kWaves; ++w) wr += s_vpart[w];
      P.stats[0] = stale_recomputes;
      P.stats[1] = wr;
      P.stats[2] = sweeps;
      P.stats[3] = phases;
    }
  }
}

size_t loop_lds_bytes(int n) { return lds_layout(n).total; }

hipError_t launch_loop(const LoopParams& p, hipStream_t s) {
  const size_t lds = loop_lds_bytes(p.n);
  hipError_t e = hipFuncSetAttribute((const void*)tmfg_loop_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(tmfg_loop_kernel, dim3(1), dim3(kBlock), lds, s, p);
  return hipGetLastError();
}

}  // namespace tmfg
