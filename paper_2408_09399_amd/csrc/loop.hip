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
// stale pairs are recomputed lazily, only when they could decide an insertion. The global
// maximum is tracked with a two-level structure instead of a heap: face records in global
// memory (16 B each) and, per 64-face chunk, the maximum record in LDS.
//
// One selection phase (wave 0 scans the chunk maxima):
//   * if the top record is fresh, its vertex is inserted; the chunks of the three new
//     faces are queued, plus every chunk whose maximum is stale once that vertex is
//     inserted and ranks above the best fresh record that remains;
//   * otherwise every chunk whose maximum is stale and ranks above the best fresh record
//     is queued.
// Every queued chunk is loaded (one wave each). Its stale records ranked above that floor
// and the new faces are recomputed in parallel (one group of 16 lanes per face), published,
// and the chunk maxima are rebuilt from the loaded records.
//
// Best vertex of a face: the threshold walk over the three corners' sorted rows (the
// per-vertex sort of Algorithm 1, with the similarity of every entry stored beside its id).
// Each round takes the first kCand uninserted entries at or after each list's position and
// evaluates each with the similarity its list carries and the other two read from W (a
// vertex found in several lists is evaluated once per list, to the same gain). Any vertex
// not yet evaluated has W[x][u] <= the value of the bound entry of x's list (the next
// uninserted entry, or the last position scanned) for x = a, b, c, so its gain is at most
// T = (A + B) + C of those values (float32 addition is monotone). The walk stops when the
// best gain seen is strictly above T, or a list is used up. Every walk moves each list's
// cached start (the first uninserted position: the paper's MaxCorrs pointer) forward. A
// walk that needs more than its round limit (64 unless a batch's autotuner picks another)
// is finished by a sweep of the three full rows by the whole workgroup. Both give the
// exact best pair.
#include <algorithm>
#include <climits>

#include "common.h"
#include "facerule.h"
#include "internal.h"

namespace tmfg {

namespace {
constexpr int kBlock = 1024;
constexpr int kWaves = kBlock / kWave;
constexpr int kGroups = kBlock / kGroup;         // face walks in flight
constexpr int kScan = 4;                         // list entries per lane and round
constexpr int kSpan = kScan * kGroup;            // list positions scanned per round
constexpr int kCand = 8;                         // candidates taken per list and round
constexpr int kSlots = (3 * kCand + kGroup - 1) / kGroup;   // staged candidates per lane
constexpr int kSkipLoads = 4;                    // 16-byte loads per lane in a skip scan
constexpr int kMaxWork = 256;                    // faces recomputed per selection phase
constexpr int kMaxSel = 48;                      // chunks loaded per selection phase
constexpr int kSelPerWave = kMaxSel / kWaves;    // chunks each wave loads
constexpr int kSelWaves = 4;                     // waves that share the exact rule's selection
constexpr int kAdvRow = 16;                      // selection's word kAdvRow + u: advance u's row
static_assert(kMaxSel % kWaves == 0, "chunks split evenly over the waves");
static_assert(kMaxWork <= kBlock, "one thread publishes each recomputed face");
// 64-face chunks of a build and the chunk maxima each lane of a wave covers: the loop is
// compiled for two bounds, up to n = 20480 (batches and most builds) and up to kMaxN
constexpr int chunk_iters(int n_max) { return ((2 * n_max - 4 + 63) / 64 + kWave - 1) / kWave; }
constexpr int kItersSmall = chunk_iters(kMaxBatchN), kItersBig = chunk_iters(kMaxN);
// Time the sub-steps of one walk group (stats [16..19]); the waits it adds slow that group.
constexpr bool kWalkDiag = false;

// Per-group staging of a walk round. List t's slots start at t * kSlot: slot r < kCand holds
// the uninserted entry of rank r (id, similarity); slot kCand holds the list's bound entry,
// the entry of rank kCand (its position in place of an id, and its similarity) or, when the
// span held at most kCand uninserted entries, the similarity at the span's last position.
constexpr int kSlot = kCand + 1;
struct GroupBuf {
  uint16_t cid[3 * kSlot];
  float cval[3 * kSlot];
};

// What the selecting waves post to each other in a selection phase (exact rule).
struct SelShare {
  uint64_t part[kSelWaves][3];   // each wave's best record, best fresh record, and best fresh
                                 // record of another vertex than the best fresh one's
  int sync;                      // waves that have posted
  int napp;                      // stale chunks appended to sel[] after the phase's own ones
};

struct Work {
  int f;            // face id
  int a, b, c;      // corners, ascending
  uint64_t best;    // (ord(gain) << 32) | (0xffff - u), 0 when no candidate
  int sweep;        // 1 when the walk gave up and a full sweep is needed
};


// Threshold walk for one face by a group of kGroup lanes (gl = lane within the group,
// gbase = first lane of the group).
//
// Each round scans kSpan positions of every list (kScan per lane) and takes the first kCand
// uninserted entries at or after the list's position; the lane that holds such an entry
// evaluates it, with the similarity to that list's corner carried by the sorted row and the
// other two read from W. Ranks come from a scan of the lanes' counts over the group
// (positions are ordered by lane, then by entry); the candidates and each list's bound entry
// are staged in the group's LDS buffer by the lanes that hold them, and read back by all. An
// uninserted vertex not yet evaluated sits after the list's bound entry (the next uninserted
// entry, or the last position scanned), so its similarity to that corner is at most the
// bound entry's value. Each lane keeps the best key of the candidates it evaluated; the walk
// ends when any lane's key beats the bound, and the group's best is taken once at the end.
// A list whose span holds no uninserted entry is then scanned kSkipLoads * 128 positions at
// a time (bitmap only) until one is found. The code is written without data-dependent
// branches around loads, so each round costs two dependent trips to memory (list entries,
// then candidate similarities), plus one per skip scan. Returns false when it ran out of
// rounds.
__device__ bool walk_face(const LoopParams& P, int m, const uint32_t* bits, uint16_t* ptr, GroupBuf& gb, int a,
                          int b, int c, int gl, int gbase, uint64_t& best_out, int* rounds, int* gathers, int* skips,
                          unsigned long long* wt) {
  const int n = P.n;
  const int ldi = (int)P.ldi;
  const int x3[3] = {a, b, c};
  const float* Wx[3] = {P.W + (size_t)a * n, P.W + (size_t)b * n, P.W + (size_t)c * n};
  int pos[3], newp[3];
  bool tight[3], skip[3];
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    pos[t] = ptr[x3[t]];              // every entry before it is inserted
    newp[t] = pos[t];
    tight[t] = false;
    skip[t] = false;
  }
  uint64_t best = 0;
  bool done = false;
  int r = 0, ng = 0;
#define TMFG_WT(i)                                                  \
  if (wt) {                                                         \
    asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory");     \
    const uint64_t c_ = wall_clock64();                             \
    if (gl == 0) wt[i] += c_ - tw;                                  \
    tw = c_;                                                        \
  }
  uint64_t tw = wt ? wall_clock64() : 0;
  for (; r < P.max_rounds && !done; ++r) {
    // (1) this round's span of every list: ids and similarities (addresses kept inside
    //     the row; entries at or past m are masked below)
    int q[3];
    uint2 iv[3];
    float4 vv[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      q[t] = (pos[t] & ~(kScan - 1)) + kScan * gl;
      const int qc = min(q[t], ldi - kScan);
      const size_t off = (size_t)x3[t] * ldi + qc;
      iv[t] = *(const uint2*)(P.idx + off);
      vv[t] = *(const float4*)(P.vals + off);
    }
    // (2) uninserted entries, their ranks, and which are taken this round. The inserted
    //     bits of all twelve entries are read from the LDS before any is used (one trip).
    int id[3][kScan];
    float val[3][kScan];
    uint32_t um[3], take[3], insw[3][kScan];
    int seen[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      const uint32_t wd[2] = {iv[t].x, iv[t].y};
#pragma unroll
      for (int j = 0; j < kScan; ++j) {
        id[t][j] = (int)((wd[j >> 1] >> (16 * (j & 1))) & 0xffffu);
        // entries past the row's end hold 0xffff (masked below): the address stays in the bitmap
        insw[t][j] = bits[min(id[t][j], n - 1) >> 5];
      }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      val[t][0] = vv[t].x;
      val[t][1] = vv[t].y;
      val[t][2] = vv[t].z;
      val[t][3] = vv[t].w;
      // positions in [pos, m) of this lane's kScan entries: only the group's first lane can
      // start before pos, and only lanes near the row's end reach m (every entry before m
      // holds a vertex id below n)
      const uint32_t full = (1u << kScan) - 1;
      const uint32_t lo = gl == 0 ? (full << (pos[t] & (kScan - 1))) & full : full;
      const int room = m - q[t];
      const uint32_t hi = room >= kScan ? full : room > 0 ? (1u << room) - 1 : 0u;
      um[t] = 0;
#pragma unroll
      for (int j = 0; j < kScan; ++j) um[t] |= (~(insw[t][j] >> (id[t][j] & 31)) & 1u) << j;
      um[t] &= skip[t] ? 0u : (lo & hi);
      // ranks: an inclusive scan of the lanes' counts over the group by DPP row shifts;
      // the group total is the scan's value in the group's last lane
      const uint32_t cnt = (uint32_t)__popc(um[t]);
      const uint32_t incl = row_scan_u32(cnt);
      const int before = (int)(incl - cnt);
      seen[t] = (int)row_last_u32(incl);
      // ranks 0 .. kCand - 1 are staged as candidates; rank kCand, the bound entry, with its
      // position in place of the id
#pragma unroll
      for (int j = 0; j < kScan; ++j) {
        const int rank = before + __popc(um[t] & ((1u << j) - 1));
        if (((um[t] >> j) & 1u) && rank <= kCand) {
          gb.cid[t * kSlot + rank] = (uint16_t)(rank < kCand ? id[t][j] : q[t] + j);
          gb.cval[t * kSlot + rank] = val[t][j];
        }
      }
      // a span with at most kCand uninserted entries: the last position scanned bounds it
      if (gl == kGroup - 1 && seen[t] <= kCand) gb.cval[t * kSlot + kCand] = val[t][kScan - 1];
      take[t] = seen[t] < kCand ? seen[t] : kCand;
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    TMFG_WT(0);
    // (3) evaluate the staged candidates, two per lane: lane gl takes slot gl of list a
    //     (gl < kCand) or of list b (the others), and slot gl of list c (lanes gl < kCand).
    //     The two similarities not carried by the list are read from W, all loads issued
    //     before any is used. The gain keeps the order ((W[a][u] + W[b][u]) + W[c][u]); for a
    //     candidate of list a or b the first sum is the list's own value plus the other of
    //     a, b (addition commutes).
    static_assert(kCand == 8 && kGroup == 16 && kSlots == 2, "the slot layout below");
    const bool second = gl >= kCand;                  // slot gl holds a list-b candidate
    const bool ok0 = (gl & (kCand - 1)) < (int)(second ? take[1] : take[0]);
    const bool ok1 = !second && gl < (int)take[2];
    const int slc0 = gl + (second ? kSlot - kCand : 0);
    const int slc1 = second ? 3 * kSlot - 1 : 2 * kSlot + gl;   // a slot inside the buffer
    const int cu0 = (int)gb.cid[slc0], cu1 = (int)gb.cid[slc1];
    const float cv0 = gb.cval[slc0], cv1 = gb.cval[slc1];
    float bv[3];
    int bp[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      bv[t] = gb.cval[t * kSlot + kCand];
      bp[t] = (int)gb.cid[t * kSlot + kCand];
    }
    const int u0 = ok0 ? cu0 : 0, u1 = ok1 ? cu1 : 0;
    const float wo0 = (second ? Wx[0] : Wx[1])[u0];   // the other of a, b
    const float wc0 = Wx[2][u0];
    const float wa1 = Wx[0][u1], wb1 = Wx[1][u1];
    const uint64_t k0 = cand_key((cv0 + wo0) + wc0, u0);
    const uint64_t k1 = cand_key((wa1 + wb1) + cv1, u1);
    uint64_t k = ok0 ? k0 : 0;
    k = (ok1 && k1 > k) ? k1 : k;
    best = k > best ? k : best;
    ng += (ok0 ? 2 : 0) + (ok1 ? 2 : 0);
    TMFG_WT(1);
    // (4) bounds, next positions, cached starts, all uniform over the group. The span's first
    //     uninserted position is needed only until the list's cached start is settled. A list
    //     being skipped this round keeps its state.
    float bound[3];
    bool exhausted = false, skipping = false;
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      const bool live = !skip[t];
      const int end = (pos[t] & ~(kScan - 1)) + kSpan;
      const bool big = seen[t] > kCand;
      if (!tight[t]) {
        // positions grow with the lane
        const int first = group_min_i32(um[t] ? q[t] + (int)__builtin_ctz(um[t]) : 0x7fffffff);
        newp[t] = live ? (first != 0x7fffffff ? first : min(end, m)) : newp[t];
        tight[t] = live && first != 0x7fffffff;
      }
      skipping |= !live;
      bound[t] = (live && (big || end < m)) ? bv[t] : -INFINITY;
      exhausted |= live && !big && end >= m;         // the list is used up: nothing unseen
      pos[t] = live ? (big ? bp[t] : min(end, m)) : pos[t];
      skip[t] = !live || (!big && end < m && seen[t] == 0);   // a fully inserted stretch: scan ahead wide
    }
    const float T = (bound[0] + bound[1]) + bound[2];
    // A list being skipped has no bound this round; only exhaustion can end the walk then.
    // The group's best beats T exactly when some lane's does.
    const uint64_t beat = __builtin_amdgcn_ballot_w64((uint32_t)(best >> 32) > ord_f32(T));
    done = exhausted || (!skipping && ((beat >> gbase) & 0xffffu) != 0);
    TMFG_WT(2);
    // (5) wide scans, one list at a time, for lists in a fully inserted stretch
    if (!done && (skip[0] || skip[1] || skip[2])) {
      ++*skips;
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        if (!skip[t]) continue;
        uint4 sv[kSkipLoads];
#pragma unroll
        for (int w = 0; w < kSkipLoads; ++w) {
          const int qs = (pos[t] & ~7) + (w * kGroup + gl) * 8;
          sv[w] = *(const uint4*)(P.idx + (size_t)x3[t] * ldi + min(qs, ldi - 8));
        }
        int fp = 0x7fffffff;
#pragma unroll
        for (int w = 0; w < kSkipLoads; ++w) {
          const int qs = (pos[t] & ~7) + (w * kGroup + gl) * 8;
          const uint32_t mk = open_mask8(bits, sv[w], n, qs, pos[t], m);
          fp = mk ? min(fp, qs + (int)__builtin_ctz(mk)) : fp;
        }
        const int f = group_min_i32(fp);
        const int end = (pos[t] & ~7) + kSkipLoads * kGroup * 8;
        if (f != 0x7fffffff) {
          pos[t] = f;
          skip[t] = false;
          if (!tight[t]) {
            tight[t] = true;
            newp[t] = f;
          }
        } else {
          pos[t] = end < m ? end : m;
          if (!tight[t]) newp[t] = pos[t];
          if (end >= m) done = true;             // nothing uninserted is left in this list
        }
      }
    }
    TMFG_WT(3);
  }
  if (gl == 0) {
#pragma unroll
    for (int t = 0; t < 3; ++t)
      if (newp[t] > (int)ptr[x3[t]]) ptr[x3[t]] = (uint16_t)newp[t];
  }
#undef TMFG_WT
  *rounds += r;
  *gathers += ng;
  best_out = group_max_u64(best);
  return done;
}

}  // namespace

// ---------------------------------------------------------------------------------------
// Bulk exact best vertex of many faces by sweeping their three rows (one workgroup per
// face). Reads 12n bytes of W plus the n-bit inserted set per face. A face with a corner
// outside [0, n) reads nothing and gets best_u = -2 and a NaN gain.
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
  if ((unsigned)a >= (unsigned)n || (unsigned)b >= (unsigned)n || (unsigned)c >= (unsigned)n) {
    if (threadIdx.x == 0) {      // the whole workgroup leaves here: no barrier is skipped by part of it
      best_u[f] = -2;
      best_gain[f] = __builtin_nanf("");
    }
    return;
  }
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

__device__ __forceinline__ uint4 make_rec(const Work& w) { return face_record(w.f, w.a, w.b, w.c, w.best); }

// Wave 0: append to sel[] (after its first `cnt` entries) every chunk whose maximum record is
// stale and ranks above `floor`, other than chunks c1 and c2 (already listed). The lane holds
// the maxima of chunks lane + i * kWave (key words khi/klo, inserted flags in insm). Returns
// the new length, at most kMaxSel.
template <int CI>
__device__ int append_stale_chunks(const uint32_t (&khi)[CI], const uint32_t (&klo)[CI],
                                   uint32_t insm, int nchunk, uint64_t floor, int c1, int c2, int* sel, int cnt,
                                   int lane) {
#pragma unroll
  for (int i = 0; i < CI; ++i) {
    const int ch = lane + i * kWave;
    const uint64_t k = ((uint64_t)khi[i] << 32) | klo[i];
    const bool pick = ch < nchunk && ch != c1 && ch != c2 && k > floor && ((insm >> i) & 1u);
    const uint64_t msk = __ballot(pick);
    if (pick) {
      const int slot = cnt + (int)__popcll(msk & ((1ull << lane) - 1));
      if (slot < kMaxSel) sel[slot] = ch;
    }
    cnt += (int)__popcll(msk);
  }
  return cnt < kMaxSel ? cnt : kMaxSel;
}

// Paper rule, wave 0: of the chunks whose maximum record is stale and ranks above `floor`
// (other than c1 and c2), append to sel[] the kPaperChunks of highest maximum, in key order.
// *rest receives the largest maximum of the others (0 if none), the same in every lane: no
// record of an unlisted chunk ranks above it. Returns the new length.
constexpr int kPaperChunks = 4;
template <int CI>
__device__ int pick_top_stale_chunks(const uint32_t (&khi)[CI], const uint32_t (&klo)[CI],
                                     uint32_t insm, int nchunk, uint64_t floor, int c1, int c2, int* sel, int cnt,
                                     int lane, uint64_t* rest) {
  uint32_t cm = 0;                       // this lane's candidate chunks, by i
#pragma unroll
  for (int i = 0; i < CI; ++i) {
    const int ch = lane + i * kWave;
    const uint64_t k = ((uint64_t)khi[i] << 32) | klo[i];
    cm |= (ch < nchunk && ch != c1 && ch != c2 && k > floor && ((insm >> i) & 1u)) ? (1u << i) : 0u;
  }
  uint64_t lm = 0;                       // this lane's largest candidate and its index
  int li = 0;
  auto local_max = [&]() {
    lm = 0;
#pragma unroll
    for (int i = 0; i < CI; ++i) {
      const uint64_t k = ((uint64_t)khi[i] << 32) | klo[i];
      const bool c = ((cm >> i) & 1u) && k > lm;
      lm = c ? k : lm;
      li = c ? i : li;
    }
  };
  local_max();
  for (int s = 0; s < kPaperChunks; ++s) {
    const uint64_t g = wave_max_dpp(lm);
    if (g == 0) break;
    if (lm == g) {                       // keys are unique: one lane holds it
      sel[cnt] = lane + li * kWave;
      cm &= ~(1u << li);
      local_max();
    }
    ++cnt;
  }
  *rest = wave_max_dpp(lm);
  return cnt;
}
static_assert(kPaperChunks + 2 <= kMaxSel, "the paper rule's chunks fit the load list");

// Wave: move vertex v's row position to its first uninserted entry, 512 entries per trip
// (entries before the position are inserted; the position only grows).
__device__ __forceinline__ void advance_row(const uint16_t* __restrict__ idx, int ldi, const uint32_t* bits,
                                            uint16_t* ptr, int v, int m, int n, int lane) {
  const uint16_t* row = idx + (size_t)v * ldi;
  int p = ptr[v];
  for (;;) {
    const int qs = (p & ~7) + lane * 8;
    const uint4 sv = *(const uint4*)(row + min(qs, ldi - 8));
    const uint32_t mk = open_mask8(bits, sv, n, qs, p, m);
    const int fp = mk ? qs + (int)__builtin_ctz(mk) : 0x7fffffff;
    const int f = wave_min_i32(fp);
    if (f != 0x7fffffff) {
      p = f;
      break;
    }
    p = (p & ~7) + kWave * 8;
    if (p >= m) {
      p = m;
      break;
    }
  }
  if (lane == 0 && p > (int)ptr[v]) ptr[v] = (uint16_t)p;
}

// The record a work item publishes, as one sortable key (0 when it has no vertex).
__device__ __forceinline__ uint64_t work_key(const Work& w) { return rec_key(make_rec(w)); }

__device__ __forceinline__ uint64_t clock_ticks() { return wall_clock64(); }
}  // namespace

// Paper selects the paper's face rule (Algorithm 2) in place of the exact one. Its cached
// pairs are no upper bounds (a recomputed pair can rank higher than the one it replaces), so
// the order of recomputation is part of the result: the heap pops stale pairs one at a time
// in key order, and a pair made fresh at once competes with the next stale one. Each phase
// recomputes in parallel the stale pairs ranked above the best fresh one, then commits a
// recomputed pair only if its old key ranks above every fresh pair (those of the new faces
// included), every recomputed pair of a stale record ranked above it, and every stale record
// that was not recomputed; a pair not committed keeps its old record. This is the order in
// which the heap would pop them. The top record of a phase that finds a stale maximum is
// always recomputed and committed, so every such phase makes progress.
// Stats records the counters and step timers of tmfg_plan_stats (P.stats is then set); they
// sit on the loop's critical path (LDS atomics after every walk, clock reads between steps),
// so a build that does not ask for them compiles them out.
template <bool Paper, int CI, bool Stats>
__device__ void run_loop(const LoopParams& P, uint8_t* smem) {
  __shared__ Work work[kMaxWork];
  __shared__ int sel[kMaxSel];
  __shared__ GroupBuf gbuf[kGroups];
  __shared__ uint4 s_crec[kMaxSel][kWave];       // the loaded chunk records
  __shared__ int16_t s_link[kMaxSel][kWave];     // work item replacing each record, or -1
  __shared__ int s_nwork, s_nnew, s_nsel, s_ins, s_F, s_stop, s_nsweep, s_bmax, s_seed[4], s_next;
  __shared__ int s_b0;                           // waves done with their share of phase B0
  __shared__ SelShare s_sel;                     // the exact rule's selecting waves' posts
  __shared__ int s_u4[4];                        // the vertex the last single-wave selection
                                                 // inserted, and the corners of the face it split
  __shared__ int s_adv;                          // selection's word to the advancing waves: 0 not yet,
                                                 // 1 advance s_u4's rows, 2 nothing to advance,
                                                 // kAdvRow + u advance u's row only
  __shared__ uint64_t s_floor;
  __shared__ int s_pre;                          // a vertex whose row position is at its first
                                                 // uninserted entry since the last insertion, or -1
  // paper rule: old keys and new keys of the work items, the best fresh record of the loaded
  // chunks that stays, and the best stale record that was not recomputed
  __shared__ uint64_t s_old[Paper ? kMaxWork : 1], s_newk[Paper ? kMaxWork : 1];
  __shared__ uint64_t s_best0, s_unloaded, s_rest;
  __shared__ uint64_t s_part[kWaves];
  __shared__ int s_vpart[kWaves];

  const int n = P.n;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int gl = lane & (kGroup - 1), gbase = lane & ~(kGroup - 1);
  const int gid = tid / kGroup;                              // face-walk group of this lane
  const LdsLayout LL = lds_layout(n);
  uint4* cmax = (uint4*)(smem + LL.off_cmax);
  uint32_t* bits = (uint32_t*)(smem + LL.off_bits);
  uint16_t* ptr = (uint16_t*)(smem + LL.off_ptr);
  const int nf = 2 * n - 4;
  const uint64_t t_start = clock_ticks();
  LoopStateHeader* hdr = (LoopStateHeader*)P.state;
  // entries per sorted row and the loop time of earlier segments, kept in LDS so that they
  // hold no registers in the loop
  __shared__ int s_m;
  __shared__ unsigned long long s_tbase;

  if (P.resume) {
    // A later segment has nothing to do when the build ended or stopped in an earlier one.
    // Every thread reads the flag before thread 0 clears it (after the first barrier below).
    if (!hdr->live) return;
  } else {
    if (hdr && tid == 0) hdr->live = 0;
    // Errors raised by the kernels that produced W stop the build here.
    const uint32_t fl = *P.flags;
    if (fl) {
      const int32_t st = (fl & kFlagNonFinite) ? 3 : (fl & kFlagAsymmetric) ? 4 : (fl & kFlagDegenerate) ? 5 : 8;
      if (tid == 0) *P.status = st;
      if (P.hout.order) publish_outputs(P.hout, P.order, P.edges, P.steps, P.step_gain, P.faces, n, st);
      return;
    }
  }

  if (!P.resume) {
    for (int i = tid; i < nf; i += kBlock) P.frec[i] = make_uint4(0, 0, 0, 0);
    for (int i = tid; i < LL.nchunk; i += kBlock) cmax[i] = make_uint4(0, 0, 0, 0);
    for (int i = tid; i < LL.nw; i += kBlock) bits[i] = 0;
    for (int i = tid; i < n; i += kBlock) ptr[i] = 0;

    // Seed: top-4 by (score desc, id asc).
    seed_top4<kBlock>(P.scores, n, s_seed, s_part, s_vpart);
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
        work[f] = Work{f, x, y, z, 0, 0};
      }
      s_nwork = 4;
      s_nnew = 4;
      sel[0] = 0;
      s_nsel = 1;
      s_floor = ~0ull;
      s_ins = 4;
      s_F = 4;
      s_stop = 0;
      s_nsweep = 0;
      s_bmax = 0;
      s_next = 0;
      s_b0 = 0;
      s_sel.sync = 0;
      s_sel.napp = 0;
      s_pre = -1;
      if (Paper) {
        s_best0 = 0;
        s_unloaded = 0;
        s_rest = 0;
      }
      s_m = P.m;
      s_tbase = 0;
    }
  } else {
    // Resume at a phase boundary: the LDS image comes back, every row position restarts at 0
    // (the rows were compacted since, so every entry is uninserted but the filler), and an
    // empty phase leads to the next selection.
    const uint32_t* img = (const uint32_t*)(P.state + kStateHeader);
    for (int i = tid; i < (int)(LL.total / 4); i += kBlock) ((uint32_t*)smem)[i] = img[i];
    __syncthreads();
    for (int i = tid; i < n; i += kBlock) ptr[i] = 0;
    if (tid == 0) {
      s_nwork = 0;
      s_nnew = 0;
      s_nsel = 0;
      s_floor = ~0ull;
      s_ins = hdr->ins;
      s_F = hdr->F;
      s_stop = 0;
      s_nsweep = 0;
      s_bmax = 0;
      s_next = 0;
      s_b0 = 0;
      s_sel.sync = 0;
      s_sel.napp = 0;
      s_pre = -1;
      if (Paper) {
        s_best0 = 0;
        s_unloaded = 0;
        s_rest = 0;
      }
      s_m = hdr->m_new;
      s_tbase = hdr->ticks;
      hdr->live = 0;
    }
  }
  __syncthreads();

  // Counters (tmfg_plan_stats): kept in LDS so that they hold no registers in the loop.
  //   [0] stale recomputes [1] walk rounds [2] sweeps [3] phases [4] walk batches
  //   [5..9] ticks in select/load/walk/sweep/publish [11] W reads [12] critical rounds
  //   [13] walks >= 4 rounds [14] walks >= 16 rounds [15] skip scans [16] stale maxima
  //   [17] work overflows [18] chunk overflows [19] recomputed pairs not committed (paper)
  __shared__ unsigned long long s_cnt[20];
  __shared__ unsigned long long s_wt[4];         // walk sub-step ticks of group 0 (diagnostics)
  __shared__ int s_since_insert, s_compactions;
  __shared__ unsigned long long s_t0;
  if (tid < 20) s_cnt[tid] = P.resume ? hdr->cnt[tid] : 0;
  if (tid < 4) s_wt[tid] = 0;
  if (tid == 0) {
    s_since_insert = P.resume ? hdr->since_insert : 0;
    s_compactions = P.resume ? hdr->compactions : 0;
    s_t0 = clock_ticks();
  }
  __syncthreads();
#define TMFG_LAP(slot)                    \
  if (Stats && tid == 0) {                \
    const uint64_t t1_ = clock_ticks();   \
    s_cnt[slot] += t1_ - s_t0;            \
    s_t0 = t1_;                           \
  }
  for (;;) {
    // The thread index is made opaque each phase, so that the many LDS addresses derived from
    // it are formed anew rather than held (and spilled) across the loop.
    int tid_o = tid;
    asm volatile("" : "+v"(tid_o));
    const int tid = tid_o, lane = tid & 63, wave = tid >> 6;
    const int gl = lane & (kGroup - 1), gbase = lane & ~(kGroup - 1);
    const int gid = tid / kGroup;
    // Phase B0: load the records of the queued chunks (one wave per chunk, one record per
    // lane). Each record is linked to the work item that will replace it: a new face, or a
    // stale record ranked above the floor, which is queued for recomputation.
    const int nsel = min(s_nsel + s_sel.napp, kMaxSel), nnew = s_nnew;
    const uint64_t floor = s_floor;
    // paper rule: stale records at or below the largest record of the chunks left unloaded
    // cannot be committed this phase, so they are not recomputed
    const uint64_t cut = Paper ? max64(floor, s_rest) : floor;
    if (wave < nsel) {
      // all of this wave's records are requested before any is used (one trip to memory)
      uint4 crecs[kSelPerWave];
#pragma unroll
      for (int i = 0; i < kSelPerWave; ++i) {
        const int sl = wave + i * kWaves;
        const int f = (sl < nsel ? sel[sl] : 0) * 64 + lane;
        crecs[i] = P.frec[f < nf ? f : nf - 1];
      }
#pragma unroll
      for (int i = 0; i < kSelPerWave; ++i) {
        const int sl = wave + i * kWaves;
        if (sl >= nsel) break;
        const int f = sel[sl] * 64 + lane;
        const uint4 crec = f < nf ? crecs[i] : make_uint4(0, 0, 0, 0);
        int link = -1;
        for (int q = 0; q < nnew; ++q)
          if (work[q].f == f) link = q;
        uint64_t kfresh = 0;
        if (link < 0 && s_ins < n) {
          const uint64_t k = rec_key(crec);
          const bool stale = is_ins(bits, rec_vertex(crec));
          if (k != 0 && k > cut && stale) {
            const int slot = atomicAdd(&s_nwork, 1);
            if (slot < kMaxWork) {
              work[slot] = Work{f, (int)(crec.z & 0xffffu), (int)(crec.z >> 16), (int)crec.w, 0, 0};
              if (Paper) s_old[slot] = k;
              link = slot;
            } else if (Paper) {
              atomicMax(&s_unloaded, (unsigned long long)k);
            }
          }
          if (Paper && !stale) kfresh = k;
        }
        if (Paper) {
          kfresh = wave_max_dpp(kfresh);
          if (lane == 0 && kfresh > s_best0) atomicMax(&s_best0, (unsigned long long)kfresh);
        }
        s_crec[sl][lane] = crec;
        s_link[sl][lane] = (int16_t)link;
      }
    }
    // This wave's share of B0 is done. The stale work items are final once every wave has
    // said so; the new faces' items were written by the selection, so their walks need not
    // wait for B0 (no barrier here: the other waves' loads of chunk records overlap them).
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    if (lane == 0) {
      const int done = __hip_atomic_fetch_add(&s_b0, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
      if (Stats && done == kWaves - 1) {
        const int nw = s_nwork < kMaxWork ? s_nwork : kMaxWork;
        s_cnt[0] += nw - nnew;
        if (s_nwork > kMaxWork) s_cnt[17] += 1;
        if (nsel >= kMaxSel) s_cnt[18] += 1;
        const uint64_t t1 = clock_ticks();
        s_cnt[6] += t1 - s_t0;
        s_t0 = t1;
      }
    }
    const bool have_cand = s_ins < n;
    if (wave == kWaves - 1 && have_cand) {
      // The last wave, before it takes walks, moves the row position of the best fresh
      // record's vertex (the floor) to its first uninserted entry. That vertex is usually the
      // next one inserted, and its row is then already advanced when the selection names it:
      // the vertex's own insertion changes nothing in its row. It is no face corner, so no
      // walk reads or moves its position meanwhile.
      const int v = (int)(floor & 0xffffu);
      if (floor != 0 && floor != ~0ull && v < n && v != s_pre && !is_ins(bits, v)) {
        advance_row(P.idx, (int)P.ldi, bits, ptr, v, s_m, n, lane);
        if (lane == 0) s_pre = v;
      }
    }
    // Phase B: best pair of every queued face, one group of kGroup lanes per face. A wave
    // takes the next batch of kWave / kGroup faces from a counter when it is free, so a deep
    // walk holds up only its own wave. Batch 0 is the new faces (items [0, nnew)), taken by
    // the first wave to get here; batch b >= 1 holds stale items nnew + (b - 1) * 4 ... and is
    // walked once B0 is done everywhere.
    for (;;) {
      int b = 0;
      if (lane == 0) b = atomicAdd(&s_next, 1);
      b = __builtin_amdgcn_readfirstlane(b);
      int base = 0, limit = nnew;
      if (b > 0) {
        // a bounded wait: the other waves' B0 shares take one trip to memory; should it ever
        // run out, the build stops with an internal error rather than walk unqueued items
        int it = 0;
        while (__hip_atomic_load(&s_b0, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < kWaves && it < (1 << 24))
          ++it;
        if (it >= (1 << 24)) {
          if (lane == 0) {
            *P.status = 8;
            s_stop = 1;
          }
          break;
        }
        base = nnew + (b - 1) * (kWave / kGroup);
        limit = s_nwork < kMaxWork ? s_nwork : kMaxWork;
        if (base >= limit) break;
      } else if (nnew == 0) {
        continue;
      }
      if (Stats && lane == 0) atomicAdd(&s_cnt[4], 1ull);
      const int item = base + (lane / kGroup);
      if (item < limit) {
        Work& w = work[item];
        uint64_t best = 0;
        bool ok = true;
        int rw = 0, gw = 0, sw = 0;
        if (have_cand) {
          if (Paper)
            best = paper_face(P.W, P.idx, n, s_m, (int)P.ldi, bits, ptr, w.a, w.b, w.c, gl, &rw);
          else
            ok = walk_face(P, s_m, bits, ptr, gbuf[gid], w.a, w.b, w.c, gl, gbase, best, &rw, &gw, &sw,
                           (kWalkDiag && P.stats && gid == 0) ? s_wt : nullptr);
        }
        // per-lane W reads, summed over the group
        if (Stats) gw = group_sum_i32(gw);
        if (gl == 0) {
          w.best = best;
          w.sweep = ok ? 0 : 1;
          if (!ok) atomicAdd(&s_nsweep, 1);
          if (Stats) {
            atomicMax(&s_bmax, rw);
            atomicAdd(&s_cnt[1], (unsigned long long)rw);
            atomicAdd(&s_cnt[11], (unsigned long long)gw);
            atomicAdd(&s_cnt[15], (unsigned long long)sw);
            if (rw >= 4) atomicAdd(&s_cnt[13], 1ull);
            if (rw >= 16) atomicAdd(&s_cnt[14], 1ull);
          }
        }
      }
    }
    __syncthreads();
    const int nwork = s_nwork < kMaxWork ? s_nwork : kMaxWork;
    if (Stats && tid == 0) {
      s_cnt[12] += s_bmax;
      s_bmax = 0;
    }
    TMFG_LAP(7);
    // Phase B2: faces whose walk gave up are swept by the whole workgroup, one at a time.
    for (int q = 0; s_nsweep && q < nwork; ++q) {
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
      best = wave_max_dpp(best);
      if (lane == 0) s_part[wave] = best;
      __syncthreads();
      if (tid == 0) {
        uint64_t k = s_part[0];
        for (int w = 1; w < kWaves; ++w) k = s_part[w] > k ? s_part[w] : k;
        work[q].best = k;
        work[q].sweep = 0;
        s_cnt[2] += 1;
      }
      __syncthreads();
    }
    if (Paper && nwork > nnew) {
      // Ordered commit (paper rule): items [0, nnew) are always committed.
      if (tid < nwork) s_newk[tid] = work_key(work[tid]);
      __syncthreads();
      if (tid >= nnew && tid < nwork) {
        const uint64_t old = s_old[tid];
        uint64_t lim = max64(max64(floor, s_best0), s_unloaded);
        for (int q = 0; q < nnew; ++q) lim = max64(lim, s_newk[q]);
        for (int q = nnew; q < nwork; ++q) lim = s_old[q] > old ? max64(lim, s_newk[q]) : lim;
        if (old <= lim) {
          // keep the old record: (gain, vertex) back into the item's pair
          work[tid].best = (old & 0xffffffff00000000ull) | (0xffffull - (old & 0xffffull));
          if (Stats) atomicAdd(&s_cnt[19], 1ull);
        }
      }
      __syncthreads();
    }
    TMFG_LAP(8);
    // Phase B3: publish the new face records. Phase C: rebuild the maxima of the loaded
    // chunks from the records held in registers, with the recomputed ones substituted.
    if (tid == 0) {
      s_nsweep = 0;
      s_next = 0;
      s_b0 = 0;
      s_adv = 0;
      s_sel.sync = 0;
      s_sel.napp = 0;
      if (Paper) {
        s_best0 = 0;
        s_unloaded = 0;
        s_rest = 0;
      }
    }
    if (tid < nwork) P.frec[work[tid].f] = make_rec(work[tid]);
    for (int sl = wave; sl < nsel; sl += kWaves) {
      const int link = s_link[sl][lane];
      const uint4 crec = link >= 0 ? make_rec(work[link]) : s_crec[sl][lane];
      const uint64_t k = rec_key(crec);
      const uint64_t mx = wave_max_dpp(k);
      const uint64_t msk = __ballot(k == mx);
      if (lane == (int)__builtin_ctzll(msk)) cmax[sel[sl]] = crec;
    }
    __syncthreads();
    TMFG_LAP(9);
    if (s_ins >= n || s_stop) break;
    if (s_ins >= P.stop_at) {
      // Checkpoint (single builds): save the state and return; the rows are compacted before
      // the next segment resumes here.
      uint32_t* img = (uint32_t*)(P.state + kStateHeader);
      for (int i = tid; i < (int)(LL.total / 4); i += kBlock) img[i] = ((const uint32_t*)smem)[i];
      if (tid == 0) {
        hdr->ins = s_ins;
        hdr->F = s_F;
        hdr->since_insert = s_since_insert;
        hdr->compactions = s_compactions + 1;
        hdr->m_old = s_m;
        hdr->m_new = n - s_ins;
        hdr->off_bits = (int)LL.off_bits;
        hdr->off_ptr = (int)LL.off_ptr;
        hdr->ticks = s_tbase + (clock_ticks() - t_start);
        for (int i = 0; i < 20; ++i) hdr->cnt[i] = s_cnt[i];
        hdr->live = 1;
      }
      return;
    }
    // Phase A: select. For large builds the exact rule spreads the scan of the chunk maxima
    // over kSelWaves waves (below); otherwise, and always for the paper rule (whose choice of
    // stale chunks is ordered), wave 0 selects alone.
    if (Stats && tid == 0) s_cnt[3] += 1;
    // builds of more than two chunk maxima per lane share the scan; smaller ones gain less
    // from it than the waves' exchanges cost
    const bool multi = !Paper && LL.nchunk > 2 * kWave;
    if (multi && wave < kSelWaves) {
      // Each of the kSelWaves waves reads the maxima of its share of the chunks (lane + i *
      // kWave for i in its range) and the inserted bits of their vertices, and posts its best
      // record, its best fresh record, and its best fresh record of another vertex than that
      // one's; all of them then take the same decision from the posted values. On an
      // insertion of u, the floor (the best fresh record once u counts as inserted) is the
      // largest over the waves of their best fresh record, or of the other one where the best
      // is u's. Each wave appends its own stale chunks ranked above the floor to sel[] through
      // a counter. Which stale chunks are recomputed in a phase, and in which order, decides
      // no result: every cached key is an upper bound, and only a fresh maximum is inserted.
      constexpr int CIW = (CI + kSelWaves - 1) / kSelWaves;
      const int ins = s_ins, F = s_F, since = s_since_insert;   // read before any wave changes them
      uint32_t khi[CIW], klo[CIW];
      uint32_t insm = 0;
      int sl_lane = lane;
      asm volatile("" : "+v"(sl_lane));
      const int i0 = wave * CIW;
#pragma unroll
      for (int j = 0; j < CIW; ++j) {
        const int ch = sl_lane + (i0 + j) * kWave;
        const uint4 r = cmax[ch < LL.nchunk ? ch : 0];
        khi[j] = ch < LL.nchunk ? r.x : 0u;
        klo[j] = ch < LL.nchunk ? r.y : 0u;
      }
#pragma unroll
      for (int j = 0; j < CIW; ++j)
        insm |= is_ins(bits, (int)(klo[j] & 0xffffu)) ? (1u << j) : 0u;
      // k1: best record; b1: best fresh record, of vertex v1; b2: best fresh record of a
      // vertex other than v1
      uint64_t k1 = 0, b1 = 0, b2 = 0;
      uint32_t v1 = 0xffffffffu;
#pragma unroll
      for (int j = 0; j < CIW; ++j) {
        const uint64_t k = ((uint64_t)khi[j] << 32) | klo[j];
        const uint32_t v = klo[j] & 0xffffu;
        k1 = max64(k1, k);
        if (!((insm >> j) & 1u) && k != 0) {
          if (k > b1) {
            b2 = v != v1 ? b1 : b2;
            b1 = k;
            v1 = v;
          } else if (v != v1) {
            b2 = max64(b2, k);
          }
        }
      }
      k1 = wave_max_dpp(k1);
      const uint64_t B1 = wave_max_dpp(b1);
      const uint64_t B2 = wave_max_dpp(v1 != ((uint32_t)B1 & 0xffffu) ? b1 : b2);
      // post, then wait (a bounded wait: the other selecting waves do the same work and wait
      // for nothing else) and combine
      if (lane == 0) {
        s_sel.part[wave][0] = k1;
        s_sel.part[wave][1] = B1;
        s_sel.part[wave][2] = B2;
        __hip_atomic_fetch_add(&s_sel.sync, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
      int it = 0;
      while (__hip_atomic_load(&s_sel.sync, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < kSelWaves &&
             it < (1 << 24))
        ++it;
      const bool ok = it < (1 << 24);
      uint64_t K1 = 0, KF = 0;
#pragma unroll
      for (int w = 0; w < kSelWaves; ++w) {
        K1 = max64(K1, s_sel.part[w][0]);
        KF = max64(KF, s_sel.part[w][1]);
      }
      const int f1 = 0xffff - (int)((uint32_t)K1 >> 16);
      int ns0 = 1, c1 = f1 >> 6, c2 = c1;
      uint64_t fl = KF;                          // the floor for the stale chunks to append
      bool append = ok;
      if (!ok) {
        append = false;
      } else if (K1 != 0 && K1 == KF) {
        // Fresh maximum: insert its vertex.
        const uint32_t u = (uint32_t)K1 & 0xffffu;
        c2 = F >> 6;                             // F is even, so F and F + 1 share a chunk
        ns0 = c2 != c1 ? 2 : 1;
        if (wave == 0) {
          if (lane == 0) {
            // first what the advancing wave needs, u itself, in the word that releases it: u's
            // own row holds no entry of u, so it may be advanced before u's bit is set
            __hip_atomic_store(&s_adv, kAdvRow + (int)u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
            atomicOr(&bits[u >> 5], 1u << (u & 31));
          }
          const uint4 r = cmax[c1];
          const int x = (int)(r.z & 0xffffu), y = (int)(r.z >> 16), z = (int)r.w;
          if (lane == 0) {
            const int st = ins - 4;
            P.order[ins] = (int)u;
            int32_t* e = P.edges + 2 * (6 + 3 * st);
            e[0] = u; e[1] = x; e[2] = u; e[3] = y; e[4] = u; e[5] = z;
            int32_t* sp = P.steps + 4 * st;
            sp[0] = f1; sp[1] = x; sp[2] = y; sp[3] = z;
            P.step_gain[st] = unord_f32(r.x);
            int t0_ = u, t1_ = x, t2_ = y;
            sort3(t0_, t1_, t2_);
            work[0] = Work{f1, t0_, t1_, t2_, 0, 0};
            t0_ = u; t1_ = y; t2_ = z;
            sort3(t0_, t1_, t2_);
            work[1] = Work{F, t0_, t1_, t2_, 0, 0};
            t0_ = u; t1_ = x; t2_ = z;
            sort3(t0_, t1_, t2_);
            work[2] = Work{F + 1, t0_, t1_, t2_, 0, 0};
            s_ins = ins + 1;
            s_F = F + 2;
            s_nwork = 3;
            s_nnew = 3;
            sel[0] = c1;
            sel[1] = c2;
          }
        }
        // The chunks of the three new faces are reloaded. Faces whose cached vertex was u are
        // stale now; the chunks whose maximum is stale and ranks above the best fresh record
        // that remains are loaded too, and every stale record in them ranked above that floor
        // is recomputed along with the new faces.
        if (ins + 1 < n) {
#pragma unroll
          for (int j = 0; j < CIW; ++j)
            if ((klo[j] & 0xffffu) == u) insm |= 1u << j;
          fl = 0;
#pragma unroll
          for (int w = 0; w < kSelWaves; ++w) {
            const uint64_t p1 = s_sel.part[w][1], p2 = s_sel.part[w][2];
            fl = max64(fl, ((uint32_t)p1 & 0xffffu) != u ? p1 : p2);
          }
        } else {
          fl = ~0ull;
          append = false;
        }
        if (wave == 0 && lane == 0) {
          s_nsel = ns0;
          s_floor = fl;
          s_since_insert = 0;
        }
      } else if (K1 == 0 || since + 1 > nf + 8) {
        append = false;
        if (wave == 0 && lane == 0) {
          *P.status = 8;
          s_stop = 1;
          s_nwork = 0;
          s_nnew = 0;
          s_nsel = 0;
          __hip_atomic_store(&s_adv, 2, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
      } else {
        // Stale maximum: load every chunk whose maximum is stale and ranks above the best
        // fresh record (the top one first) and recompute their stale records above it.
        if (wave == 0 && lane == 0) {
          if (Stats) s_cnt[16] += 1;
          sel[0] = c1;
          __hip_atomic_store(&s_adv, 2, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
          s_nsel = 1;
          s_floor = KF;
          s_nwork = 0;
          s_nnew = 0;
          s_since_insert = since + 1;
        }
      }
      if (!ok && wave == 0 && lane == 0) {
        // the wait ran out (it cannot, as each selecting wave posts without waiting for
        // anything): stop the build with an internal error
        *P.status = 8;
        s_stop = 1;
        s_nwork = 0;
        s_nnew = 0;
        s_nsel = 0;
        __hip_atomic_store(&s_adv, 2, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
      if (append) {
        // this wave's stale chunks above the floor, after the ns0 chunks of the phase's own
        // list: one counter addition per wave, then each lane its slots
        uint32_t pm = 0;
#pragma unroll
        for (int j = 0; j < CIW; ++j) {
          const int ch = sl_lane + (i0 + j) * kWave;
          const uint64_t k = ((uint64_t)khi[j] << 32) | klo[j];
          pm |= (ch < LL.nchunk && ch != c1 && ch != c2 && k > fl && ((insm >> j) & 1u)) ? (1u << j) : 0u;
        }
        int cnt = 0;
        uint64_t msk[CIW];
#pragma unroll
        for (int j = 0; j < CIW; ++j) {
          msk[j] = __ballot((pm >> j) & 1u);
          cnt += (int)__popcll(msk[j]);
        }
        int base = 0;
        if (lane == 0 && cnt) base = atomicAdd(&s_sel.napp, cnt);
        base = __builtin_amdgcn_readfirstlane(base);
#pragma unroll
        for (int j = 0; j < CIW; ++j) {
          if ((pm >> j) & 1u) {
            const int slot = ns0 + base + (int)__popcll(msk[j] & ((1ull << lane) - 1));
            if (slot < kMaxSel) sel[slot] = sl_lane + (i0 + j) * kWave;
          }
          base += (int)__popcll(msk[j]);
        }
      }
    } else if (!multi && wave == 0) {
      // Every chunk maximum this lane covers is read once (all loads in flight together),
      // then the inserted bits of their vertices; the top record, the best fresh one, the
      // floor after an insertion and the stale chunks to reload all come from these.
      uint32_t khi[CI], klo[CI];
      uint32_t insm = 0;
      // the lane index is made opaque here so that the chunk addresses below are formed anew
      // each phase rather than held in registers across the whole loop
      int sl_lane = lane;
      asm volatile("" : "+v"(sl_lane));
#pragma unroll
      for (int i = 0; i < CI; ++i) {
        const int ch = sl_lane + i * kWave;
        const uint4 r = cmax[ch < LL.nchunk ? ch : 0];
        khi[i] = ch < LL.nchunk ? r.x : 0u;
        klo[i] = ch < LL.nchunk ? r.y : 0u;
      }
#pragma unroll
      for (int i = 0; i < CI; ++i)
        insm |= is_ins(bits, (int)(klo[i] & 0xffffu)) ? (1u << i) : 0u;
      uint64_t k1 = 0, kf = 0;
#pragma unroll
      for (int i = 0; i < CI; ++i) {
        const uint64_t k = ((uint64_t)khi[i] << 32) | klo[i];
        k1 = max64(k1, k);
        kf = ((insm >> i) & 1u) ? kf : max64(kf, k);
      }
      k1 = wave_max_dpp(k1);
      kf = wave_max_dpp(kf);
      const int f1 = 0xffff - (int)((uint32_t)k1 >> 16);
      if (k1 != 0 && k1 == kf) {
        // Fresh maximum: insert its vertex.
        const uint4 r = cmax[f1 >> 6];
        const int u = rec_vertex(r);
        const int x = (int)(r.z & 0xffffu), y = (int)(r.z >> 16), z = (int)r.w;
        const int F = s_F;
        const int ins = s_ins;                 // vertices inserted before this one
        if (lane == 0) {
          const int st = ins - 4;
          P.order[ins] = u;
          int32_t* e = P.edges + 2 * (6 + 3 * st);
          e[0] = u; e[1] = x; e[2] = u; e[3] = y; e[4] = u; e[5] = z;
          int32_t* sp = P.steps + 4 * st;
          sp[0] = f1; sp[1] = x; sp[2] = y; sp[3] = z;
          P.step_gain[st] = unord_f32(r.x);
          bits[u >> 5] |= 1u << (u & 31);
          int t0_ = u, t1_ = x, t2_ = y;
          sort3(t0_, t1_, t2_);
          work[0] = Work{f1, t0_, t1_, t2_, 0, 0};
          t0_ = u; t1_ = y; t2_ = z;
          sort3(t0_, t1_, t2_);
          work[1] = Work{F, t0_, t1_, t2_, 0, 0};
          t0_ = u; t1_ = x; t2_ = z;
          sort3(t0_, t1_, t2_);
          work[2] = Work{F + 1, t0_, t1_, t2_, 0, 0};
          s_ins = ins + 1;
          s_u4[0] = u;
          s_u4[1] = x;
          s_u4[2] = y;
          s_u4[3] = z;
          s_F = F + 2;
          s_nwork = 3;
          s_nnew = 3;
          sel[0] = f1 >> 6;
          sel[1] = F >> 6;       // F is even, so F and F + 1 share a chunk
          // u's bit and the four rows are written: the advancing waves may start
          __hip_atomic_store(&s_adv, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        // The chunks of the three new faces are reloaded. Faces whose cached vertex was u
        // are stale now; the chunks whose maximum is stale and ranks above the best fresh
        // record that remains are loaded too, and every stale record in them ranked above
        // that floor is recomputed along with the new faces.
        const int c1 = f1 >> 6, c2 = F >> 6;
        int ns = c2 != c1 ? 2 : 1;
        uint64_t kf2 = ~0ull;
        if (ins + 1 < n) {
#pragma unroll
          for (int i = 0; i < CI; ++i)
            if ((klo[i] & 0xffffu) == (uint32_t)u) insm |= 1u << i;
          kf2 = 0;
#pragma unroll
          for (int i = 0; i < CI; ++i) {
            const uint64_t k = ((uint64_t)khi[i] << 32) | klo[i];
            kf2 = ((insm >> i) & 1u) ? kf2 : max64(kf2, k);
          }
          kf2 = wave_max_dpp(kf2);
          if (Paper) {
            uint64_t rest = 0;
            ns = pick_top_stale_chunks(khi, klo, insm, LL.nchunk, kf2, c1, c2, sel, ns, sl_lane, &rest);
            if (lane == 0) s_unloaded = s_rest = rest;
          } else {
            ns = append_stale_chunks(khi, klo, insm, LL.nchunk, kf2, c1, c2, sel, ns, sl_lane);
          }
        }
        if (lane == 0) {
          s_nsel = ns;
          s_floor = kf2;
          s_since_insert = 0;
        }
      } else if (k1 == 0 || s_since_insert + 1 > nf + 8) {
        if (lane == 0) {
          *P.status = 8;
          s_stop = 1;
          s_nwork = 0;
          s_nnew = 0;
          s_nsel = 0;
          __hip_atomic_store(&s_adv, 2, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
      } else {
        // Stale maximum: load every chunk whose maximum is stale and ranks above the best
        // fresh record (the top one first) and recompute their stale records above it.
        const int c1 = f1 >> 6;
        if (Stats && lane == 0) s_cnt[16] += 1;
        if (lane == 0) sel[0] = c1;
        uint64_t rest = 0;
        const int ns = Paper ? pick_top_stale_chunks(khi, klo, insm, LL.nchunk, kf, c1, c1, sel, 1, sl_lane, &rest)
                             : append_stale_chunks(khi, klo, insm, LL.nchunk, kf, c1, c1, sel, 1, sl_lane);
        if (lane == 0) {
          __hip_atomic_store(&s_adv, 2, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
          s_nsel = ns;
          s_floor = kf;
          s_nwork = 0;
          s_nnew = 0;
          s_since_insert += 1;
          if (Paper) {
            // the top record is recomputed and committed first, whatever else fits
            const uint4 r = cmax[c1];
            work[0] = Work{f1, (int)(r.z & 0xffffu), (int)(r.z >> 16), (int)r.w, 0, 0};
            s_nwork = 1;
            s_nnew = 1;
            if (Stats) s_cnt[0] += 1;
            s_unloaded = s_rest = rest;
          }
        }
      }
    } else if (wave >= kWaves - (multi ? 1 : 4)) {
      // The new faces share the new vertex u, whose row no walk has read (a vertex is a face
      // corner only once inserted): its position is 0 while its most similar vertices (its
      // cluster) are mostly inserted already. The new faces' walks, usually the deepest of the
      // next phase, would each cross that stretch. Once the selection above has named u (a
      // bounded wait; past the bound nothing is done, which changes no result), the last wave
      // moves u's row position to its first uninserted entry, beside the rest of the
      // selection, unless the last walk step did so already (no vertex has been inserted
      // since, and u's own insertion changes nothing in its row). After a single-wave
      // selection, three more waves do the same for the corners of the face u split; after a
      // four-wave one that step would end the selection later than it shortens the walks.
      int st = 0;
      for (int it = 0; it < 8192 && st == 0; ++it) {
        st = __hip_atomic_load(&s_adv, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (st == 0) __builtin_amdgcn_s_sleep(1);
      }
      if (st == 1 || st >= kAdvRow) {
        const int v = st == 1 ? s_u4[kWaves - 1 - wave] : st - kAdvRow;
        if (wave != kWaves - 1 || v != s_pre) advance_row(P.idx, (int)P.ldi, bits, ptr, v, s_m, n, lane);
        // the word described the bits before this insertion
        if (wave == kWaves - 1 && lane == 0) s_pre = -1;
      }
    }
    __syncthreads();
    TMFG_LAP(5);
  }
#undef TMFG_LAP

  // Final faces, ascending triples in face-id order.
  __syncthreads();
  for (int f = tid; f < nf; f += kBlock) {
    const uint4 r = P.frec[f];
    P.faces[3 * f] = (int)(r.z & 0xffffu);
    P.faces[3 * f + 1] = (int)(r.z >> 16);
    P.faces[3 * f + 2] = (int)r.w;
  }
  __syncthreads();
  if (tid == 0) {
    if (!s_stop) *P.status = 0;
    if (Stats && P.stats) {
      for (int i = 0; i < 16; ++i) {
        const unsigned long long v = (i == 10) ? s_tbase + (clock_ticks() - t_start) : s_cnt[i];
        P.stats[i] = (int32_t)(v > 0x7fffffffull ? 0x7fffffffull : v);
      }
      for (int i = 0; i < 4; ++i) P.stats[16 + i] = (int32_t)(s_wt[i] > 0x7fffffffull ? 0x7fffffffull : s_wt[i]);
      for (int i = 0; i < 4; ++i) P.stats[20 + i] = (int32_t)(s_cnt[16 + i] > 0x7fffffffull ? 0x7fffffffull : s_cnt[16 + i]);
      P.stats[24] = s_compactions;
      for (int i = 25; i < 32; ++i) P.stats[i] = 0;
    }
  }
  if (P.hout.order)
    publish_outputs(P.hout, P.order, P.edges, P.steps, P.step_gain, P.faces, n, s_stop ? 8 : 0);
}

template <bool Paper, int CI, bool Stats>
__global__ __launch_bounds__(kBlock) void tmfg_loop_kernel(LoopParams P) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  run_loop<Paper, CI, Stats>(P, smem);
}

// Batched form: persistent workgroups take instances, largest first, from a shared counter;
// each runs that instance's whole insertion loop. The counter is read by one thread and
// every workgroup ends when the list is used up.
template <bool Paper>
__global__ __launch_bounds__(kBlock) void batch_loop_kernel(const BatchJob* __restrict__ jobs,
                                                            const int* __restrict__ order, int count,
                                                            int* __restrict__ queue_head, int max_rounds) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  __shared__ int s_job;
  for (;;) {
    if (threadIdx.x == 0) s_job = atomicAdd(queue_head, 1);
    __syncthreads();
    const int q = s_job;
    __syncthreads();
    if (q >= count) break;
    const BatchJob& J = jobs[order[q]];
    LoopParams P;
    P.W = J.W;
    P.n = J.n;
    P.idx = J.idx;
    P.vals = J.vals;
    P.ldi = J.ldi;
    P.scores = J.scores;
    P.frec = J.frec;
    P.flags = J.flags;
    P.order = J.order;
    P.edges = J.edges;
    P.steps = J.steps;
    P.step_gain = J.step_gain;
    P.faces = J.faces;
    P.status = J.status;
    P.stats = nullptr;
    P.paper = Paper;
    P.prefix = 0;
    P.m = J.n - 1;
    P.stop_at = INT_MAX;
    P.resume = 0;
    P.state = nullptr;
    P.max_rounds = max_rounds;
    P.hout = J.hout;
    run_loop<Paper, kItersSmall, false>(P, smem);
    __syncthreads();
  }
}

size_t loop_lds_bytes(int n) { return lds_layout(n).total; }

hipError_t batch_loop_occupancy(int* per_cu, int n_max, bool paper) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(
      per_cu, paper ? (const void*)batch_loop_kernel<true> : (const void*)batch_loop_kernel<false>, kBlock,
      loop_lds_bytes(n_max));
}

hipError_t loop_init_attributes() {
  const void* ks[10] = {(const void*)tmfg_loop_kernel<false, kItersSmall, false>,
                        (const void*)tmfg_loop_kernel<true, kItersSmall, false>,
                        (const void*)tmfg_loop_kernel<false, kItersBig, false>,
                        (const void*)tmfg_loop_kernel<true, kItersBig, false>,
                        (const void*)tmfg_loop_kernel<false, kItersSmall, true>,
                        (const void*)tmfg_loop_kernel<true, kItersSmall, true>,
                        (const void*)tmfg_loop_kernel<false, kItersBig, true>,
                        (const void*)tmfg_loop_kernel<true, kItersBig, true>,
                        (const void*)batch_loop_kernel<false>,
                        (const void*)batch_loop_kernel<true>};
  for (const void* k : ks) {
    hipFuncAttributes a;
    hipError_t e = hipFuncGetAttributes(&a, k);
    if (e != hipSuccess) return e;
    if (a.sharedSizeBytes + loop_lds_bytes(kMaxN) > (size_t)kLdsBytes) return hipErrorInvalidConfiguration;
    e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(kLdsBytes - a.sharedSizeBytes));
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_batch_loop(const BatchJob* jobs, const int* order, int count, int* queue_head, int grid,
                             int n_max, bool paper, int max_rounds, hipStream_t s) {
  const size_t lds = loop_lds_bytes(n_max);
  if (paper)
    hipLaunchKernelGGL(batch_loop_kernel<true>, dim3(grid), dim3(kBlock), lds, s, jobs, order, count, queue_head,
                       max_rounds);
  else
    hipLaunchKernelGGL(batch_loop_kernel<false>, dim3(grid), dim3(kBlock), lds, s, jobs, order, count, queue_head,
                       max_rounds);
  return hipGetLastError();
}

// Row compaction at a checkpoint of a single build, one workgroup per row (grid-stride): the
// uninserted entries of row x keep their order and move to positions [0, cnt); positions
// [cnt, m_new) take a filler entry (the first seed vertex, inserted from the start, with
// similarity -inf), so every row holds m_new = n - s entries after s insertions. Entries
// before the row's saved position are inserted, so the scan starts at its 8-aligned floor.
// All of a pass's loads complete before the barrier of its scan and its stores land below its
// own span, so the rows are rewritten in place. The row lengths and where the inserted bitmap
// and the row positions sit in the saved image come from the state header; nothing runs
// unless the loop stopped at a checkpoint.
constexpr int kCompactBlock = 256;
__global__ __launch_bounds__(kCompactBlock) void compact_rows_kernel(uint16_t* __restrict__ idx,
                                                                     float* __restrict__ vals, int n, int64_t ldi,
                                                                     const uint8_t* __restrict__ state,
                                                                     const int32_t* __restrict__ order) {
  const LoopStateHeader* hdr = (const LoopStateHeader*)state;
  if (!hdr->live) return;
  __shared__ uint32_t s_bits[(kMaxN + 31) / 32];
  __shared__ int s_wsum[kCompactBlock / kWave];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m_old = hdr->m_old, m_new = hdr->m_new;
  const uint8_t* img = state + kStateHeader;
  const uint32_t* bits = (const uint32_t*)(img + hdr->off_bits);
  const uint16_t* pos0 = (const uint16_t*)(img + hdr->off_ptr);
  for (int i = tid; i < (n + 31) / 32; i += kCompactBlock) s_bits[i] = bits[i];
  __syncthreads();
  const uint16_t filler = (uint16_t)order[0];
  for (int x = blockIdx.x; x < n; x += gridDim.x) {
    uint16_t* ri = idx + (size_t)x * ldi;
    float* rv = vals + (size_t)x * ldi;
    int out = 0;
    for (int base = (int)pos0[x] & ~7; base < m_old; base += kCompactBlock * 8) {
      const int p = base + tid * 8;            // a multiple of 8 below ldi when p < m_old
      uint4 iw = make_uint4(0xffffffffu, 0xffffffffu, 0xffffffffu, 0xffffffffu);
      float4 v0 = make_float4(0.f, 0.f, 0.f, 0.f), v1 = v0;
      if (p < m_old) {
        iw = *(const uint4*)(ri + p);
        v0 = *(const float4*)(rv + p);
        v1 = *(const float4*)(rv + p + 4);
      }
      const uint32_t wd[4] = {iw.x, iw.y, iw.z, iw.w};
      const float vv[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
      uint32_t keep = 0;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int u = (int)((wd[j >> 1] >> (16 * (j & 1))) & 0xffffu);
        keep |= open_entry(s_bits, u, n, p + j, 0, m_old) << j;
      }
      // exclusive prefix of the kept counts over the workgroup
      const int c = __popc(keep);
      int incl = c;
#pragma unroll
      for (int off = 1; off < kWave; off <<= 1) {
        const int t = __shfl_up(incl, off, kWave);
        incl += lane >= off ? t : 0;
      }
      if (lane == kWave - 1) s_wsum[wave] = incl;
      __syncthreads();
      int before = incl - c, total = 0;
#pragma unroll
      for (int w = 0; w < kCompactBlock / kWave; ++w) {
        before += w < wave ? s_wsum[w] : 0;
        total += s_wsum[w];
      }
      int o = out + before;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        if ((keep >> j) & 1u) {
          ri[o] = (uint16_t)((wd[j >> 1] >> (16 * (j & 1))) & 0xffffu);
          rv[o] = vv[j];
          ++o;
        }
      }
      out += total;
      __syncthreads();                         // s_wsum is reused
    }
    for (int q = out + tid; q < m_new; q += kCompactBlock) {
      ri[q] = filler;
      rv[q] = -INFINITY;
    }
  }
}

size_t loop_state_bytes(int n) {
  const size_t img = std::max(lds_layout(n).total, corr_lds_bytes(n));
  return kStateHeader + (img + 15) / 16 * 16;
}

// Inserted counts at which the rows are compacted: n - n/4, n - n/8, ... while at least
// kCompactMinLeft vertices remain uninserted. Early in a build most of a row's leading entries
// are uninserted and a walk finds its candidates at once; late, a walk crosses long inserted
// stretches (whole clusters sit between a row's head and its remaining vertices), and a
// compacted row holds only what is left. corr-tmfg inserts up to p vertices per round, so
// it stops at the first round boundary at or past each count.
constexpr int kCompactMinLeft = 128;
int loop_checkpoints(int n, int* s_out, int max) {
  int k = 0;
  for (int d = 4; k < max && n / d >= kCompactMinLeft; d *= 2) s_out[k++] = n - n / d;
  return k;
}

hipError_t launch_loop_compacting(LoopParams p, uint16_t* idx, float* vals, hipStream_t s) {
  int cp[16];
  const int nc = p.state ? loop_checkpoints(p.n, cp, 16) : 0;
  p.m = p.n - 1;
  p.resume = 0;
  p.stop_at = nc ? cp[0] : INT_MAX;
  auto segment = [&]() { return p.prefix > 0 ? launch_corr(p, s) : launch_loop(p, s); };
  hipError_t e = segment();
  for (int k = 0; k < nc && e == hipSuccess; ++k) {
    hipLaunchKernelGGL(compact_rows_kernel, dim3(p.n), dim3(kCompactBlock), 0, s, idx, vals, p.n, p.ldi,
                       (const uint8_t*)p.state, (const int32_t*)p.order);
    e = hipGetLastError();
    if (e != hipSuccess) break;
    p.resume = 1;
    p.stop_at = k + 1 < nc ? cp[k + 1] : INT_MAX;
    e = segment();
  }
  return e;
}

template <bool Stats>
static void launch_loop_as(const LoopParams& p, size_t lds, bool small, hipStream_t s) {
  if (p.paper && small)
    hipLaunchKernelGGL((tmfg_loop_kernel<true, kItersSmall, Stats>), dim3(1), dim3(kBlock), lds, s, p);
  else if (p.paper)
    hipLaunchKernelGGL((tmfg_loop_kernel<true, kItersBig, Stats>), dim3(1), dim3(kBlock), lds, s, p);
  else if (small)
    hipLaunchKernelGGL((tmfg_loop_kernel<false, kItersSmall, Stats>), dim3(1), dim3(kBlock), lds, s, p);
  else
    hipLaunchKernelGGL((tmfg_loop_kernel<false, kItersBig, Stats>), dim3(1), dim3(kBlock), lds, s, p);
}

hipError_t launch_loop(const LoopParams& p, hipStream_t s) {
  const size_t lds = loop_lds_bytes(p.n);
  // the chunk maxima of n vertices fit the smaller register layout up to n = 20480
  const bool small = chunk_iters(p.n) <= kItersSmall;
  if (p.stats)
    launch_loop_as<true>(p, lds, small, s);
  else
    launch_loop_as<false>(p, lds, small, s);
  return hipGetLastError();
}

}  // namespace tmfg
