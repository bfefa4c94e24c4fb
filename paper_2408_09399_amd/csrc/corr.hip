// corr-tmfg with a prefix size (Section 4.1, Algorithm 1): one persistent workgroup runs the
// rounds of one build on the device.
//
// Every face holds one pair: the best, by gain, of the MaxCorrs of its three corners (the
// first uninserted entry of each corner's sorted row). A round takes the p pairs of largest
// (gain, then lowest face id), keeps for each vertex only the first of its pairs among them,
// and applies the kept pairs in that order (three edges each, the face split in three, the
// new faces taking the next ids in turn). Then every face whose pair vertex was just inserted
// and every new face gets its pair again: the update is eager, so after a round no pair
// names an inserted vertex, and the order in which the pairs are recomputed does not matter.
// That makes a round's recomputations independent of each other, unlike the heap schedule
// of Algorithm 2, whose recomputations form a chain.
//
// Layout. Face records (16 B, the same format as the lazy loop's) live in global memory; in
// LDS sit the inserted bitmap, the per-vertex first-uninserted positions, the maximum key of
// every 64-face chunk, and the pair vertex of every face (0xffff: none, or being rebuilt).
// One round:
//   A  wave 0 takes the p chunks of largest maximum (the p best pairs lie in them), loads
//      their keys, picks the p best, drops repeated vertices, reads the kept faces' corners
//      and applies them; the new faces become work items;
//   S  every face whose pair vertex is inserted is found by a scan of the pair vertices and
//      becomes a work item (at most one per thread; more wait for another pass);
//   B  each work item's pair, one group of cGroup lanes per face;
//   P  records and pair vertices are published; the chunks they touch are marked;
//   R  the maxima of the touched chunks are rebuilt from their records.
#include <climits>

#include "common.h"
#include "facerule.h"
#include "internal.h"

namespace tmfg {

namespace {
constexpr int cBlock = 1024;
constexpr int cWaves = cBlock / kWave;
constexpr int cMaxWork = cBlock;                 // faces recomputed per pass, one per thread
constexpr int cMaxChunks = (2 * kMaxCorrN - 4 + 63) / 64;
constexpr int cChunkIters = (cMaxChunks + kWave - 1) / kWave;
constexpr uint16_t kNoVertex = 0xffff;
constexpr int cGroup = 8;                        // lanes per face pair (a half row)
constexpr int cLoads = 1;                        // 16-byte loads per lane and corner in a row scan
static_assert(kMaxPrefix <= kWave, "the prefix fits one wave's selection");
static_assert(kMaxPrefix <= cWaves, "one wave per chosen chunk");

struct CorrLds {
  int nchunk;
  size_t off_ckey, off_bits, off_ptr, off_fvert, total;
};
__host__ __device__ inline CorrLds corr_layout(int n) {
  CorrLds L;
  const int nf = 2 * n - 4;
  L.nchunk = (nf + 63) / 64;
  auto r16 = [](size_t b) { return (b + 15) / 16 * 16; };         // every array 16-byte aligned
  L.off_ckey = 0;                                                  // uint64[nchunk]
  L.off_bits = L.off_ckey + r16((size_t)L.nchunk * 8);             // uint32[(n + 31) / 32]
  L.off_ptr = L.off_bits + r16((size_t)((n + 31) / 32) * 4);       // uint16[n]
  L.off_fvert = L.off_ptr + r16((size_t)n * 2);                    // uint16[nf], padded to 8
  L.total = L.off_fvert + r16((size_t)nf * 2);
  return L;
}

struct CWork {
  int f, a, b, c;
  uint64_t best;
};
}  // namespace

// Stats records the counters and step timers of tmfg_plan_stats (P.stats is then set); a
// build that does not ask for them compiles them out.
template <bool Stats>
__device__ void run_corr(const LoopParams& P, uint8_t* smem) {
  __shared__ CWork work[cMaxWork];
  __shared__ int s_sel[kMaxPrefix];                // the round's chunks, in key order
  __shared__ uint64_t s_top[kMaxPrefix][kMaxPrefix];  // each chunk's best keys, in order
  __shared__ int s_ntop[kMaxPrefix], s_nsel;
  __shared__ int s_newu[kMaxPrefix], s_nnewu;        // the vertices the last round inserted
  __shared__ uint64_t s_list[kMaxPrefix];           // the round's best keys, in order
  __shared__ uint32_t s_touch[(cMaxChunks + 31) / 32];
  __shared__ int s_tlist[cMaxChunks];
  __shared__ int s_nwork, s_listed, s_more, s_ins, s_F, s_stop, s_next, s_ntouch, s_seed[4], s_compactions;
  __shared__ uint64_t s_part[cWaves];
  __shared__ int s_vpart[cWaves];
  // counters: [0] stale recomputes [1] row-scan trips [2] extra passes [3] rounds
  // [4..8] clock ticks in the scan, the pairs, publishing, rebuilding and selection
  __shared__ unsigned long long s_cnt[9];
  __shared__ unsigned long long s_t0;

  const int n = P.n, p = P.prefix;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int gl = lane & (cGroup - 1);
  const CorrLds LL = corr_layout(n);
  uint64_t* ckey = (uint64_t*)(smem + LL.off_ckey);
  uint32_t* bits = (uint32_t*)(smem + LL.off_bits);
  uint16_t* ptr = (uint16_t*)(smem + LL.off_ptr);
  uint16_t* fvert = (uint16_t*)(smem + LL.off_fvert);
  const int nf = 2 * n - 4;
  const int nw = (n + 31) / 32;
  const uint64_t t_start = wall_clock64();
  LoopStateHeader* hdr = (LoopStateHeader*)P.state;
  // entries per sorted row and the loop time of earlier segments, kept in LDS so that they
  // hold no registers in the loop
  __shared__ int s_m;
  __shared__ unsigned long long s_tbase;

  if (P.resume) {
    // A later segment has nothing to do when the build ended or stopped in an earlier one.
    // Every thread reads the flag before thread 0 clears it (after a barrier below).
    if (!hdr->live) return;
  } else {
    if (hdr && tid == 0) hdr->live = 0;
    const uint32_t fl = *P.flags;
    if (fl) {
      const int32_t st = (fl & kFlagNonFinite) ? 3 : (fl & kFlagAsymmetric) ? 4 : (fl & kFlagDegenerate) ? 5 : 8;
      if (tid == 0) *P.status = st;
      if (P.hout.order) publish_outputs(P.hout, P.order, P.edges, P.steps, P.step_gain, P.faces, n, st);
      return;
    }
  }

  for (int i = tid; i < (cMaxChunks + 31) / 32; i += cBlock) s_touch[i] = 0;
  if (tid < 9) s_cnt[tid] = P.resume ? hdr->cnt[tid] : 0;
  if (tid == 0) s_t0 = wall_clock64();
#define CORR_LAP(slot)                    \
  if (Stats && tid == 0) {                \
    const uint64_t t1_ = wall_clock64();  \
    s_cnt[slot] += t1_ - s_t0;            \
    s_t0 = t1_;                           \
  }

  if (P.resume) {
    // Resume at a round boundary: the LDS image comes back, every row position restarts at 0
    // (the rows were compacted since), and a first pass that finds nothing to recompute leads
    // to the next selection.
    const uint32_t* img = (const uint32_t*)(P.state + kStateHeader);
    for (int i = tid; i < (int)(LL.total / 4); i += cBlock) ((uint32_t*)smem)[i] = img[i];
    __syncthreads();
    for (int i = tid; i < n; i += cBlock) ptr[i] = 0;
    if (tid == 0) {
      s_nwork = 0;
      s_listed = 0;
      s_ins = hdr->ins;
      s_F = hdr->F;
      s_stop = 0;
      s_more = 0;
      s_next = 0;
      s_compactions = hdr->compactions;
      s_nnewu = 0;
      s_m = hdr->m_new;
      s_tbase = hdr->ticks;
      hdr->live = 0;
    }
    __syncthreads();
  } else {
    for (int i = tid; i < nf; i += cBlock) P.frec[i] = make_uint4(0, 0, 0, 0);
    for (int i = tid; i < LL.nchunk; i += cBlock) ckey[i] = 0;
    for (int i = tid; i < nw; i += cBlock) bits[i] = 0;
    for (int i = tid; i < n; i += cBlock) ptr[i] = 0;
    for (int i = tid; i < (int)((LL.total - LL.off_fvert) / 2); i += cBlock) fvert[i] = kNoVertex;
    seed_top4<cBlock>(P.scores, n, s_seed, s_part, s_vpart);
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
        work[f] = CWork{f, x, y, z, 0};
      }
      s_nwork = 4;
      s_listed = 4;
      s_ins = 4;
      s_F = 4;
      s_stop = 0;
      s_more = 0;
      s_next = 0;
      s_compactions = 0;
      s_nnewu = 0;
      s_m = P.m;
      s_tbase = 0;
    }
  }
  __syncthreads();

  for (;;) {
    const bool have_cand = s_ins < n;
    // ---- passes: the listed faces and every face whose pair vertex is inserted
    for (int pass = 0;; ++pass) {
      if (have_cand) {
        // The new faces of the round's vertices search those vertices' rows, which no pair
        // search has read (a vertex is a face corner only once inserted): their positions
        // are 0 while their most similar vertices are mostly inserted. In the first pass one
        // wave per new vertex moves its position to the first uninserted entry, 512 entries
        // per trip, beside the scan below.
        if (pass == 0 && wave < s_nnewu) {
          const int u = s_newu[wave];
          const uint16_t* row = P.idx + (size_t)u * P.ldi;
          const int ldi = (int)P.ldi, mr = s_m;
          int pu = ptr[u];
          for (;;) {
            const int qs = (pu & ~7) + lane * 8;
            const uint4 sv = *(const uint4*)(row + min(qs, ldi - 8));
            const uint32_t mk = open_mask8(bits, sv, n, qs, pu, mr);
            const int fp = mk ? qs + (int)__builtin_ctz(mk) : 0x7fffffff;
            const int f = wave_min_i32(fp);
            if (f != 0x7fffffff) {
              pu = f;
              break;
            }
            pu = (pu & ~7) + kWave * 8;
            if (pu >= mr) {
              pu = mr;
              break;
            }
          }
          if (lane == 0 && pu > (int)ptr[u]) ptr[u] = (uint16_t)pu;
        }
        // S: pair vertices, eight per 16-byte read; the matching faces' corners come from
        // their records
        const int F = s_F;
        for (int q = tid; q * 8 < F; q += cBlock) {
          const uint4 v8 = *(const uint4*)(fvert + 8 * q);
          const uint32_t wd[4] = {v8.x, v8.y, v8.z, v8.w};
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const int f = 8 * q + j;
            const int v = (int)((wd[j >> 1] >> (16 * (j & 1))) & 0xffffu);
            if (f < F && v != kNoVertex && is_ins(bits, v)) {
              const int slot = atomicAdd(&s_nwork, 1);
              if (slot < cMaxWork) {
                const uint4 r = P.frec[f];
                work[slot] = CWork{f, (int)(r.z & 0xffffu), (int)(r.z >> 16), (int)r.w, 0};
              } else {
                s_more = 1;
              }
            }
          }
        }
        __syncthreads();
        if (Stats && tid == 0) s_cnt[0] += (unsigned long long)((s_nwork < cMaxWork ? s_nwork : cMaxWork) - s_listed);
        CORR_LAP(4);
      }
      const int nwork = s_nwork < cMaxWork ? s_nwork : cMaxWork;
      // B: the pair of every listed face
      for (;;) {
        int base = 0;
        if (lane == 0) base = atomicAdd(&s_next, kWave / cGroup);
        base = __builtin_amdgcn_readfirstlane(base);
        if (base >= nwork) break;
        const int item = base + (lane / cGroup);
        if (item < nwork) {
          CWork& w = work[item];
          int trips = 0;
          const uint64_t best =
              have_cand ? paper_face<cGroup, cLoads>(P.W, P.idx, n, s_m, (int)P.ldi, bits, ptr, w.a, w.b, w.c, gl, &trips) : 0;
          if (gl == 0) {
            w.best = best;
            if (Stats) atomicAdd(&s_cnt[1], (unsigned long long)trips);
          }
        }
      }
      __syncthreads();
      CORR_LAP(5);
      // P: publish
      if (tid < nwork) {
        const CWork& w = work[tid];
        P.frec[w.f] = face_record(w.f, w.a, w.b, w.c, w.best);
        fvert[w.f] = w.best ? (uint16_t)(0xffffu - (uint32_t)(w.best & 0xffffu)) : kNoVertex;
        const int ch = w.f >> 6;
        atomicOr(&s_touch[ch >> 5], 1u << (ch & 31));
      }
      __syncthreads();
      CORR_LAP(6);
      // R: rebuild the touched chunks' maxima from their records
      if (wave == 0) {
        int cnt = 0;
        for (int i = 0; i < cChunkIters; ++i) {
          const int ch = lane + i * kWave;
          const bool t = ch < LL.nchunk && ((s_touch[ch >> 5] >> (ch & 31)) & 1u);
          const uint64_t msk = __ballot(t);
          if (t) s_tlist[cnt + (int)__popcll(msk & ((1ull << lane) - 1))] = ch;
          cnt += (int)__popcll(msk);
        }
        if (lane == 0) s_ntouch = cnt;
        for (int i = lane; i < (cMaxChunks + 31) / 32; i += kWave) s_touch[i] = 0;
      }
      if (tid == 0) {
        s_nwork = 0;
        s_listed = 0;
        s_next = 0;
      }
      __syncthreads();
      const int nt = s_ntouch;
      for (int j0 = wave; j0 < nt; j0 += 4 * cWaves) {
        uint4 r[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int j = j0 + u * cWaves;
          const int f = (j < nt ? s_tlist[j] : 0) * 64 + lane;
          r[u] = P.frec[f < nf ? f : nf - 1];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int j = j0 + u * cWaves;
          if (j >= nt) break;
          const int f = s_tlist[j] * 64 + lane;
          const uint64_t k = wave_max_dpp(f < nf ? rec_key(r[u]) : 0);
          if (lane == 0) ckey[s_tlist[j]] = k;
        }
      }
      const int more = s_more;
      __syncthreads();
      CORR_LAP(7);
      if (!more || !have_cand) break;
      if (pass > nf / cMaxWork + 2) {           // every pass clears up to cMaxWork faces
        if (tid == 0) {
          *P.status = 8;
          s_stop = 1;
        }
        __syncthreads();
        break;
      }
      if (tid == 0) {
        s_more = 0;
        s_cnt[2] += 1;
      }
      __syncthreads();
    }
    if (s_ins >= n || s_stop) break;
    if (s_ins >= P.stop_at) {
      // Checkpoint (single builds): every pair names an uninserted vertex and no face is
      // listed; save the state and return, and the rows are compacted before the next segment
      // resumes here.
      uint32_t* img = (uint32_t*)(P.state + kStateHeader);
      for (int i = tid; i < (int)(LL.total / 4); i += cBlock) img[i] = ((const uint32_t*)smem)[i];
      if (tid == 0) {
        hdr->ins = s_ins;
        hdr->F = s_F;
        hdr->since_insert = 0;
        hdr->compactions = s_compactions + 1;
        hdr->m_old = s_m;
        hdr->m_new = n - s_ins;
        hdr->off_bits = (int)LL.off_bits;
        hdr->off_ptr = (int)LL.off_ptr;
        hdr->ticks = s_tbase + (wall_clock64() - t_start);
        for (int i = 0; i < 9; ++i) hdr->cnt[i] = s_cnt[i];
        hdr->live = 1;
      }
      return;
    }

    // ---- A: the round's prefix
    // A1 (wave 0): the p chunks of largest maximum, in key order. The p best pairs lie in them:
    // a pair in any other chunk has p chunk maxima above it.
    if (wave == 0) {
      if (Stats && lane == 0) s_cnt[3] += 1;
      // the lane index is made opaque so that the chunk addresses are formed anew each round
      // rather than held in registers across the whole loop
      int sl_lane = lane;
      asm volatile("" : "+v"(sl_lane));
      uint64_t ck[cChunkIters];
      uint32_t cm = 0;
#pragma unroll
      for (int i = 0; i < cChunkIters; ++i) {
        const int ch = sl_lane + i * kWave;
        ck[i] = ch < LL.nchunk ? ckey[ch] : 0;
        cm |= ck[i] ? (1u << i) : 0u;
      }
      int nsel = 0;
      for (int s = 0; s < p; ++s) {
        uint64_t lm = 0;
        int li = 0;
#pragma unroll
        for (int i = 0; i < cChunkIters; ++i) {
          const bool c = ((cm >> i) & 1u) && ck[i] > lm;
          lm = c ? ck[i] : lm;
          li = c ? i : li;
        }
        const uint64_t g = wave_max_dpp(lm);
        if (g == 0) break;
        if (lm == g) {
          s_sel[nsel] = sl_lane + li * kWave;
          cm &= ~(1u << li);
        }
        ++nsel;
      }
      if (lane == 0) s_nsel = nsel;
    }
    __syncthreads();
    // A2 (one wave per chosen chunk): the chunk's p best record keys, in order. Keys are
    // unique (they hold the face id), so one lane matches each maximum.
    const int nsel = s_nsel;
    if (wave < nsel) {
      const int f = s_sel[wave] * 64 + lane;
      uint64_t k = f < nf ? rec_key(P.frec[f]) : 0;
      int cnt = 0;
      for (; cnt < p; ++cnt) {
        const uint64_t g = wave_max_dpp(k);
        if (g == 0) break;
        if (lane == 0) s_top[wave][cnt] = g;
        k = k == g ? 0 : k;
      }
      if (lane == 0) s_ntop[wave] = cnt;
    }
    __syncthreads();
    // A3 (wave 0): merge the chunks' lists into the round's p best keys, in order; a pair
    // whose vertex an earlier one has is dropped, and the kept pairs are applied in order,
    // one lane each.
    if (wave == 0) {
      const int nt = lane < nsel ? s_ntop[lane] : 0;
      int h = 0;
      uint64_t head = nt > 0 ? s_top[lane][0] : 0;
      int nlist = 0;
      for (; nlist < p; ++nlist) {
        const uint64_t g = wave_max_dpp(head);
        if (g == 0) break;
        if (lane == 0) s_list[nlist] = g;
        if (head == g) {
          ++h;
          head = h < nt ? s_top[lane][h] : 0;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
      const uint64_t mine = lane < nlist ? s_list[lane] : 0;
      const uint32_t u = (uint32_t)(mine & 0xffffu);
      bool keep = lane < nlist;
      for (int q = 0; q < nlist; ++q) keep = keep && !(q < lane && (uint32_t)(s_list[q] & 0xffffu) == u);
      const uint64_t kmask = __ballot(keep);
      const int nl = (int)__popcll(kmask);
      const int r = (int)__popcll(kmask & ((1ull << lane) - 1));
      const int ins0 = s_ins, F0 = s_F;
      bool bad = false;
      if (keep) {
        const int f = 0xffff - (int)((uint32_t)mine >> 16);
        const uint4 rec = P.frec[f];
        const int x = (int)(rec.z & 0xffffu), y = (int)(rec.z >> 16), z = (int)rec.w;
        const int ins = ins0 + r, F = F0 + 2 * r;
        // a pair naming an inserted vertex, or more pairs than vertices left: cannot happen
        bad = ins >= n || is_ins(bits, (int)u);
        if (!bad) {
          const int st = ins - 4;
          P.order[ins] = (int)u;
          int32_t* e = P.edges + 2 * (6 + 3 * st);
          e[0] = (int)u; e[1] = x; e[2] = (int)u; e[3] = y; e[4] = (int)u; e[5] = z;
          int32_t* sp = P.steps + 4 * st;
          sp[0] = f; sp[1] = x; sp[2] = y; sp[3] = z;
          P.step_gain[st] = unord_f32(rec.x);
          fvert[f] = kNoVertex;
          int t0 = (int)u, t1 = x, t2 = y;
          sort3(t0, t1, t2);
          work[3 * r] = CWork{f, t0, t1, t2, 0};
          t0 = (int)u; t1 = y; t2 = z;
          sort3(t0, t1, t2);
          work[3 * r + 1] = CWork{F, t0, t1, t2, 0};
          t0 = (int)u; t1 = x; t2 = z;
          sort3(t0, t1, t2);
          work[3 * r + 2] = CWork{F + 1, t0, t1, t2, 0};
        }
      }
      const bool any_bad = __ballot(bad) != 0;
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
      if (keep && !bad) {
        atomicOr(&bits[u >> 5], 1u << (u & 31));
        s_newu[r] = (int)u;
      }
      if (lane == 0) {
        s_nnewu = any_bad ? 0 : nl;
        if (nl == 0 || any_bad) {
          *P.status = 8;                   // no pair while vertices are left: cannot happen
          s_stop = 1;
        }
        s_ins = ins0 + nl;
        s_F = F0 + 2 * nl;
        s_nwork = 3 * nl;
        s_listed = 3 * nl;
      }
    }
    __syncthreads();
    CORR_LAP(8);
    if (s_stop) break;
  }
#undef CORR_LAP

  __syncthreads();
  for (int f = tid; f < nf; f += cBlock) {
    const uint4 r = P.frec[f];
    P.faces[3 * f] = (int)(r.z & 0xffffu);
    P.faces[3 * f + 1] = (int)(r.z >> 16);
    P.faces[3 * f + 2] = (int)r.w;
  }
  __syncthreads();
  if (tid == 0) {
    if (!s_stop) *P.status = 0;
    if (Stats && P.stats) {
      for (int i = 0; i < 32; ++i) P.stats[i] = 0;
      P.stats[0] = (int32_t)(s_cnt[0] > 0x7fffffffull ? 0x7fffffffull : s_cnt[0]);
      P.stats[1] = (int32_t)(s_cnt[1] > 0x7fffffffull ? 0x7fffffffull : s_cnt[1]);
      P.stats[2] = (int32_t)s_cnt[2];
      P.stats[3] = (int32_t)s_cnt[3];
      for (int i = 0; i < 5; ++i) P.stats[5 + i] = (int32_t)(s_cnt[4 + i] > 0x7fffffffull ? 0x7fffffffull : s_cnt[4 + i]);
      const unsigned long long t = s_tbase + (wall_clock64() - t_start);
      P.stats[10] = (int32_t)(t > 0x7fffffffull ? 0x7fffffffull : t);
      P.stats[24] = s_compactions;
    }
  }
  if (P.hout.order)
    publish_outputs(P.hout, P.order, P.edges, P.steps, P.step_gain, P.faces, n, s_stop ? 8 : 0);
}

template <bool Stats>
__global__ __launch_bounds__(cBlock) void tmfg_corr_kernel(LoopParams P) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  run_corr<Stats>(P, smem);
}

// Batched form: as the lazy loop's, persistent workgroups take instances largest first.
__global__ __launch_bounds__(cBlock) void batch_corr_kernel(const BatchJob* __restrict__ jobs,
                                                            const int* __restrict__ order, int count,
                                                            int* __restrict__ queue_head, int prefix) {
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
    P.paper = false;
    P.prefix = prefix;
    P.m = J.n - 1;
    P.stop_at = INT_MAX;
    P.resume = 0;
    P.state = nullptr;
    P.max_rounds = kWalkRounds;
    P.hout = J.hout;
    run_corr<false>(P, smem);
    __syncthreads();
  }

}

size_t corr_lds_bytes(int n) { return corr_layout(n).total; }

hipError_t corr_init_attributes() {
  const void* ks[3] = {(const void*)tmfg_corr_kernel<false>, (const void*)tmfg_corr_kernel<true>,
                       (const void*)batch_corr_kernel};
  for (const void* k : ks) {
    hipFuncAttributes a;
    hipError_t e = hipFuncGetAttributes(&a, k);
    if (e != hipSuccess) return e;
    if (a.sharedSizeBytes + corr_lds_bytes(kMaxCorrN) > (size_t)kLdsBytes) return hipErrorInvalidConfiguration;
    e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(kLdsBytes - a.sharedSizeBytes));
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t batch_corr_occupancy(int* per_cu, int n_max) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, batch_corr_kernel, cBlock, corr_lds_bytes(n_max));
}

hipError_t launch_corr(const LoopParams& p, hipStream_t s) {
  if (p.stats)
    hipLaunchKernelGGL(tmfg_corr_kernel<true>, dim3(1), dim3(cBlock), corr_lds_bytes(p.n), s, p);
  else
    hipLaunchKernelGGL(tmfg_corr_kernel<false>, dim3(1), dim3(cBlock), corr_lds_bytes(p.n), s, p);
  return hipGetLastError();
}

hipError_t launch_batch_corr(const BatchJob* jobs, const int* order, int count, int* queue_head, int grid,
                             int n_max, int prefix, hipStream_t s) {
  hipLaunchKernelGGL(batch_corr_kernel, dim3(grid), dim3(cBlock), corr_lds_bytes(n_max), s, jobs, order, count,
                     queue_head, prefix);
  return hipGetLastError();
}

}  // namespace tmfg
