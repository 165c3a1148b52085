// search.hpp -- the witness-path search of one source by one group of G
// lanes (Alg. 4, "Step 1: Local Search with Memoization").
//
// For a source s in V_W the group
//   1. gathers the target set V_n: every out-neighbour v != s of every
//      affected out-neighbour u of s (u in V_A) whose pair (s, v) is not in
//      the memo, and the radius D_s = the largest w(s,u) + w(u,v) over the
//      gathered pairs;
//   2. computes the exact overlay distance from s to every vertex within
//      radius D_s by label-correcting relaxation (frontier lists and a
//      vertex -> distance hash in a per-group table);
//   3. writes dist(s, v) into the memo for every target.
// Every target's distance is at most its own two-arc length, so radius D_s
// returns exact values, and those values do not depend on the relaxation
// order.  The table lives in LDS (fast path) or in global memory (the
// fallback for searches that outgrow LDS); `GL` selects the accessors.
#pragma once

#include "common.hpp"

namespace sp {

struct Overlay {
  uint32_t n;
  uint32_t m;
  const uint32_t *foff;  // n+1
  uint2 *farc;           // m: {head, weight}; weight SP_INF32 marks a pruned arc
  uint32_t *fmid;        // m: middle vertex (original id) or SP_NOMID
  const uint32_t *roff;  // n+1
  uint2 *rarc;           // m: {tail, weight}
  uint32_t *rmid;        // m
  const uint32_t *gid;   // n: original id of each local vertex
};

enum : int { kCtrUsed = 0, kCtrF0 = 1, kCtrF1 = 2, kCtrOvf = 3 };
// Witness-search modes (the values of CH_WPS_EXACT, CH_WPS_HOP, CH_WPS_SETTLED).
enum : int { kWpsExact = 0, kWpsHop = 1, kWpsSettled = 2 };

template <typename IdxT, bool GL>
struct Tab {
  uint32_t *key;   // vertex (local id) or SP_EMPTY32
  uint32_t *dist;  // tentative distance; during target collection 0xFFFFFFFF - max via
  uint32_t *dist2; // hop mode: the distances of the level being computed (else null)
  uint32_t *tgt;   // bitmap: slot holds a target
  uint32_t *front; // bitmap: slot is in the next frontier list
  IdxT *order;     // slots in insertion order (limit entries)
  IdxT *fr0, *fr1; // frontier slot lists (fcap entries each)
  uint32_t *ctr;   // used, |fr0|, |fr1|, overflow
  uint32_t cap;    // power of two
  uint32_t shift;  // 32 - log2(cap)
  uint32_t limit;  // overflow when more slots than this are used
  uint32_t fcap;   // frontier list capacity (>= limit)

  __device__ __forceinline__ uint32_t ld(const uint32_t *p) const {
    if constexpr (GL) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else return *p;
  }
  __device__ __forceinline__ void st(uint32_t *p, uint32_t v) const {
    if constexpr (GL) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else *p = v;
  }
  __device__ __forceinline__ IdxT ldi(const IdxT *p) const {
    if constexpr (GL) return (IdxT)__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else return *p;
  }
  __device__ __forceinline__ void sti(IdxT *p, IdxT v) const {
    if constexpr (GL) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else *p = v;
  }
  __device__ __forceinline__ void sync() const {
    if constexpr (GL) __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "agent");
    wave_sync();
  }

  // Find or insert vertex v; returns its slot or -1 when the table is full.
  __device__ __forceinline__ int insert(uint32_t v) const {
    uint32_t h = (v * 0x9E3779B1u) >> shift;
    for (uint32_t probes = 0; probes < cap; probes++) {
      uint32_t k = ld(&key[h]);
      if (k == v) return (int)h;
      if (k == SP_EMPTY32) {
        uint32_t prev = atomicCAS(&key[h], SP_EMPTY32, v);
        if (prev == SP_EMPTY32) {
          uint32_t idx = atomicAdd(&ctr[kCtrUsed], 1u);
          if (idx < limit) sti(&order[idx], (IdxT)h);
          else atomicOr(&ctr[kCtrOvf], 1u);
          return (int)h;
        }
        if (prev == v) return (int)h;
      }
      h = (h + 1) & (cap - 1);
    }
    atomicOr(&ctr[kCtrOvf], 1u);
    return -1;
  }
};

// Arcs of up to G rows spread over the group: row r of lane r holds rl arcs
// from farc[rs]; entry idx (< total, the sum of rl) belongs to the first lane
// whose inclusive prefix `incl` exceeds it.  arc_batch<G>() entries per lane are
// loaded before any is used (one latency per batch instead of per entry);
// f(arc, aux of the owning row) runs for each, then the group syncs.
// Wide groups read long rows (dense overlays); narrow groups keep their
// registers for occupancy.
template <int G>
constexpr int arc_batch() { return G >= 64 ? 8 : 4; }
template <int G>
constexpr int memo_batch() { return G >= 32 ? kPairBatch : 2; }

template <int G, typename IdxT, bool GL, typename Fn>
__device__ __forceinline__ void for_row_arcs(const Tab<IdxT, GL> &T, const uint2 *__restrict__ farc,
                                             uint32_t incl, uint32_t rs, uint32_t rl,
                                             uint32_t aux, uint32_t total, Fn f) {
  constexpr int kArcBatch = arc_batch<G>();
  const int gl = glane<G>();
  for (uint32_t i0 = 0; i0 < total; i0 += G * kArcBatch) {
    uint2 b[kArcBatch];
    uint32_t sa[kArcBatch];
#pragma unroll
    for (int u = 0; u < kArcBatch; u++) {
      const uint32_t idx = i0 + u * G + gl;
      b[u] = make_uint2(SP_EMPTY32, 0u);
      sa[u] = 0;
      if (i0 + u * G < total) {  // uniform across the group
        const int src = gfind<G>(incl, idx);
        const uint32_t srs = gshfl<G>(rs, src), sinc = gshfl<G>(incl, src);
        const uint32_t srl = gshfl<G>(rl, src);
        sa[u] = gshfl<G>(aux, src);
        if (idx < total) b[u] = farc[srs + (idx - (sinc - srl))];
      }
    }
#pragma unroll
    for (int u = 0; u < kArcBatch; u++)
      if (b[u].x != SP_EMPTY32) f(b[u], sa[u]);
    T.sync();
    if (T.ld(&T.ctr[kCtrOvf])) break;
  }
}

struct SearchStats {
  uint32_t rows = 0, arcs = 0, probes = 0, inserts = 0, targets = 0, searched = 0;
};

// A search is run by NW waves of one block together (NW > 1, G = 64: the
// block-wide tiers for searches that outgrow a wave's table) or by one group
// of G lanes (NW = 1).  Collective loops stride over all NT = G * NW lanes;
// row expansion stays per wave (for_row_arcs), so waves never wait on each
// other inside a level.  Coop holds this lane's place and a small LDS array
// for reductions across the waves.
template <int G, int NW>
struct Coop {
  static constexpr int NT = G * NW;
  uint32_t *red;  // 2 * NW words of LDS (NW > 1)
  __device__ __forceinline__ int tl() const {
    if constexpr (NW == 1) return glane<G>();
    else return (int)threadIdx.x;
  }
  __device__ __forceinline__ int wv() const {
    if constexpr (NW == 1) return 0;
    else return (int)(threadIdx.x / kWave);
  }
  // barrier of the lanes that share the search (and the table's fence)
  template <typename TabT>
  __device__ __forceinline__ void sync(const TabT &T) const {
    if constexpr (NW == 1) {
      T.sync();
    } else {
      T.sync();
      __syncthreads();
    }
  }
  template <typename TabT>
  __device__ __forceinline__ uint32_t sum(uint32_t v, const TabT &T) const {
    v = gsum<G>(v);
    if constexpr (NW > 1) {
      if (lane_id() == 0) red[wv()] = v;
      __syncthreads();
      v = 0;
#pragma unroll
      for (int i = 0; i < NW; i++) v += red[i];
      __syncthreads();
    }
    return v;
  }
  // minimum of a 64-bit key over the lanes (uses red as NW 64-bit words)
  template <typename TabT>
  __device__ __forceinline__ uint64_t min64(uint64_t v, const TabT &T) const {
    v = gmin64<G>(v);
    if constexpr (NW > 1) {
      uint64_t *r = reinterpret_cast<uint64_t *>(red);
      if (lane_id() == 0) r[wv()] = v;
      __syncthreads();
      v = r[0];
#pragma unroll
      for (int i = 1; i < NW; i++) v = r[i] < v ? r[i] : v;
      __syncthreads();
    }
    return v;
  }
  // x of the one lane with `mine` set (exactly one lane of the search has it)
  template <typename TabT>
  __device__ __forceinline__ uint32_t pick(uint32_t x, bool mine, const TabT &T) const {
    if constexpr (NW == 1) {
      const uint64_t b = gballot<G>(mine);
      return gshfl<G>(x, b ? __builtin_ctzll(b) : 0);
    } else {
      if (mine) red[0] = x;
      __syncthreads();
      x = red[0];
      __syncthreads();
      return x;
    }
  }
  template <typename TabT>
  __device__ __forceinline__ uint32_t max(uint32_t v, const TabT &T) const {
    v = gmax<G>(v);
    if constexpr (NW > 1) {
      if (lane_id() == 0) red[NW + wv()] = v;
      __syncthreads();
      v = 0;
#pragma unroll
      for (int i = 0; i < NW; i++) v = v > red[NW + i] ? v : red[NW + i];
      __syncthreads();
    }
    return v;
  }
};

// Clears the slots listed in `order` (and the counters) after a search.
template <int G, int NW, typename IdxT, bool GL>
__device__ __forceinline__ void tab_reset(const Tab<IdxT, GL> &T, const Coop<G, NW> &C) {
  constexpr int NT = Coop<G, NW>::NT;
  const int tl = C.tl();
  C.sync(T);
  uint32_t used = T.ld(&T.ctr[kCtrUsed]);
  if (used > T.limit) used = T.limit;
  for (uint32_t i = tl; i < used; i += NT) {
    IdxT s = T.ldi(&T.order[i]);
    T.st(&T.key[s], SP_EMPTY32);
    T.st(&T.dist[s], SP_INF32);
    if (T.dist2) T.st(&T.dist2[s], SP_INF32);
  }
  for (uint32_t i = tl; i < T.cap / 32; i += NT) {
    T.st(&T.tgt[i], 0u);
    T.st(&T.front[i], 0u);
  }
  C.sync(T);
  if (used >= T.limit) {  // an overflowing insert may have left unlisted keys
    for (uint32_t i = tl; i < T.cap; i += NT) {
      T.st(&T.key[i], SP_EMPTY32);
      T.st(&T.dist[i], SP_INF32);
      if (T.dist2) T.st(&T.dist2[i], SP_INF32);
    }
  }
  if (tl < 4) T.st(&T.ctr[tl], 0u);
  C.sync(T);
}

// Steps 2 and 3 of the settled(theta) mode (the paper's literal bound, Alg.
// 4: a search stops once theta vertices are settled or once every target
// is): Dijkstra from s that settles one vertex per step, the open vertex with
// the smallest (distance, label) found by a min-reduction over the table;
// s is the first settled vertex.  Only settled vertices are relaxed from and
// only settled targets get a memo entry.  dist2 holds each slot's label, the
// frontier bitmap marks settled slots; `hops` is theta.
template <int G, int NW, typename IdxT, bool GL>
__device__ bool settled_search(const Overlay &ov, const MemoRef &memo, const Tab<IdxT, GL> &T,
                               uint32_t s, uint32_t gs, uint32_t D, uint32_t nt, SearchStats &ss,
                               uint32_t *__restrict__ ws, uint32_t theta, const Coop<G, NW> &C,
                               const uint32_t *__restrict__ label) {
  constexpr int NT = Coop<G, NW>::NT;
  const int tl = C.tl();
  C.sync(T);
  if (tl == 0) {
    const int slot = T.insert(s);
    if (slot >= 0) {
      T.st(&T.dist[slot], 0u);
      T.st(&T.dist2[slot], label[gs]);
    }
  }
  C.sync(T);
  uint32_t pops = 0, tdone = 0;
  while (pops < theta && tdone < nt && !T.ld(&T.ctr[kCtrOvf])) {
    const uint32_t used = min(T.ld(&T.ctr[kCtrUsed]), T.limit);
    uint64_t mk = ~0ull;
    uint32_t mslot = 0;
    for (uint32_t i = tl; i < used; i += NT) {
      const IdxT slot = T.ldi(&T.order[i]);
      if ((T.ld(&T.front[slot >> 5]) >> (slot & 31)) & 1u) continue;  // settled
      const uint32_t d = T.ld(&T.dist[slot]);
      if (d == SP_INF32) continue;
      const uint64_t k = ((uint64_t)d << 32) | T.ld(&T.dist2[slot]);
      if (k < mk) {
        mk = k;
        mslot = slot;
      }
    }
    const uint64_t best = C.min64(mk, T);
    if (best == ~0ull) break;  // nothing left to settle
    // labels are distinct, so exactly one lane holds the minimum
    const uint32_t bs = C.pick(mslot, mk == best, T);
    const uint32_t d = (uint32_t)(best >> 32);
    const bool is_tgt = (T.ld(&T.tgt[bs >> 5]) >> (bs & 31)) & 1u;
    const uint32_t x = T.ld(&T.key[bs]);
    C.sync(T);
    if (tl == 0) {
      atomicOr(&T.front[bs >> 5], 1u << (bs & 31));
      ss.rows++;
    }
    pops++;
    tdone += is_tgt ? 1u : 0u;
    const uint32_t a0 = ov.foff[x], a1 = ov.foff[x + 1];
    for (uint32_t e = a0 + tl; e < a1; e += NT) {
      const uint2 b = ov.farc[e];
      ss.arcs++;
      const uint64_t nd = (uint64_t)d + b.y;
      if (nd > D) continue;
      const int y = T.insert(b.x);
      if (y < 0) continue;
      if ((T.ld(&T.front[y >> 5]) >> (y & 31)) & 1u) continue;  // settled
      const uint32_t old = atomicMin(&T.dist[y], (uint32_t)nd);
      if ((uint32_t)nd < old) T.st(&T.dist2[y], label[ov.gid[b.x]]);
    }
    C.sync(T);
  }
  C.sync(T);
  if (T.ld(&T.ctr[kCtrOvf])) {
    tab_reset(T, C);
    return false;
  }
  ss.targets += (tl == 0) ? nt : 0;
  ss.searched += (tl == 0) ? 1 : 0;
  {
    const uint32_t used = T.ld(&T.ctr[kCtrUsed]);
    for (uint32_t i = tl; i < used; i += NT) {
      const IdxT slot = T.ldi(&T.order[i]);
      const bool tg = (T.ld(&T.tgt[slot >> 5]) >> (slot & 31)) & 1u;
      const bool st = (T.ld(&T.front[slot >> 5]) >> (slot & 31)) & 1u;
      if (tg && st) {
        memo_put(memo, gs, ov.gid[T.ld(&T.key[slot])], T.ld(&T.dist[slot]));
        ss.inserts++;
      }
    }
    if (ws && tl == 0) ws[gs] = pops;
  }
  tab_reset(T, C);
  return true;
}

// Exact mode: distance-bucket shift of a search step (the default of
// ch_params_t.ls_step); 32 expands the whole frontier every step.
constexpr uint32_t kLsStepDefault = 2;

// One source.  Returns false when the table overflowed (nothing written).
// Exact mode, wave-wide groups (G = 64): a step expands the frontier
// vertices whose distance is below the smallest frontier distance plus
// D >> `hops` (the bucket shift; 32 = the whole frontier); the others stay
// in the frontier for a later step.  Narrow groups run the small searches of
// sparse rounds, where the extra reduction per step costs more than it saves
// (road-like 24M: 137 -> 152 ms per build in the 16-lane kernel), so they
// expand the whole frontier.
// Expanding near vertices first re-expands fewer vertices whose distance
// drops later; the result is the same for every shift (every tentative value
// is a path length and the search ends only when no distance can drop).
// HOP: hop-synchronous search of at most `hops` levels -- level k expands
// the vertices whose distance changed in level k-1 with their level-(k-1)
// distance (dist) and writes dist2; at the end of the level the changed
// entries are copied back.  The result is the minimum over walks of at most
// `hops` arcs within the radius, independent of the order of relaxations.
// Targets the walks do not reach get no memo entry.
template <int G, int NW, int M, typename IdxT, bool GL>
__device__ bool search_source(const Overlay &ov, const uint8_t *__restrict__ aflag,
                              const MemoRef &memo, const Tab<IdxT, GL> &T, uint32_t s, SearchStats &ss,
                              uint32_t *__restrict__ ws, uint32_t *__restrict__ err,
                              uint32_t hops, const Coop<G, NW> &C,
                              const uint32_t *__restrict__ label) {
  static_assert(NW == 1 || G == kWave, "cooperating waves use whole waves");
  constexpr bool HOP = M == kWpsHop, SET = M == kWpsSettled;
  constexpr int NT = Coop<G, NW>::NT;
  const int gl = glane<G>();
  const int tl = C.tl();
  const uint32_t wbase = (uint32_t)C.wv() * G;  // this wave's first lane in the search
  const uint32_t gs = ov.gid[s];

  // ---- 1. targets and radius ------------------------------------------
  const uint32_t a0 = ov.foff[s], a1 = ov.foff[s + 1];
  for (uint32_t base = a0 + wbase; base < a1; base += NT) {
    const uint32_t e = base + gl;
    uint32_t rs = 0, rl = 0, wsu = 0;
    if (e < a1) {
      const uint2 a = ov.farc[e];
      if (aflag[a.x]) {
        rs = ov.foff[a.x];
        rl = ov.foff[a.x + 1] - rs;
        wsu = a.y;
        ss.rows++;
      }
    }
    const uint32_t incl = gscan_incl<G>(rl);
    const uint32_t total = gshfl<G>(incl, G - 1);
    for_row_arcs<G>(T, ov.farc, incl, rs, rl, wsu, total, [&](uint2 b, uint32_t sw) {
      ss.arcs++;
      if (b.x != s) {
        const uint64_t via = (uint64_t)sw + b.y;
        const uint32_t viac = via > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)via;
        const int slot = T.insert(b.x);
        if (slot >= 0) atomicMin(&T.dist[slot], 0xFFFFFFFFu - viac);
      }
    });
    if (T.ld(&T.ctr[kCtrOvf])) break;
  }
  C.sync(T);
  if (T.ld(&T.ctr[kCtrOvf])) {
    tab_reset(T, C);
    return false;
  }
  uint32_t D = 0, nt = 0;
  {
    constexpr int K = memo_batch<G>();
    const uint32_t used = T.ld(&T.ctr[kCtrUsed]);
    for (uint32_t i0 = tl; i0 < used; i0 += NT * K) {
      IdxT slot[K];
      uint32_t ks[K], kv[K], got[K];
      bool act[K];
#pragma unroll
      for (int q = 0; q < K; q++) {
        const uint32_t i = i0 + q * NT;
        act[q] = i < used;
        slot[q] = act[q] ? T.ldi(&T.order[i]) : (IdxT)0;
        ks[q] = gs;
        kv[q] = act[q] ? ov.gid[T.ld(&T.key[slot[q]])] : 0u;
      }
      memo_get_batch<K>(memo, ks, kv, act, got, &ss.probes);
#pragma unroll
      for (int q = 0; q < K; q++) {
        if (!act[q]) continue;
        if (got[q] == SP_INF32) {
          atomicOr(&T.tgt[slot[q] >> 5], 1u << (slot[q] & 31));
          D = max(D, 0xFFFFFFFFu - T.ld(&T.dist[slot[q]]));
          nt++;
        }
        T.st(&T.dist[slot[q]], SP_INF32);
      }
    }
  }
  D = C.max(D, T);
  nt = C.sum(nt, T);
  if (nt == 0) {
    tab_reset(T, C);
    return true;
  }
  if (D > SP_MAXW) {
    if (tl == 0) atomicOr(err, kErrOverflow);
    tab_reset(T, C);
    return true;
  }

  if constexpr (SET) return settled_search(ov, memo, T, s, gs, D, nt, ss, ws, hops, C, label);

  // ---- 2. bounded search from s: label-correcting (exact) or
  //         hop-synchronous (HOP) ------------------------------------------
  C.sync(T);
  if (tl == 0) {
    const int slot = T.insert(s);
    if (slot >= 0) {
      T.st(&T.dist[slot], 0u);
      if constexpr (HOP) T.st(&T.dist2[slot], 0u);
      atomicOr(&T.front[slot >> 5], 1u << (slot & 31));
      T.sti(&T.fr0[0], (IdxT)slot);
      T.st(&T.ctr[kCtrF0], 1u);
    }
  }
  C.sync(T);
  int cur = 0;
  uint32_t level = 0;
  while (!T.ld(&T.ctr[kCtrOvf])) {
    IdxT *fc = cur ? T.fr1 : T.fr0;
    IdxT *fn = cur ? T.fr0 : T.fr1;
    uint32_t *nc = &T.ctr[cur ? kCtrF1 : kCtrF0];
    uint32_t *nn = &T.ctr[cur ? kCtrF0 : kCtrF1];
    const uint32_t ncur = T.ld(nc);
    if (ncur == 0) break;
    if constexpr (HOP) {
      if (level == hops) break;
    }
    // exact mode: the step's distance bound (frontier entries at or above
    // it wait for a later step)
    uint32_t B = 0xFFFFFFFFu;
    if constexpr (!HOP && G == kWave) {  // wave and block searches (dense rounds)
      if (hops < 32) {
        uint32_t mn = SP_INF32;
        for (uint32_t i = tl; i < ncur; i += NT) mn = min(mn, T.ld(&T.dist[T.ldi(&fc[i])]));
        mn = (uint32_t)C.min64((uint64_t)mn, T);
        const uint32_t width = max(D >> hops, 1u);
        B = mn > 0xFFFFFFFFu - width ? 0xFFFFFFFFu : mn + width;
      }
    }
    C.sync(T);
    if (tl == 0) T.st(nn, 0u);
    C.sync(T);
    for (uint32_t fb = wbase; fb < ncur; fb += NT) {
      const uint32_t i = fb + gl;
      uint32_t rs = 0, rl = 0, dx = 0;
      if (i < ncur) {
        const IdxT x = T.ldi(&fc[i]);
        bool later = false;
        if constexpr (!HOP) {
          if (T.ld(&T.dist[x]) >= B) {
            // stays flagged and goes to the next list; an improvement made
            // meanwhile finds the bit set and does not add x again
            later = true;
            const uint32_t p = atomicAdd(nn, 1u);
            if (p < T.fcap) T.sti(&fn[p], x);
          } else {
            // the bit is cleared before the distance is read: an improvement
            // made after the read re-flags x for the next level
            atomicAnd(&T.front[x >> 5], ~(1u << (x & 31)));
            if constexpr (GL) __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "agent");
            else if constexpr (NW == 1) __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            else __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
          }
        }
        if (!later) {
          dx = T.ld(&T.dist[x]);
          const uint32_t vx = T.ld(&T.key[x]);
          rs = ov.foff[vx];
          rl = ov.foff[vx + 1] - rs;
          ss.rows++;
        }
      }
      const uint32_t incl = gscan_incl<G>(rl);
      const uint32_t total = gshfl<G>(incl, G - 1);
      for_row_arcs<G>(T, ov.farc, incl, rs, rl, dx, total, [&](uint2 b, uint32_t sdx) {
        ss.arcs++;
        const uint64_t nd = (uint64_t)sdx + b.y;
        if (nd <= D) {
          const int y = T.insert(b.x);
          if (y >= 0) {
            uint32_t *dw = HOP ? T.dist2 : T.dist;
            const uint32_t old = atomicMin(&dw[y], (uint32_t)nd);
            if ((uint32_t)nd < old) {
              const uint32_t bit = 1u << (y & 31);
              const uint32_t f = atomicOr(&T.front[y >> 5], bit);
              if (!(f & bit)) {
                // more than fcap distinct slots means more than limit used:
                // the overflow is flagged and the search discarded
                const uint32_t p = atomicAdd(nn, 1u);
                if (p < T.fcap) T.sti(&fn[p], (IdxT)y);
              }
            }
          }
        }
      });
      if (T.ld(&T.ctr[kCtrOvf])) break;
    }
    C.sync(T);
    if constexpr (HOP) {
      // end of the level: the changed entries take their new distance and
      // may change again in the next level
      const uint32_t nnext = min(T.ld(nn), T.fcap);
      for (uint32_t i = tl; i < nnext; i += NT) {
        const IdxT y = T.ldi(&fn[i]);
        T.st(&T.dist[y], T.ld(&T.dist2[y]));
        atomicAnd(&T.front[y >> 5], ~(1u << (y & 31)));
      }
      C.sync(T);
      level++;
    }
    cur ^= 1;
  }
  C.sync(T);
  if (T.ld(&T.ctr[kCtrOvf])) {
    tab_reset(T, C);
    return false;
  }

  // ---- 3. memoize the targets' distances ------------------------------
  ss.targets += (tl == 0) ? nt : 0;  // counted once, by the attempt that completes
  ss.searched += (tl == 0) ? 1 : 0;
  {
    const uint32_t used = T.ld(&T.ctr[kCtrUsed]);
    uint32_t ball = 0;  // vertices within radius D of s (s included)
    for (uint32_t i = tl; i < used; i += NT) {
      const IdxT slot = T.ldi(&T.order[i]);
      if (ws) ball += T.ld(&T.dist[slot]) <= D ? 1u : 0u;
      if ((T.ld(&T.tgt[slot >> 5]) >> (slot & 31)) & 1u) {
        const uint32_t d = T.ld(&T.dist[slot]);
        if (d <= D) {
          memo_put(memo, gs, ov.gid[T.ld(&T.key[slot])], d);
          ss.inserts++;
        } else if (!HOP) {
          atomicOr(err, kErrCapacity);  // cannot happen: every target is within D
        }
      }
    }
    if (ws) {
      ball = C.sum(ball, T);
      if (tl == 0) ws[gs] = ball;
    }
  }
  tab_reset(T, C);
  return true;
}

}  // namespace sp
