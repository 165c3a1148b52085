// round_kernels.hpp -- kernels of one contraction round and of the input
// ingest, for gfx950.  The host driver is builder.hip.
//
// Vertex ids inside a round are local ids 0..n_o-1 of the current overlay;
// `gid` maps them to original ids.  Overlay rows are sorted by neighbour id.
#pragma once

#include "common.hpp"
#include "search.hpp"

namespace sp {

// ===========================================================================
// ingest
// ===========================================================================

// key = (tail << kb) | head for every input arc; self-loops get the
// sentinel SP_EMPTY64 (sorted last, dropped).  Also validates the input.
// With `inv` (new id of each input vertex), the keys are in the new ids.
__global__ void k_ingest_keys(uint32_t n, uint64_t m, int kb, const uint64_t *__restrict__ off,
                              const uint32_t *__restrict__ dst, const uint32_t *__restrict__ w,
                              uint64_t *__restrict__ key, uint32_t *__restrict__ val,
                              uint32_t *__restrict__ bad, const uint32_t *__restrict__ inv) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += stride) {
    const uint64_t a = off[u], b = off[u + 1];
    if (a > b || b > m) {
      atomicOr(bad, 1u);
      continue;
    }
    for (uint64_t e = a; e < b; e++) {
      const uint32_t v = dst[e], ww = w[e];
      if (v >= n || ww == SP_INF32) atomicOr(bad, 2u);
      key[e] = (v == u || v >= n) ? SP_EMPTY64
               : inv ? (((uint64_t)inv[u] << kb) | inv[v])
                     : (((uint64_t)u << kb) | v);
      val[e] = ww;
    }
  }
}

// ---------------------------------------------------------------------------
// locality order of the input (the build runs on it; results are mapped
// back to the input's ids before postprocessing)
// ---------------------------------------------------------------------------
// One step of min-label propagation along the input arcs: L2[v] = the
// smallest of L[v] and L over v's out-neighbours.  Bad rows and heads are
// skipped here (the key pass reports them).
__global__ void k_minlabel_step(uint32_t n, uint64_t m, const uint64_t *__restrict__ off,
                                const uint32_t *__restrict__ dst, const uint32_t *__restrict__ L,
                                uint32_t *__restrict__ L2) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    const uint64_t a = off[v], b = off[v + 1];
    uint32_t x = L[v];
    if (a <= b && b <= m)
      for (uint64_t e = a; e < b; e++) {
        const uint32_t u = dst[e];
        if (u < n) x = min(x, L[u]);
      }
    L2[v] = x;
  }
}

// key = (coarse label << kb) | fine label: vertices of one coarse cluster
// end up together, and inside it those of one fine cluster.
__global__ void k_order_keys(uint32_t n, int kb, const uint32_t *__restrict__ coarse,
                             const uint32_t *__restrict__ fine, uint64_t *__restrict__ key) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
    key[v] = ((uint64_t)coarse[v] << kb) | fine[v];
}

// out[idx[i]] = in[i] (scatter) or out[i] = in[idx[i]] (gather).
__global__ void k_permute_u32(uint32_t n, const uint32_t *__restrict__ idx,
                              const uint32_t *__restrict__ in, uint32_t *__restrict__ out,
                              int scatter) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    if (scatter) out[idx[i]] = in[i];
    else out[i] = in[idx[i]];
  }
}

// Vertex ids x -> map[x] in place (SP_NOMID stays).
__global__ void k_map_ids(uint64_t m, uint32_t *__restrict__ x, const uint32_t *__restrict__ map) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
    const uint32_t v = x[i];
    if (v != SP_NOMID) x[i] = map[v];
  }
}

// Marks the first element of each run of equal (non-sentinel) keys.
__global__ void k_run_heads(const uint64_t *__restrict__ key, uint32_t m, uint8_t *__restrict__ head) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride)
    head[i] = key[i] != SP_EMPTY64 && (i == 0 || key[i] != key[i - 1]);
}

// For each run head: the run's minimum weight.  Output arc k = (key, w).
__global__ void k_run_min(const uint64_t *__restrict__ key, const uint32_t *__restrict__ w,
                          uint32_t m, const uint32_t *__restrict__ heads, const uint32_t *nheads,
                          uint64_t *__restrict__ okey, uint32_t *__restrict__ ow) {
  const uint32_t nh = *nheads;
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < nh; k += stride) {
    uint32_t i = heads[k];
    const uint64_t kk = key[i];
    uint32_t best = w[i];
    for (uint32_t j = i + 1; j < m && key[j] == kk; j++) best = min(best, w[j]);
    okey[k] = kk;
    ow[k] = best;
  }
}

// CSR from arcs sorted by key = (row << kb) | col: off[r] = first arc of row r.
__global__ void k_csr_from_sorted(const uint64_t *__restrict__ key, const uint32_t *__restrict__ w,
                                  const uint32_t *mcount, uint32_t n, int kb,
                                  uint32_t *__restrict__ off, uint2 *__restrict__ arc,
                                  uint32_t *__restrict__ mid) {
  const uint32_t m = *mcount;
  const uint64_t lowmask = (1ull << kb) - 1ull;
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += stride) {
    const uint64_t target = (uint64_t)i << kb;
    uint32_t lo = 0, hi = m;
    while (lo < hi) {
      const uint32_t md = (lo + hi) >> 1;
      if (key[md] < target) lo = md + 1;
      else hi = md;
    }
    off[i] = lo;
  }
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
    arc[i] = make_uint2((uint32_t)(key[i] & lowmask), w[i]);
    mid[i] = SP_NOMID;
  }
}

// (a << kb) | b  ->  (b << kb) | a
// out[i] = in[i] with its two kb-bit halves swapped for i < *mcount; the
// entries up to cap get UINT64_MAX, which no key reaches (its halves would
// be equal), so a sort over cap entries leaves the *mcount keys in front.
__global__ void k_swap_key(const uint64_t *__restrict__ in, const uint32_t *mcount, uint32_t cap,
                           int kb, uint64_t *__restrict__ out) {
  const uint32_t m = *mcount;
  const uint64_t lowmask = (1ull << kb) - 1ull;
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < cap; i += stride) {
    if (i < m) {
      const uint64_t k = in[i];
      out[i] = ((k & lowmask) << kb) | (k >> kb);
    } else {
      out[i] = ~0ull;
    }
  }
}

// Default labels: fmix32(v ^ mixseed), or the id itself (raw).
__global__ void k_default_labels(uint32_t n, uint32_t mixseed, bool raw,
                                 uint32_t *__restrict__ lab) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
    lab[v] = raw ? v : fmix32(v ^ mixseed);
}

__global__ void k_labels_to_keys(uint32_t n, const uint32_t *__restrict__ lab,
                                 uint64_t *__restrict__ key) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) key[v] = lab[v];
}

__global__ void k_adjacent_equal(uint32_t n, const uint64_t *__restrict__ key,
                                 uint32_t *__restrict__ bad) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x + 1; i < n; i += stride)
    if (key[i] == key[i - 1]) atomicOr(bad, 4u);
}

// ===========================================================================
// LocalSearch
// ===========================================================================

// Upper bound on the next round's memo inserts.  A search from s inserts
// at most outdeg(u) targets through each affected out-neighbour u of s, so
// the sum of outdeg(u) over arcs s -> u into affected vertices bounds every
// round; summing it over all in-arcs of the affected vertices, indeg(u) x
// outdeg(u), bounds it again and reads the offsets in order (the exact sum
// would read every source's row at random).
__global__ void k_ls_bound_affected(Overlay ov, const uint8_t *__restrict__ aflag,
                                    unsigned long long *__restrict__ out) {
  uint64_t acc = 0;
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < ov.n; u += stride)
    if (aflag[u])
      acc += (uint64_t)(ov.roff[u + 1] - ov.roff[u]) * (ov.foff[u + 1] - ov.foff[u]);
  acc = gsum64<kWave>(acc);
  if (lane_id() == 0 && acc) atomicAdd(out, (unsigned long long)acc);
}

// Counters of the local search (device, accumulated per launch).
struct LsCounters {
  unsigned long long rows, arcs, probes, inserts, targets, searched;
};

template <int G>
__device__ __forceinline__ void flush_stats(const SearchStats &ss, LsCounters *c) {
  uint64_t r = gsum64<kWave>(ss.rows), a = gsum64<kWave>(ss.arcs);
  uint64_t p = gsum64<kWave>(ss.probes), in = gsum64<kWave>(ss.inserts);
  uint64_t t = gsum64<kWave>(ss.targets), sr = gsum64<kWave>(ss.searched);
  if (lane_id() == 0) {
    atomicAdd(&c->rows, (unsigned long long)r);
    atomicAdd(&c->arcs, (unsigned long long)a);
    atomicAdd(&c->probes, (unsigned long long)p);
    atomicAdd(&c->inserts, (unsigned long long)in);
    atomicAdd(&c->targets, (unsigned long long)t);
    atomicAdd(&c->searched, (unsigned long long)sr);
  }
}

constexpr int kLsBlock = 64;  // one wave per workgroup

// LDS search tables: a search overflows past 3/4 of its slots, so the
// insertion-order and frontier lists hold that many entries.
constexpr int ls_limit(int cap) { return cap * 3 / 4; }
// LDS bytes of one k_local_search block (kLsBlock / G tables): keys,
// distances, hop-mode second distances, target and frontier bitmaps, four
// counters, insertion order and two frontier lists.
constexpr size_t ls_lds_bytes(int g, int cap, bool hop) {
  return (size_t)(kLsBlock / g) *
         (4 * (size_t)cap * (hop ? 3 : 2) + (hop ? 0 : 4) + 8 * (size_t)(cap / 32) + 16 +
          6 * (size_t)ls_limit(cap));
}

// LDS fast path: groups of G lanes, CAP-slot table per group.  Persistent:
// every group takes `chunk` sources at a time from a global counter.
template <int G, int CAP, int M>
__global__ void __launch_bounds__(kLsBlock) k_local_search(
    Overlay ov, const uint32_t *__restrict__ vw, uint32_t nw, const uint8_t *__restrict__ aflag,
    MemoRef memo, LsCounters *__restrict__ cnt,
    const uint32_t *__restrict__ nw_dev, uint32_t *__restrict__ work,
    uint32_t *__restrict__ ovf_list, uint32_t *__restrict__ ovf_count, uint32_t chunk,
    uint32_t *__restrict__ ws, uint32_t *__restrict__ err, uint32_t hops,
    const uint32_t *__restrict__ label) {
  constexpr int NG = kLsBlock / G;
  // second array (hop-mode distances, settled-mode labels) only in those modes
  constexpr bool HOP = M != kWpsExact;
  constexpr int CAP2 = HOP ? CAP : 1;
  constexpr int LIM = ls_limit(CAP);
  static_assert(ls_lds_bytes(G, CAP, HOP) ==
                    sizeof(uint32_t) * (3 * NG * CAP + NG * (CAP2 - CAP) + 2 * NG * (CAP / 32) +
                                        4 * NG) +
                        sizeof(uint16_t) * 3 * NG * LIM,
                "host LDS size of the search tables");
  if (nw_dev) nw = *nw_dev;  // source count produced by an earlier kernel
  if (nw == 0) return;
  __shared__ uint32_t s_key[NG][CAP];
  __shared__ uint32_t s_dist[NG][CAP];
  __shared__ uint32_t s_dist2[NG][CAP2];
  __shared__ uint32_t s_bits[NG][2][CAP / 32];  // target, frontier
  __shared__ uint16_t s_order[NG][LIM];
  __shared__ uint16_t s_fr[NG][2][LIM];
  __shared__ uint32_t s_ctr[NG][4];
  const int g = threadIdx.x / G, gl = glane<G>();
  for (int i = gl; i < CAP; i += G) {
    s_key[g][i] = SP_EMPTY32;
    s_dist[g][i] = SP_INF32;
    if constexpr (HOP) s_dist2[g][i] = SP_INF32;
  }
  for (int i = gl; i < CAP / 32; i += G) {
    s_bits[g][0][i] = 0;
    s_bits[g][1][i] = 0;
  }
  if (gl < 4) s_ctr[g][gl] = 0;
  wave_sync();
  Tab<uint16_t, false> T;
  T.key = s_key[g];
  T.dist = s_dist[g];
  T.dist2 = HOP ? s_dist2[g] : nullptr;
  T.tgt = s_bits[g][0];
  T.front = s_bits[g][1];
  T.order = s_order[g];
  T.fr0 = s_fr[g][0];
  T.fr1 = s_fr[g][1];
  T.ctr = s_ctr[g];
  T.cap = CAP;
  T.shift = 32 - __builtin_ctz(CAP);
  T.limit = LIM;
  T.fcap = LIM;
  SearchStats ss;
  const Coop<G, 1> C{nullptr};
  for (;;) {
    uint32_t base = 0;
    if (gl == 0) base = atomicAdd(work, chunk);
    base = gshfl<G>(base, 0);
    if (base >= nw) break;
    const uint32_t end = min(base + chunk, nw);
    for (uint32_t i = base; i < end; i++) {
      const uint32_t s = vw[i];
      if (!search_source<G, 1, M>(ov, aflag, memo, T, s, ss, ws, err, hops, C, label)) {
        if (gl == 0) {
          const uint32_t k = atomicAdd(ovf_count, 1u);
          ovf_list[k] = s;
        }
      }
    }
  }
  flush_stats<G>(ss, cnt);
}

// Searches that outgrow a wave's table: NW waves of one block share one
// source and one CAP-slot LDS table (Coop in search.hpp), so a large search
// gets NW times the lanes per frontier level.  Persistent: blocks take
// sources one at a time from a global counter.  Eight waves (also per
// global-tier search): on road-like 24M the block and global tiers take 342
// and 129 ms per build against 372 and 132 with sixteen waves (fewer idle
// waves at a narrow frontier, cheaper barriers), 394 and 133 with four.
constexpr int kLsBlkWaves = 8;
constexpr int kLsBlkCap = 8192;
constexpr size_t ls_blk_lds_bytes(int cap, bool hop, int nw) {
  return 4 * (size_t)cap * (hop ? 3 : 2) + (hop ? 0 : 4) + 8 * (size_t)(cap / 32) + 16 +
         6 * (size_t)ls_limit(cap) + 8 * (size_t)nw + 4;
}
template <int CAP, int M, int NW>
__global__ void __launch_bounds__(kWave * NW) k_local_search_blk(
    Overlay ov, const uint32_t *__restrict__ vw, uint32_t nw, const uint8_t *__restrict__ aflag,
    MemoRef memo, LsCounters *__restrict__ cnt, const uint32_t *__restrict__ nw_dev,
    uint32_t *__restrict__ work, uint32_t *__restrict__ ovf_list, uint32_t *__restrict__ ovf_count,
    uint32_t *__restrict__ ws, uint32_t *__restrict__ err, uint32_t hops,
    const uint32_t *__restrict__ label) {
  constexpr bool HOP = M != kWpsExact;  // a second array (hop distances or settled labels)
  constexpr int CAP2 = HOP ? CAP : 1;
  constexpr int LIM = ls_limit(CAP);
  static_assert(LIM <= 65536, "16-bit slot lists");
  if (nw_dev) nw = *nw_dev;  // source count produced by an earlier kernel
  if (nw == 0) return;
  __shared__ uint32_t s_key[CAP];
  __shared__ uint32_t s_dist[CAP];
  __shared__ uint32_t s_dist2[CAP2];
  __shared__ uint32_t s_bits[2][CAP / 32];  // target, frontier
  __shared__ uint16_t s_order[LIM];
  __shared__ uint16_t s_fr[2][LIM];
  __shared__ uint32_t s_ctr[4];
  __shared__ __align__(8) uint32_t s_red[2 * NW];  // also read as NW 64-bit words
  __shared__ uint32_t s_next;
  const uint32_t tid = threadIdx.x;
  for (uint32_t i = tid; i < CAP; i += kWave * NW) {
    s_key[i] = SP_EMPTY32;
    s_dist[i] = SP_INF32;
    if constexpr (HOP) s_dist2[i] = SP_INF32;
  }
  for (uint32_t i = tid; i < CAP / 32; i += kWave * NW) {
    s_bits[0][i] = 0;
    s_bits[1][i] = 0;
  }
  if (tid < 4) s_ctr[tid] = 0;
  __syncthreads();
  Tab<uint16_t, false> T;
  T.key = s_key;
  T.dist = s_dist;
  T.dist2 = HOP ? s_dist2 : nullptr;
  T.tgt = s_bits[0];
  T.front = s_bits[1];
  T.order = s_order;
  T.fr0 = s_fr[0];
  T.fr1 = s_fr[1];
  T.ctr = s_ctr;
  T.cap = CAP;
  T.shift = 32 - __builtin_ctz(CAP);
  T.limit = LIM;
  T.fcap = LIM;
  const Coop<kWave, NW> C{s_red};
  SearchStats ss;
  for (;;) {
    if (tid == 0) s_next = atomicAdd(work, 1u);
    __syncthreads();
    const uint32_t i = s_next;
    __syncthreads();
    if (i >= nw) break;
    const uint32_t s = vw[i];
    if (!search_source<kWave, NW, M>(ov, aflag, memo, T, s, ss, ws, err, hops, C, label)) {
      if (tid == 0) {
        const uint32_t k = atomicAdd(ovf_count, 1u);
        ovf_list[k] = s;
      }
    }
  }
  flush_stats<kWave>(ss, cnt);
}

// Tables of the global tier: per table `per` words (key, dist, bitmaps and
// lists, hop-mode dist2, counters, each array `cap` words); key, dist and
// dist2 start all ones, the rest zero.
__global__ void k_gtab_init(uint32_t *__restrict__ tabs, uint64_t words, uint64_t per,
                            uint32_t cap, bool hop) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride) {
    const uint64_t o = i % per;
    const bool ones = o < 2ull * cap || (hop && o >= 6ull * cap && o < 7ull * cap);
    tabs[i] = ones ? SP_EMPTY32 : 0u;
  }
}

// Global-memory fallback: NW waves of one block per source, table of `cap`
// slots per block at tabs + block * stride_words (key, dist, a region
// holding the target and frontier bitmaps, order, fr0, fr1 and, in hop
// mode, dist2 as consecutive uint32 arrays of `cap`, then 4 counters).
template <int M, int NW>
__global__ void __launch_bounds__(kWave * NW) k_local_search_global(
    Overlay ov, const uint32_t *__restrict__ list, uint32_t nlist,
    const uint8_t *__restrict__ aflag, MemoRef memo,
    LsCounters *__restrict__ cnt, uint32_t *__restrict__ tabs, uint32_t cap,
    uint32_t *__restrict__ ws, uint32_t *__restrict__ err, uint32_t hops,
    const uint32_t *__restrict__ label) {
  constexpr bool HOP = M != kWpsExact;  // a seventh array (hop distances or settled labels)
  constexpr size_t kArrays = HOP ? 7 : 6;
  __shared__ __align__(8) uint32_t s_red[2 * NW];  // also read as NW 64-bit words
  uint32_t *base = tabs + (size_t)blockIdx.x * ((size_t)cap * kArrays + 4);
  Tab<uint32_t, true> T;
  T.key = base;
  T.dist = base + cap;
  T.tgt = base + 2 * (size_t)cap;  // the two bitmaps share a region of cap words
  T.front = T.tgt + cap / 32;
  T.order = base + 3 * (size_t)cap;
  T.fr0 = base + 4 * (size_t)cap;
  T.fr1 = base + 5 * (size_t)cap;
  T.dist2 = HOP ? base + 6 * (size_t)cap : nullptr;
  T.ctr = base + kArrays * (size_t)cap;
  T.cap = cap;
  T.shift = 32 - __builtin_ctz(cap);
  T.limit = cap;  // cap >= 2 n_o: never overflows
  T.fcap = cap;
  const Coop<kWave, NW> C{s_red};
  SearchStats ss;
  for (uint32_t i = blockIdx.x; i < nlist; i += gridDim.x) {
    if (!search_source<kWave, NW, M>(ov, aflag, memo, T, list[i], ss, ws, err, hops, C,
                                      label)) {
      if (threadIdx.x == 0) atomicOr(err, kErrCapacity);
    }
  }
  flush_stats<kWave>(ss, cnt);
}

// Pruning (end of Alg. 4): an out-arc (s, v) of a source s whose weight
// exceeds the memoized dist(s, v) is deleted (weight set to SP_INF32 in both
// the forward row of s and the reverse row of v).  A group of G lanes per
// source, lanes over its out-arcs.
template <int G>
__global__ void __launch_bounds__(256) k_prune(Overlay ov, const uint32_t *__restrict__ vw,
                                               uint32_t nw, MemoRef memo,
                                               unsigned long long *__restrict__ npruned,
                                               uint32_t *__restrict__ pw,
                                               uint32_t *__restrict__ err) {
  const uint32_t ngroups = gridDim.x * (blockDim.x / G);
  const uint32_t g0 = blockIdx.x * (blockDim.x / G) + threadIdx.x / G;
  const int gl = glane<G>();
  uint32_t probes = 0;
  uint64_t c = 0;
  for (uint32_t k = g0; k < nw; k += ngroups) {
    const uint32_t s = vw[k];
    const uint32_t gs = ov.gid[s];
    const uint32_t e1 = ov.foff[s + 1];
    for (uint32_t eb = ov.foff[s] + gl; eb < e1; eb += G * kPairBatch) {
      uint2 arc[kPairBatch];
      uint32_t ss[kPairBatch], gv[kPairBatch], dd[kPairBatch];
      bool act[kPairBatch];
#pragma unroll
      for (int q = 0; q < kPairBatch; q++) {
        const uint32_t e = eb + q * G;
        act[q] = e < e1;
        arc[q] = act[q] ? ov.farc[e] : make_uint2(0, SP_INF32);
      }
#pragma unroll
      for (int q = 0; q < kPairBatch; q++) {
        ss[q] = gs;
        gv[q] = act[q] ? ov.gid[arc[q].x] : 0u;
      }
      memo_get_batch<kPairBatch>(memo, ss, gv, act, dd, &probes);
#pragma unroll
      for (int q = 0; q < kPairBatch; q++) {
        const uint2 a = arc[q];
        // arcs pruned by an earlier pass of this round stay as they are
        if (!act[q] || a.y == SP_INF32 || dd[q] == SP_INF32 || a.y <= dd[q]) continue;
        pw[eb + q * G] = a.y;  // kept until the round's searches are known complete
        ov.farc[eb + q * G].y = SP_INF32;
        const uint32_t end = ov.roff[a.x + 1];
        uint32_t lo = ov.roff[a.x], hi = end;
        while (lo < hi) {
          const uint32_t md = (lo + hi) >> 1;
          if (ov.rarc[md].x < s) lo = md + 1;
          else hi = md;
        }
        if (lo < end && ov.rarc[lo].x == s) ov.rarc[lo].y = SP_INF32;
        else atomicOr(err, kErrCapacity);  // reverse twin missing: internal error
        c++;
      }
    }
  }
  c = gsum64<kWave>(c);
  if (lane_id() == 0 && c) atomicAdd(npruned, (unsigned long long)c);
}

// Undoes this round's pruning (the weights k_prune saved in pw) before a
// search that has to see the same overlay as the round's other searches:
// Alg. 4 prunes only once every source has been searched.  Every arc with
// weight SP_INF32 in the overlay was pruned in this round (the rebuild drops
// pruned arcs).  A wave per source, lanes over its out-arcs.
__global__ void __launch_bounds__(256) k_unprune(Overlay ov, const uint32_t *__restrict__ vw,
                                                 uint32_t nw, const uint32_t *__restrict__ pw,
                                                 uint32_t *__restrict__ err) {
  const uint32_t nwaves = gridDim.x * (blockDim.x / kWave);
  for (uint32_t k = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; k < nw;
       k += nwaves) {
    const uint32_t s = vw[k];
    const uint32_t e1 = ov.foff[s + 1];
    for (uint32_t e = ov.foff[s] + lane_id(); e < e1; e += kWave) {
      const uint2 a = ov.farc[e];
      if (a.y != SP_INF32) continue;
      const uint32_t wt = pw[e];
      ov.farc[e].y = wt;
      const uint32_t end = ov.roff[a.x + 1];
      uint32_t lo = ov.roff[a.x], hi = end;
      while (lo < hi) {
        const uint32_t md = (lo + hi) >> 1;
        if (ov.rarc[md].x < s) lo = md + 1;
        else hi = md;
      }
      if (lo < end && ov.rarc[lo].x == s) ov.rarc[lo].y = wt;
      else atomicOr(err, kErrCapacity);  // reverse twin missing: internal error
    }
  }
}

// ===========================================================================
// Score (Alg. 5) -- group of G lanes per affected vertex
// ===========================================================================
// Number of pairs (v1, v2) in N_in(u) x N_out(u), v1 != v2, both arcs live,
// whose path through u is no longer than the memoized distance or whose
// distance is not memoized.  Every group lane must call it.
// Pair p of N_in(u) x N_out(u) in row-major order: (in-arc index, out-arc
// index); 32-bit division when the pair count allows it.
__device__ __forceinline__ uint2 pair_index(uint64_t p, uint32_t dout, bool narrow) {
  if (narrow) {
    const uint32_t i = (uint32_t)p / dout;
    return make_uint2(i, (uint32_t)p - i * dout);
  }
  const uint32_t i = (uint32_t)(p / dout);
  return make_uint2(i, (uint32_t)(p - (uint64_t)i * dout));
}

// The pairs of u handled by one lane in one step: kPairBatch pairs p0 + k G,
// their arcs, via lengths and memoized distances, with all loads of a kind
// issued together.
struct PairBatch {
  uint2 a[kPairBatch], b[kPairBatch];
  uint64_t via[kPairBatch];
  uint32_t d[kPairBatch];
  bool live[kPairBatch];
};

template <int G>
__device__ __forceinline__ void load_pairs(const Overlay &ov, const MemoRef &memo,
                                           uint32_t i0, uint32_t o0, uint32_t dout, uint64_t np,
                                           bool narrow, uint64_t p0, PairBatch &B,
                                           uint32_t *probes) {
  uint32_t gs[kPairBatch], gv[kPairBatch];
#pragma unroll
  for (int k = 0; k < kPairBatch; k++) {
    const uint64_t p = p0 + (uint64_t)k * G;
    B.a[k] = make_uint2(0, SP_INF32);
    B.b[k] = make_uint2(0, SP_INF32);
    if (p < np) {
      const uint2 ij = pair_index(p, dout, narrow);
      B.a[k] = ov.rarc[i0 + ij.x];
      B.b[k] = ov.farc[o0 + ij.y];
    }
  }
#pragma unroll
  for (int k = 0; k < kPairBatch; k++) {
    B.live[k] = B.a[k].y != SP_INF32 && B.b[k].y != SP_INF32 && B.a[k].x != B.b[k].x;
    B.via[k] = (uint64_t)B.a[k].y + B.b[k].y;
    gs[k] = 0;
    gv[k] = 0;
    if (B.live[k]) {
      gs[k] = ov.gid[B.a[k].x];
      gv[k] = ov.gid[B.b[k].x];
    }
  }
  memo_get_batch<kPairBatch>(memo, gs, gv, B.live, B.d, probes);
}

template <int G>
__device__ __forceinline__ uint32_t count_pairs(const Overlay &ov, const MemoRef &memo,
                                                uint32_t u, uint32_t *probes) {
  const int gl = glane<G>();
  const uint32_t i0 = ov.roff[u], din = ov.roff[u + 1] - i0;
  const uint32_t o0 = ov.foff[u], dout = ov.foff[u + 1] - o0;
  uint32_t cnt = 0;
  const uint64_t np = (uint64_t)din * dout;
  const bool narrow = np <= 0xFFFFFFFFull;
  for (uint64_t p0 = gl; p0 < np; p0 += (uint64_t)G * kPairBatch) {
    PairBatch B;
    load_pairs<G>(ov, memo, i0, o0, dout, np, narrow, p0, B, probes);
#pragma unroll
    for (int k = 0; k < kPairBatch; k++)
      cnt += B.live[k] && (B.d[k] == SP_INF32 || B.via[k] <= B.d[k]);
  }
  return gsum<G>(cnt);
}

// Live out-degree, live in-degree and |N_in(u) union N_out(u)| over live
// arcs.  Every group lane must call it.
template <int G>
__device__ __forceinline__ uint3 count_neighbours(const Overlay &ov, uint32_t u) {
  const int gl = glane<G>();
  const uint32_t i0 = ov.roff[u], i1 = ov.roff[u + 1];
  const uint32_t o0 = ov.foff[u], o1 = ov.foff[u + 1];
  uint32_t cout = 0, cin = 0, only_in = 0;
  for (uint32_t e = o0 + gl; e < o1; e += G) cout += ov.farc[e].y != SP_INF32;
  for (uint32_t e = i0 + gl; e < i1; e += G) {
    const uint2 a = ov.rarc[e];
    if (a.y == SP_INF32) continue;
    cin++;
    uint32_t lo = o0, hi = o1;
    while (lo < hi) {
      const uint32_t md = (lo + hi) >> 1;
      if (ov.farc[md].x < a.x) lo = md + 1;
      else hi = md;
    }
    const bool both = lo < o1 && ov.farc[lo].x == a.x && ov.farc[lo].y != SP_INF32;
    only_in += both ? 0u : 1u;
  }
  cout = gsum<G>(cout);
  cin = gsum<G>(cin);
  only_in = gsum<G>(only_in);
  return make_uint3(cout, cin, cout + only_in);
}

// Per-vertex state of the score terms beyond the edge difference (original
// ids).  cn and depth are kept when the learned priority, recorded features
// or a nonzero k_cn / k_depth need them; ws and feat only for the learned
// priority and recorded features; null pointers skip that state.
struct FeatState {
  uint32_t *cn;     // contracted neighbours (or null)
  uint32_t *depth;  // hierarchy depth (or null)
  uint32_t *ws;     // vertices reached by the latest witness search (or null)
  float *feat;      // current features, 8 per vertex (or null)
  float *rec;       // features at contraction (or null)
  int32_t k_ed, k_cn, k_depth;  // integer score weights (1, 0, 0: edge difference)
};

// x / (x + c) in single precision (the learned priority's squash).
__device__ __forceinline__ float squash(uint32_t x, float c) {
  return __fdiv_rn((float)x, __fadd_rn((float)x, c));
}

// Edge difference (the plain priority) and the features of the learned one.
template <int G>
__global__ void __launch_bounds__(256) k_score(Overlay ov, const uint32_t *__restrict__ va,
                                               uint32_t na, MemoRef memo, int32_t *__restrict__ P,
                                               uint32_t *__restrict__ paircnt, FeatState fs) {
  const uint32_t ngroups = gridDim.x * (blockDim.x / G);
  const uint32_t g0 = blockIdx.x * (blockDim.x / G) + threadIdx.x / G;
  uint32_t probes = 0;
  for (uint32_t k = g0; k < na; k += ngroups) {
    const uint32_t u = va[k];
    const uint32_t pairs = count_pairs<G>(ov, memo, u, &probes);
    const uint3 deg = count_neighbours<G>(ov, u);  // out, in, |N(u)|
    if (glane<G>() == 0) {
      const int64_t e64 = (int64_t)pairs - (int64_t)deg.z;
      const uint32_t g = ov.gid[u];
      // k_ed ED + k_cn CN + k_depth depth in 64 bits, saturated to int32
      int64_t p = (int64_t)fs.k_ed * e64;
      if (fs.cn) p += (int64_t)fs.k_cn * fs.cn[g] + (int64_t)fs.k_depth * fs.depth[g];
      P[u] = (int32_t)(p > INT32_MAX ? INT32_MAX : (p < INT32_MIN ? INT32_MIN : p));
      paircnt[u] = pairs;
      if (!fs.feat) continue;
      const int32_t ed = (int32_t)(e64 > INT32_MAX ? INT32_MAX : (e64 < INT32_MIN ? INT32_MIN : e64));
      float *f = fs.feat + (size_t)g * 8;
      const uint32_t mag = ed < 0 ? (uint32_t)(-(int64_t)ed) : (uint32_t)ed;
      f[0] = __fdiv_rn((float)ed, __fadd_rn((float)mag, 8.0f));
      f[1] = squash(fs.cn[g], 8.0f);
      f[2] = squash(deg.y, 8.0f);
      f[3] = squash(deg.x, 8.0f);
      f[4] = squash(fs.depth[g], 8.0f);
      f[5] = squash(fs.ws[g], 64.0f);
      f[6] = squash(deg.z, 8.0f);
      f[7] = squash(pairs, 8.0f);
    }
  }
}

// ===========================================================================
// Select (Alg. 6)
// ===========================================================================
// Selection keys (priority, label); also clears the per-vertex flags S and
// newA that the contraction sets and the shortcut-row bounds (4 arrays of n)
// that k_row_bounds fills.
__global__ void k_keys(uint32_t n, const int32_t *__restrict__ P, const uint32_t *__restrict__ gid,
                       const uint32_t *__restrict__ label, uint64_t *__restrict__ key,
                       uint8_t *__restrict__ S, uint8_t *__restrict__ newA,
                       uint32_t *__restrict__ bounds) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += stride) {
    key[u] = ((uint64_t)((uint32_t)P[u] ^ 0x80000000u) << 32) | label[gid[u]];
    S[u] = 0;
    newA[u] = 0;
    bounds[u] = 0;
    bounds[(size_t)n + u] = 0;
    bounds[2 * (size_t)n + u] = 0;
    bounds[3 * (size_t)n + u] = 0;
  }
}

// Row bounds of sorted (row << kb | col) keys: for every row r with keys,
// first[r] = index of its first key and stop[r] = one past its last (rows
// without keys keep 0, 0 from k_keys).  blockIdx.y selects the key set:
// (keys0, first0, stop0) or (keys1, first1, stop1).
__global__ void k_row_bounds(const uint64_t *__restrict__ keys0,
                             const uint64_t *__restrict__ keys1, const uint32_t *nkeys, int kb,
                             uint32_t *__restrict__ first0, uint32_t *__restrict__ stop0,
                             uint32_t *__restrict__ first1, uint32_t *__restrict__ stop1) {
  const uint64_t *keys = blockIdx.y ? keys1 : keys0;
  uint32_t *first = blockIdx.y ? first1 : first0;
  uint32_t *stop = blockIdx.y ? stop1 : stop0;
  const uint32_t m = *nkeys;
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
    const uint32_t r = (uint32_t)(keys[i] >> kb);
    if (i == 0 || (uint32_t)(keys[i - 1] >> kb) != r) first[r] = i;
    if (i + 1 == m || (uint32_t)(keys[i + 1] >> kb) != r) stop[r] = i + 1;
  }
}

// u is selected iff key(u) < key(v) for every live neighbour v (keys are
// distinct because labels are).
template <int G>
__global__ void __launch_bounds__(256) k_select(Overlay ov, const uint64_t *__restrict__ key,
                                                uint8_t *__restrict__ F) {
  const uint32_t ngroups = gridDim.x * (blockDim.x / G);
  const uint32_t g0 = blockIdx.x * (blockDim.x / G) + threadIdx.x / G;
  const int gl = glane<G>();
  for (uint32_t u = g0; u < ov.n; u += ngroups) {
    const uint64_t ku = key[u];
    bool beaten = false;
    for (uint32_t e = ov.foff[u] + gl; e < ov.foff[u + 1]; e += G) {
      const uint2 b = ov.farc[e];
      beaten |= b.y != SP_INF32 && key[b.x] < ku;
    }
    for (uint32_t e = ov.roff[u] + gl; e < ov.roff[u + 1]; e += G) {
      const uint2 a = ov.rarc[e];
      beaten |= a.y != SP_INF32 && key[a.x] < ku;
    }
    beaten = gany<G>(beaten);
    if (gl == 0) F[u] = beaten ? 0 : 1;
  }
}

// ===========================================================================
// Contract (Alg. 7)
// ===========================================================================
// Per selected vertex: live out-arcs, live in-arcs, shortcut pairs (the
// pair count of the score when the vertex was rescored this round).
// The selected count *nfp is read on the device; entries nf .. cap - 1 of
// the three count arrays are set to zero so that they can be scanned over
// cap entries.
template <int G>
__global__ void __launch_bounds__(256) k_contract_count(
    Overlay ov, const uint32_t *__restrict__ vf, const uint32_t *nfp, uint32_t cap,
    const uint8_t *__restrict__ aflag, const uint32_t *__restrict__ paircnt,
    MemoRef memo, uint32_t *__restrict__ cup,
    uint32_t *__restrict__ cdn, uint32_t *__restrict__ cpair) {
  const uint32_t ngroups = gridDim.x * (blockDim.x / G);
  const uint32_t g0 = blockIdx.x * (blockDim.x / G) + threadIdx.x / G;
  const int gl = glane<G>();
  const uint32_t nf = *nfp;
  for (uint32_t k = nf + blockIdx.x * blockDim.x + threadIdx.x; k < cap;
       k += gridDim.x * blockDim.x) {
    cup[k] = 0;
    cdn[k] = 0;
    cpair[k] = 0;
  }
  uint32_t probes = 0;
  for (uint32_t k = g0; k < nf; k += ngroups) {
    const uint32_t u = vf[k];
    uint32_t co = 0, ci = 0;
    for (uint32_t e = ov.foff[u] + gl; e < ov.foff[u + 1]; e += G) co += ov.farc[e].y != SP_INF32;
    for (uint32_t e = ov.roff[u] + gl; e < ov.roff[u + 1]; e += G) ci += ov.rarc[e].y != SP_INF32;
    co = gsum<G>(co);
    ci = gsum<G>(ci);
    uint32_t pc;
    if (aflag[u]) pc = paircnt[u];
    else pc = count_pairs<G>(ov, memo, u, &probes);
    if (gl == 0) {
      cup[k] = co;
      cdn[k] = ci;
      cpair[k] = pc;
    }
  }
}

struct ArcOut {
  uint32_t *t, *h, *w, *m;
};

// Marks the entry of vertex x in row r (sorted by neighbour) as deleted: the
// contracted vertex x leaves the overlay, and the rebuild then needs no
// per-arc lookup of the contraction flag.  Rows of different contracted
// vertices' neighbours never share an entry (the contracted set is
// independent), so the write has no contention.
__device__ __forceinline__ void kill_twin(const uint32_t *__restrict__ off, uint2 *__restrict__ arc,
                                          uint32_t r, uint32_t x) {
  uint32_t lo = off[r], hi = off[r + 1];
  const uint32_t end = hi;
  while (lo < hi) {
    const uint32_t md = (lo + hi) >> 1;
    if (arc[md].x < x) lo = md + 1;
    else hi = md;
  }
  if (lo < end && arc[lo].x == x) arc[lo].y = SP_INF32;
}

// Moves the live arcs of each selected vertex into the CH (out-arcs to the
// upward set, in-arcs to the downward set) at scanned positions, emits the
// shortcut candidates (v1, v2, w1 + w2, label(u), u) and marks V_S and the
// next round's affected set.
template <int G>
__global__ void __launch_bounds__(256) k_contract(
    Overlay ov, const uint32_t *__restrict__ vf, uint32_t nf, const int32_t *__restrict__ P,
    const uint32_t *__restrict__ label, MemoRef memo,
    uint32_t round, uint32_t *__restrict__ level, int32_t *__restrict__ score,
    uint8_t *__restrict__ alive_g, const uint32_t *__restrict__ pup,
    const uint32_t *__restrict__ pdn, const uint32_t *__restrict__ ppair, ArcOut up, ArcOut dn,
    uint64_t up_base, uint64_t dn_base, const uint32_t *__restrict__ cpair, int kb,
    uint64_t *__restrict__ ekey, uint32_t *__restrict__ ew,
    uint32_t *__restrict__ elab, uint32_t *__restrict__ emid, uint8_t *__restrict__ S,
    uint8_t *__restrict__ newA, FeatState fs, uint32_t *__restrict__ err) {
  const uint32_t ngroups = gridDim.x * (blockDim.x / G);
  const uint32_t g0 = blockIdx.x * (blockDim.x / G) + threadIdx.x / G;
  const int gl = glane<G>();
  const uint64_t below = (gl == 0) ? 0ull : ((1ull << gl) - 1ull);
  uint32_t probes = 0;
  for (uint32_t k = g0; k < nf; k += ngroups) {
    const uint32_t u = vf[k];
    const uint32_t gu = ov.gid[u];
    const uint32_t lab = label[gu];
    if (gl == 0) {
      level[gu] = round;
      score[gu] = P[u];
      alive_g[gu] = 0;
    }
    if (fs.rec)
      for (int i = gl; i < 8; i += G) fs.rec[(size_t)gu * 8 + i] = fs.feat[(size_t)gu * 8 + i];
    const uint32_t dnext = fs.depth ? fs.depth[gu] + 1 : 0u;
    // out-arcs -> upward set
    uint64_t pos = up_base + pup[k];
    const uint32_t o0 = ov.foff[u], o1 = ov.foff[u + 1];
    for (uint32_t b0 = o0; b0 < o1; b0 += G) {
      const uint32_t e = b0 + gl;
      uint2 b = make_uint2(0, SP_INF32);
      if (e < o1) b = ov.farc[e];
      const bool live = e < o1 && b.y != SP_INF32;
      const uint64_t msk = gballot<G>(live);
      if (live) {
        const uint64_t at = pos + __popcll(msk & below);
        up.t[at] = gu;
        up.h[at] = ov.gid[b.x];
        up.w[at] = b.y;
        up.m[at] = ov.fmid[e];
        newA[b.x] = 1;
        if (fs.cn) {
          const uint32_t gv = ov.gid[b.x];
          atomicAdd(&fs.cn[gv], 1u);
          atomicMax(&fs.depth[gv], dnext);
        }
        kill_twin(ov.roff, ov.rarc, b.x, u);  // (u -> b.x) in the reverse row of b.x
      }
      pos += __popcll(msk);
    }
    // in-arcs -> downward set
    pos = dn_base + pdn[k];
    const uint32_t i0 = ov.roff[u], i1 = ov.roff[u + 1];
    for (uint32_t b0 = i0; b0 < i1; b0 += G) {
      const uint32_t e = b0 + gl;
      uint2 a = make_uint2(0, SP_INF32);
      if (e < i1) a = ov.rarc[e];
      const bool live = e < i1 && a.y != SP_INF32;
      const uint64_t msk = gballot<G>(live);
      if (live) {
        const uint64_t at = pos + __popcll(msk & below);
        dn.t[at] = ov.gid[a.x];
        dn.h[at] = gu;
        dn.w[at] = a.y;
        dn.m[at] = ov.rmid[e];
        newA[a.x] = 1;
        if (fs.cn) {
          // one more contracted neighbour, unless a.x is also a live
          // out-neighbour (counted above)
          uint32_t lo = o0, hi = o1;
          while (lo < hi) {
            const uint32_t md = (lo + hi) >> 1;
            if (ov.farc[md].x < a.x) lo = md + 1;
            else hi = md;
          }
          const bool both = lo < o1 && ov.farc[lo].x == a.x && ov.farc[lo].y != SP_INF32;
          const uint32_t gv = ov.gid[a.x];
          if (!both) atomicAdd(&fs.cn[gv], 1u);
          atomicMax(&fs.depth[gv], dnext);
        }
        kill_twin(ov.foff, ov.farc, a.x, u);  // (a.x -> u) in the forward row of a.x
      }
      pos += __popcll(msk);
    }
    // shortcut candidates, in pair order
    pos = ppair[k];
    const uint64_t pend = pos + cpair[k];
    const uint32_t din = i1 - i0, dout = o1 - o0;
    const uint64_t np = (uint64_t)din * dout;
    const bool narrow = np <= 0xFFFFFFFFull;
    for (uint64_t q0 = 0; q0 < np; q0 += (uint64_t)G * kPairBatch) {
      PairBatch B;
      load_pairs<G>(ov, memo, i0, o0, dout, np, narrow, q0 + gl, B, &probes);
      // emit in pair order: chunk k holds pairs q0 + k G .. q0 + k G + G - 1
#pragma unroll
      for (int k = 0; k < kPairBatch; k++) {
        const bool emit = B.live[k] && (B.d[k] == SP_INF32 || B.via[k] <= B.d[k]);
        const uint64_t msk = gballot<G>(emit);
        if (emit) {
          if (B.via[k] > SP_MAXW) atomicOr(err, kErrOverflow);
          const uint64_t at = pos + __popcll(msk & below);
          if (at >= pend) {
            atomicOr(err, kErrCapacity);
          } else {
            ekey[at] = ((uint64_t)B.a[k].x << kb) | B.b[k].x;
            ew[at] = (uint32_t)B.via[k];
            elab[at] = lab;
            emid[at] = gu;
            S[B.a[k].x] = 1;
          }
        }
        pos += __popcll(msk);
      }
    }
  }
}

// After sorting the candidates by (v1, v2): one record per distinct pair
// with the smallest (weight, label of the middle vertex), and the pair's
// key with its halves swapped, (v2 << kb) | v1, in rkey; rkey entries from
// the pair count up to ne get UINT64_MAX (no key reaches it), so a sort of
// all ne entries leaves the real keys in front.
__global__ void k_eplus_reduce(const uint64_t *__restrict__ key, const uint32_t *__restrict__ idx,
                               uint32_t ne, const uint32_t *__restrict__ heads,
                               const uint32_t *nheads, const uint32_t *__restrict__ ew,
                               const uint32_t *__restrict__ elab, const uint32_t *__restrict__ emid,
                               int kb, uint64_t *__restrict__ ukey, uint32_t *__restrict__ uw,
                               uint32_t *__restrict__ umid, uint64_t *__restrict__ rkey) {
  const uint32_t nh = *nheads;
  const uint64_t lowmask = (1ull << kb) - 1ull;
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < ne; k += stride) {
    if (k >= nh) {
      rkey[k] = ~0ull;
      continue;
    }
    const uint32_t i = heads[k];
    const uint64_t kk = key[i];
    uint32_t bi = idx[i];
    uint32_t bw = ew[bi], bl = elab[bi];
    for (uint32_t j = i + 1; j < ne && key[j] == kk; j++) {
      const uint32_t c = idx[j];
      if (ew[c] < bw || (ew[c] == bw && elab[c] < bl)) {
        bi = c;
        bw = ew[c];
        bl = elab[c];
      }
    }
    ukey[k] = kk;
    uw[k] = bw;
    umid[k] = emid[bi];
    rkey[k] = ((kk & lowmask) << kb) | (kk >> kb);
  }
}

// ---------------------------------------------------------------------------
// disjoint-union batch preparation
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t graph_of(const uint32_t *vbase, uint32_t k, uint32_t v) {
  uint32_t lo = 0, hi = k;  // last g with vbase[g] <= v
  while (hi - lo > 1) {
    const uint32_t md = (lo + hi) >> 1;
    if (vbase[md] <= v) lo = md;
    else hi = md;
  }
  return lo;
}

// Union offsets from the graphs' own offsets (staged: graph g's n_g + 1
// values start at vbase[g] + g).  Also records the graph of each vertex and
// validates each graph's first and last offset.
__global__ void k_batch_offsets(uint32_t n, uint32_t k, const uint32_t *__restrict__ vbase,
                                const uint64_t *__restrict__ abase,
                                const uint64_t *__restrict__ stage, uint64_t *__restrict__ off,
                                uint32_t *__restrict__ gof, uint32_t *__restrict__ bad) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    const uint32_t g = graph_of(vbase, k, v);
    const uint32_t i = v - vbase[g];
    const uint64_t local = stage[(uint64_t)vbase[g] + g + i];
    const uint64_t mg = abase[g + 1] - abase[g];
    if (local > mg) {
      atomicOr(bad, 1u);
      off[v] = abase[g];
    } else {
      off[v] = abase[g] + local;
    }
    gof[v] = g;
    if (i == 0) {
      const uint32_t ng = vbase[g + 1] - vbase[g];
      if (local != 0 || stage[(uint64_t)vbase[g] + g + ng] != mg) atomicOr(bad, 8u);
    }
  }
}

// Shift arc heads into union ids; a head >= n_g is an error.
__global__ void k_batch_arcs(uint64_t m, uint32_t k, const uint32_t *__restrict__ vbase,
                             const uint64_t *__restrict__ abase, uint32_t *__restrict__ dst,
                             uint32_t *__restrict__ bad) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += stride) {
    uint32_t lo = 0, hi = k;  // last g with abase[g] <= e and a non-empty arc range
    while (hi - lo > 1) {
      const uint32_t md = (lo + hi) >> 1;
      if (abase[md] <= e) lo = md;
      else hi = md;
    }
    const uint32_t g = lo;
    const uint32_t ng = vbase[g + 1] - vbase[g];
    const uint32_t h = dst[e];
    if (h >= ng) {
      atomicOr(bad, 2u);
      dst[e] = vbase[g];
    } else {
      dst[e] = vbase[g] + h;
    }
  }
}

// Default labels per graph: fmix32(local id ^ mix), or the local id (raw).
__global__ void k_batch_default_labels(uint32_t n, uint32_t k, const uint32_t *__restrict__ vbase,
                                       uint32_t mix, bool raw, uint32_t *__restrict__ lab) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    const uint32_t l = v - vbase[graph_of(vbase, k, v)];
    lab[v] = raw ? l : fmix32(l ^ mix);
  }
}

// key = (graph << 32) | label, for the per-graph distinctness check.
__global__ void k_graph_label_keys(uint32_t n, const uint32_t *__restrict__ gof,
                                   const uint32_t *__restrict__ lab, uint64_t *__restrict__ key) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
    key[v] = ((uint64_t)gof[v] << 32) | lab[v];
}

// Row lengths of the (union) forward CSR summed per graph.
__global__ void k_rowlen_by_graph(uint32_t n, const uint32_t *__restrict__ foff,
                                  const uint32_t *__restrict__ gof,
                                  unsigned long long *__restrict__ cnt) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    const uint32_t len = foff[v + 1] - foff[v];
    if (len) atomicAdd(&cnt[gof[v]], (unsigned long long)len);
  }
}

// Arcs per graph (of the vertex `a[i]`), for splitting sorted arc lists.
__global__ void k_arcs_by_graph(uint64_t m, const uint32_t *__restrict__ a,
                                const uint32_t *__restrict__ gof,
                                unsigned long long *__restrict__ cnt) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride)
    atomicAdd(&cnt[gof[a[i]]], 1ull);
}

// Largest level per graph.
__global__ void k_level_max_by_graph(uint32_t n, const uint32_t *__restrict__ level,
                                     const uint32_t *__restrict__ gof, uint32_t *__restrict__ mx) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
    atomicMax(&mx[gof[v]], level[v] + 1);
}

// out[i] = in[i] - base (ids of one graph back to its local ids); SP_NOMID
// is kept when keep_nomid.
__global__ void k_sub_base(uint64_t m, const uint32_t *__restrict__ in, uint32_t base,
                           bool keep_nomid, uint32_t *__restrict__ out) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
    const uint32_t x = in[i];
    out[i] = (keep_nomid && x == SP_NOMID) ? x : x - base;
  }
}

// Batch bookkeeping: one count per distinct shortcut pair, by graph of v1.
__global__ void k_count_by_graph(const uint64_t *__restrict__ ukey, const uint32_t *nU, int kb,
                                 const uint32_t *__restrict__ gid, const uint32_t *__restrict__ gof,
                                 unsigned long long *__restrict__ cnt) {
  const uint32_t U = *nU;
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < U; i += stride)
    atomicAdd(&cnt[gof[gid[(uint32_t)(ukey[i] >> kb)]]], 1ull);
}

// ===========================================================================
// overlay rebuild
// ===========================================================================
// keep[u] = !F[u]; zeroes the row-count arrays c2, c3 (n + 1 entries) and
// the next round's flag arrays w, a (n entries).
__global__ void k_keep(uint32_t n, const uint8_t *__restrict__ F, uint32_t *__restrict__ keep,
                       uint32_t *__restrict__ c2, uint32_t *__restrict__ c3,
                       uint8_t *__restrict__ w, uint8_t *__restrict__ a) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u <= n; u += stride) {
    c2[u] = 0;
    c3[u] = 0;
    if (u == n) continue;
    keep[u] = !F[u];
    w[u] = 0;
    a[u] = 0;
  }
}

// Sequential merge of one row (the fallback for rows longer than a group's
// LDS share): old arcs (dead ones skipped) and the shortcut row, both sorted
// by neighbour; on a common neighbour the shortcut replaces the arc only if
// lighter.  Returns the merged length; MODE 1 also writes the merged row.
template <int MODE>
__device__ uint32_t merge_row_serial(uint32_t a, uint32_t a1, uint32_t b, uint32_t b1,
                                     uint64_t lowmask, const uint32_t *__restrict__ newid,
                                     const uint2 *__restrict__ arc, const uint32_t *__restrict__ mid,
                                     const uint64_t *__restrict__ ekey,
                                     const uint32_t *__restrict__ eidx,
                                     const uint32_t *__restrict__ uw,
                                     const uint32_t *__restrict__ umid, uint32_t outp,
                                     uint2 *__restrict__ narc, uint32_t *__restrict__ nmid) {
  uint32_t c = 0;
  for (;;) {
    while (a < a1 && arc[a].y == SP_INF32) a++;
    const bool ha = a < a1, hb = b < b1;
    if (!ha && !hb) break;
    const uint32_t va = ha ? arc[a].x : 0xFFFFFFFFu;
    const uint32_t vb = hb ? (uint32_t)(ekey[b] & lowmask) : 0xFFFFFFFFu;
    uint32_t v, ww, mm;
    if (ha && (!hb || va < vb)) {
      v = va;
      ww = arc[a].y;
      mm = mid[a];
      a++;
    } else if (!ha || vb < va) {
      const uint32_t r = eidx ? eidx[b] : b;
      v = vb;
      ww = uw[r];
      mm = umid[r];
      b++;
    } else {
      const uint32_t r = eidx ? eidx[b] : b;
      if (uw[r] < arc[a].y) {
        ww = uw[r];
        mm = umid[r];
      } else {
        ww = arc[a].y;
        mm = mid[a];
      }
      v = va;
      a++;
      b++;
    }
    if (MODE) {
      narc[outp] = make_uint2(newid[v], ww);
      nmid[outp] = mm;
      outp++;
    }
    c++;
  }
  return c;
}

// New overlay rows: per kept vertex u, its old row (arcs off[u] ..
// off[u+1], sorted by neighbour; dead ones -- pruned, or to a contracted
// vertex, marked by k_contract -- dropped) merged with its shortcut row
// (sorted keys (u << kb | v), bounds rfirst/rstop; eidx maps a key to its
// weight and middle vertex, or null for the identity); on a common neighbour
// the shortcut replaces the arc only if lighter (a tie keeps the arc).
// MODE 0 counts each merged row into cnt[newid[u]]; MODE 1 writes it at
// noff[newid[u]] with new neighbour ids.
//
// G lanes per row, each element placed independently: a live old arc to v
// lands after the live old arcs before it and the shortcuts to neighbours
// below v, less the shortcuts among those that share a neighbour with a live
// old arc; a shortcut to v without a live old arc to v lands after the live
// old arcs to neighbours below v and the shortcuts before it, less those
// that share a neighbour.  The live-arc prefix of the old row is kept in
// LDS; rows longer than the group's share take the sequential merge.
// One direction of the rebuild: old CSR (off, arc, mid), its shortcut rows
// (keys ekey, record map eidx or null, bounds rfirst/rstop), row counts cnt
// (MODE 0) or the new CSR (noff, narc, nmid; MODE 1).
struct MergeSide {
  const uint32_t *off;
  const uint2 *arc;
  const uint32_t *mid;
  const uint64_t *ekey;
  const uint32_t *eidx;
  const uint32_t *rfirst, *rstop;
  uint32_t *cnt;
  const uint32_t *noff;
  uint2 *narc;
  uint32_t *nmid;
};

// blockIdx.y selects the direction: 0 = fwd, 1 = rev.
template <int G, int MODE>
__global__ void __launch_bounds__(256) k_merge_rows(uint32_t n, int kb,
                                                    const uint8_t *__restrict__ F,
                                                    const uint32_t *__restrict__ newid,
                                                    const uint32_t *__restrict__ uw,
                                                    const uint32_t *__restrict__ umid,
                                                    MergeSide fwd, MergeSide rev) {
  const MergeSide &side = blockIdx.y ? rev : fwd;
  const uint32_t *__restrict__ off = side.off;
  const uint2 *__restrict__ arc = side.arc;
  const uint32_t *__restrict__ mid = side.mid;
  const uint64_t *__restrict__ ekey = side.ekey;
  const uint32_t *__restrict__ eidx = side.eidx;
  const uint32_t *__restrict__ rfirst = side.rfirst;
  const uint32_t *__restrict__ rstop = side.rstop;
  uint32_t *__restrict__ cnt = side.cnt;
  const uint32_t *__restrict__ noff = side.noff;
  uint2 *__restrict__ narc = side.narc;
  uint32_t *__restrict__ nmid = side.nmid;
  constexpr uint32_t kGroups = 256 / G;
  constexpr uint32_t kCap = 4096 / kGroups;  // live-arc prefix entries per group
  __shared__ uint16_t s_live[4096];
  uint16_t *lr = s_live + (threadIdx.x / G) * kCap;
  const uint64_t lowmask = (1ull << kb) - 1ull;
  const uint32_t ngroups = gridDim.x * kGroups;
  const uint32_t g0 = blockIdx.x * kGroups + threadIdx.x / G;
  const uint32_t gl = (uint32_t)glane<G>();
  const uint64_t below = gl == 0 ? 0ull : ((1ull << gl) - 1ull);
  for (uint32_t u = g0; u < n; u += ngroups) {
    if (F[u]) continue;
    const uint32_t a0 = off[u], na = off[u + 1] - a0;
    const uint32_t b0 = rfirst[u], nb = rstop[u] - b0;
    const uint32_t outp = MODE ? noff[newid[u]] : 0;
    if (na > kCap) {
      if (gl == 0) {
        const uint32_t c = merge_row_serial<MODE>(a0, a0 + na, b0, b0 + nb, lowmask, newid, arc,
                                                  mid, ekey, eidx, uw, umid, outp, narc, nmid);
        if (!MODE) cnt[newid[u]] = c;
      }
      continue;
    }
    // old arcs
    uint32_t live_n = 0, dup_n = 0;
    for (uint32_t x0 = 0; x0 < na; x0 += G) {
      const uint32_t i = x0 + gl;
      uint2 e = make_uint2(0u, SP_INF32);
      if (i < na) e = arc[a0 + i];
      const bool live = i < na && e.y != SP_INF32;
      uint32_t lb = 0;
      bool dup = false;
      if (live && nb) {  // first shortcut with neighbour >= e.x
        uint32_t lo = 0, hi = nb;
        while (lo < hi) {
          const uint32_t md = (lo + hi) >> 1;
          if ((uint32_t)(ekey[b0 + md] & lowmask) < e.x) lo = md + 1;
          else hi = md;
        }
        lb = lo;
        dup = lb < nb && (uint32_t)(ekey[b0 + lb] & lowmask) == e.x;
      }
      const uint64_t lm = gballot<G>(live), dm = gballot<G>(dup);
      const uint32_t lrank = live_n + (uint32_t)__popcll(lm & below);
      if (MODE && i < na) lr[i] = (uint16_t)lrank;
      if (MODE && live) {
        const uint32_t pos = lrank + lb - (dup_n + (uint32_t)__popcll(dm & below));
        uint32_t ww = e.y, mm;
        if (dup) {
          const uint32_t r = eidx ? eidx[b0 + lb] : b0 + lb;
          const uint32_t sw = uw[r];
          if (sw < e.y) {
            ww = sw;
            mm = umid[r];
          } else {
            mm = mid[a0 + i];
          }
        } else {
          mm = mid[a0 + i];
        }
        narc[outp + pos] = make_uint2(newid[e.x], ww);
        nmid[outp + pos] = mm;
      }
      live_n += (uint32_t)__popcll(lm);
      dup_n += (uint32_t)__popcll(dm);
    }
    wave_sync();  // the group's prefix entries are visible to all its lanes
    // shortcuts without a live old arc to the same neighbour
    if (MODE) {
      uint32_t in_n = 0;
      for (uint32_t y0 = 0; y0 < nb; y0 += G) {
        const uint32_t j = y0 + gl;
        const bool valid = j < nb;
        const uint32_t v = valid ? (uint32_t)(ekey[b0 + j] & lowmask) : 0u;
        uint32_t la = 0;
        bool in_a = false;
        if (valid) {  // first old arc with neighbour >= v
          uint32_t lo = 0, hi = na;
          while (lo < hi) {
            const uint32_t md = (lo + hi) >> 1;
            if (arc[a0 + md].x < v) lo = md + 1;
            else hi = md;
          }
          la = lo;
          if (la < na) {
            const uint2 e = arc[a0 + la];
            in_a = e.x == v && e.y != SP_INF32;
          }
        }
        const uint64_t im = gballot<G>(in_a);
        if (valid && !in_a) {
          const uint32_t live_below = la < na ? (uint32_t)lr[la] : live_n;
          const uint32_t pos = live_below + j - (in_n + (uint32_t)__popcll(im & below));
          const uint32_t r = eidx ? eidx[b0 + j] : b0 + j;
          narc[outp + pos] = make_uint2(newid[v], uw[r]);
          nmid[outp + pos] = umid[r];
        }
        in_n += (uint32_t)__popcll(im);
      }
    } else if (gl == 0) {
      cnt[newid[u]] = live_n + nb - dup_n;
    }
    wave_sync();  // before the next row overwrites the prefix entries
  }
}

// Carries per-vertex state to the new local ids and marks V_S in W'.
__global__ void k_carry(uint32_t n, const uint8_t *__restrict__ F, const uint32_t *__restrict__ newid,
                        const uint32_t *__restrict__ gid, const int32_t *__restrict__ P,
                        const uint8_t *__restrict__ S, const uint8_t *__restrict__ newA,
                        uint32_t *__restrict__ ngid, int32_t *__restrict__ nP,
                        uint8_t *__restrict__ nW, uint8_t *__restrict__ nA) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += stride) {
    if (F[u]) continue;
    const uint32_t nu = newid[u];
    ngid[nu] = gid[u];
    nP[nu] = P[u];
    nA[nu] = newA[u];
    if (S[u]) nW[nu] = 1;
  }
}

// V_W' = V_S union N_in(V_S) on the combined overlay.
__global__ void k_mark_in_neighbours(uint32_t n, const uint8_t *__restrict__ F,
                                     const uint8_t *__restrict__ S,
                                     const uint32_t *__restrict__ newid,
                                     const uint32_t *__restrict__ nroff,
                                     const uint2 *__restrict__ nrarc, uint8_t *__restrict__ nW) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += stride) {
    if (F[u] || !S[u]) continue;
    const uint32_t nu = newid[u];
    for (uint32_t e = nroff[nu]; e < nroff[nu + 1]; e++) nW[nrarc[e].x] = 1;
  }
}

// Entries of the memo whose endpoints are both live (the only ones looked up
// again: lookups and inserts always pair two live vertices).  Each thread
// takes four slots a stride apart per step, so all their key loads and then
// all their liveness loads are in flight together.
constexpr int kRehashBatch = 4;

__global__ void k_memo_count_live(const MemoSlot *__restrict__ old, uint64_t ocap,
                                  const uint8_t *__restrict__ alive_g,
                                  unsigned long long *__restrict__ live) {
  uint64_t c = 0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i0 < ocap;
       i0 += kRehashBatch * stride) {
    uint64_t k[kRehashBatch];
#pragma unroll
    for (int q = 0; q < kRehashBatch; q++) {
      const uint64_t i = i0 + q * stride;
      k[q] = i < ocap ? old[i].key : SP_EMPTY64;
    }
#pragma unroll
    for (int q = 0; q < kRehashBatch; q++)
      if (k[q] != SP_EMPTY64) c += alive_g[(uint32_t)(k[q] >> 32)] && alive_g[(uint32_t)k[q]];
  }
  c = gsum64<kWave>(c);
  if (lane_id() == 0 && c) atomicAdd(live, (unsigned long long)c);
}

// Memo rebuild: the live entries of `old` inserted into the empty table nt
// (its own size and source-region width), the others dropped.
__global__ void k_memo_rehash(const MemoSlot *__restrict__ old, uint64_t ocap,
                              const uint8_t *__restrict__ alive_g, MemoRef nt,
                              unsigned long long *__restrict__ kept) {
  uint64_t c = 0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i0 < ocap;
       i0 += kRehashBatch * stride) {
    ulonglong2 e[kRehashBatch];
#pragma unroll
    for (int q = 0; q < kRehashBatch; q++) {
      const uint64_t i = i0 + q * stride;
      e[q] = make_ulonglong2(SP_EMPTY64, 0ull);
      if (i < ocap) e[q] = *reinterpret_cast<const ulonglong2 *>(&old[i]);
    }
    bool keep[kRehashBatch];
#pragma unroll
    for (int q = 0; q < kRehashBatch; q++)
      keep[q] = e[q].x != SP_EMPTY64 && alive_g[(uint32_t)(e[q].x >> 32)] &&
                alive_g[(uint32_t)e[q].x];
#pragma unroll
    for (int q = 0; q < kRehashBatch; q++) {
      if (!keep[q]) continue;
      memo_put(nt, (uint32_t)(e[q].x >> 32), (uint32_t)e[q].x, (uint32_t)e[q].y);
      c++;
    }
  }
  c = gsum64<kWave>(c);
  if (lane_id() == 0 && c) atomicAdd(kept, (unsigned long long)c);
}

}  // namespace sp
