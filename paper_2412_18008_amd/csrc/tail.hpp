// tail.hpp -- the last rounds of an exact-mode build on a small overlay,
// with no host round trip per round.
//
// Once the overlay fits the all-pairs table (at most 4096 vertices), the
// remaining rounds of Alg. 3 run as a fixed sequence of five launches per
// round whose sizes live on the device: the host enqueues rounds in batches
// and reads the state back once per batch; launches after the last round
// return at once.  Vertices are table positions (0 .. n0 - 1) for the whole
// tail, so the overlay needs no renumbering between rounds:
//   - out- and in-arc bitmaps (n0 x rw words) say which arcs are live;
//   - W and MID (n0 x n0) hold the weight and middle vertex of arc (a, b);
//   - ol / il (n0 x n0, row stride n0) list each vertex's out- and
//     in-neighbours, unsorted, compacted once per round;
//   - the memo is the bitmap E of pairs (s, t) with an entry; the entry's
//     value is the table distance D[s][t] (overlay distances do not change
//     from round to round, so every entry, old or new, holds exactly that);
//   - shortcut candidates meet in SC[a][b] = min((via << 12) | label rank),
//     which is the E+ rule (smallest weight, then smallest label of the
//     middle vertex) without a sort.
// Row order never matters: searches, counts and the E+ minimum are order
// free, and the CH arc lists are sorted by rank afterwards.
#pragma once

#include "common.hpp"
#include "round_kernels.hpp"

namespace sp {

constexpr int kTailBlock = 256;
constexpr int kTailWaves = kTailBlock / kWave;
constexpr uint32_t kTailMaxN = 4096;  // positions fit 12 bits
constexpr int kTailPaths = 4;        // two-arc paths per lane in flight (search)

// Device state of the tail; list counts and flags are indexed by the
// parity of the round (cur = this round's, nxt = the next round's); every
// kernel takes the parity and the round number from the device counter of
// finished rounds, so a batch of rounds has fixed launch arguments (and is
// replayed as one captured graph).
struct TailCtr {
  uint32_t done;    // set once no vertex is left, the round limit is hit or an error is set
  uint32_t live;    // live vertices
  uint32_t rounds;  // rounds completed
  uint32_t nf, ntouched;
  uint32_t blocks;  // blocks of the merge launch that have finished
  uint32_t cntW[2], cntA[2];
  unsigned long long m;  // live overlay arcs
  unsigned long long targets, pruned, rows, arcs, probes, added;
  unsigned long long up_n, dn_n, up_prev, dn_prev;  // CH arcs written (total, before this round)
  unsigned long long clk0;  // wall clock before the first round
};

// One record per completed round (the host turns it into round stats).
struct TailRound {
  uint32_t alive_before, n_sources, n_affected, n_selected;
  unsigned long long n_targets, n_pruned, n_shortcuts, overlay_arcs;
  unsigned long long rows, arcs, probes;
  unsigned long long clk;  // wall clock at the end of the round
};

struct TailArgs {
  uint32_t n0, rw;  // vertices, bitmap words per row
  const uint32_t *D;
  uint32_t N;              // all-pairs table, row stride N
  const uint32_t *gidp;    // original id of each position
  uint32_t *lab;           // label of each position
  uint32_t *lrank;         // rank of that label among the n0 labels
  uint32_t *plr;           // position of each label rank
  uint32_t *ob, *ib, *eb;  // out-arc, in-arc and memo-entry bitmaps
  uint32_t *W, *MID;
  uint16_t *ol, *il;
  uint32_t *olen, *ilen;
  unsigned long long *SC;
  uint32_t *touched;  // pairs (a << 12) | b with an SC entry this round
  int32_t *P;         // priority (edge difference)
  uint32_t *alive;
  uint32_t *af0, *af1, *wf0, *wf1;  // V_A and V_W flags by parity
  uint16_t *la0, *la1, *lw0, *lw1;  // their lists
  uint32_t *sflag;                  // V_S of this round
  TailCtr *C;
  uint32_t *err;
};

__device__ __forceinline__ bool tbit(const uint32_t *bm, uint32_t rw, uint32_t r, uint32_t c) {
  return (bm[(size_t)r * rw + (c >> 5)] >> (c & 31)) & 1u;
}
__device__ __forceinline__ void tclear(uint32_t *bm, uint32_t rw, uint32_t r, uint32_t c) {
  atomicAnd(&bm[(size_t)r * rw + (c >> 5)], ~(1u << (c & 31)));
}
__device__ __forceinline__ void tset(uint32_t *bm, uint32_t rw, uint32_t r, uint32_t c) {
  atomicOr(&bm[(size_t)r * rw + (c >> 5)], 1u << (c & 31));
}
// Appends x to list `l` (count *cnt) the first time flag[x] is raised.
__device__ __forceinline__ void tmark(uint32_t *flag, uint16_t *l, uint32_t *cnt, uint32_t x) {
  if (atomicExch(&flag[x], 1u) == 0u) l[atomicAdd(cnt, 1u)] = (uint16_t)x;
}
__device__ __forceinline__ uint32_t tvia(uint32_t x, uint32_t y) {
  const uint64_t s = (uint64_t)x + y;
  return s > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)s;
}

// ---------------------------------------------------------------------------
// set-up (once): bitmaps cleared, SC emptied, both parities' flags zero
// ---------------------------------------------------------------------------
__global__ void k_tail_clear(TailArgs A) {
  const uint64_t nb = 3ull * A.n0 * A.rw, nn = (uint64_t)A.n0 * A.n0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t t0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (uint64_t i = t0; i < nb; i += stride) A.ob[i] = 0;  // ob, ib, eb are contiguous
  for (uint64_t i = t0; i < nn; i += stride) A.SC[i] = SP_EMPTY64;
  for (uint64_t i = t0; i < A.n0; i += stride) {
    A.af0[i] = A.af1[i] = A.wf0[i] = A.wf1[i] = 0;
    A.sflag[i] = 0;
  }
}

// Rows, weights and per-vertex state of the current overlay (local ids are
// the table positions); V_A from the affected flags, V_W from the source list.
__global__ void k_tail_load(TailArgs A, Overlay ov, const int32_t *__restrict__ P,
                            const uint8_t *__restrict__ aflag, const uint32_t *__restrict__ vw,
                            uint32_t nw, const uint32_t *__restrict__ label) {
  const uint32_t stride = gridDim.x * blockDim.x;
  const uint32_t t0 = blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long m = 0;
  for (uint32_t u = t0; u < A.n0; u += stride) {
    uint32_t c = 0;
    for (uint32_t e = ov.foff[u]; e < ov.foff[u + 1]; e++) {
      const uint2 a = ov.farc[e];
      if (a.y == SP_INF32) continue;
      A.ol[(size_t)u * A.n0 + c++] = (uint16_t)a.x;
      A.W[(size_t)u * A.n0 + a.x] = a.y;
      A.MID[(size_t)u * A.n0 + a.x] = ov.fmid[e];
      tset(A.ob, A.rw, u, a.x);
    }
    A.olen[u] = c;
    m += c;
    c = 0;
    for (uint32_t e = ov.roff[u]; e < ov.roff[u + 1]; e++) {
      const uint2 a = ov.rarc[e];
      if (a.y == SP_INF32) continue;
      A.il[(size_t)u * A.n0 + c++] = (uint16_t)a.x;
      tset(A.ib, A.rw, u, a.x);
    }
    A.ilen[u] = c;
    A.P[u] = P[u];
    A.alive[u] = 1;
    A.lab[u] = label[A.gidp[u]];
    if (aflag[u]) tmark(A.af0, A.la0, &A.C->cntA[0], u);
  }
  for (uint32_t k = t0; k < nw; k += stride) tmark(A.wf0, A.lw0, &A.C->cntW[0], vw[k]);
  if (t0 == 0) A.C->live = A.n0;
  if (m) atomicAdd(&A.C->m, m);
}

// Memo entries between two live vertices become bits of E.
__global__ void k_tail_memo(TailArgs A, const MemoSlot *__restrict__ t, uint64_t cap,
                            const uint8_t *__restrict__ alive_g,
                            const uint32_t *__restrict__ pos_of_gid) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cap; i += stride) {
    const uint64_t k = t[i].key;
    if (k == SP_EMPTY64) continue;
    const uint32_t s = (uint32_t)(k >> 32), v = (uint32_t)k;
    if (!alive_g[s] || !alive_g[v]) continue;
    const uint32_t ps = pos_of_gid[s], pv = pos_of_gid[v];
    if (ps < A.n0 && pv < A.n0) tset(A.eb, A.rw, ps, pv);
    else atomicOr(A.err, kErrCapacity);
  }
}

// Rank of each position's label among the n0 labels (labels are distinct).
__global__ void k_tail_lrank(TailArgs A) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < A.n0; p += stride) {
    const uint32_t x = A.lab[p];
    uint32_t r = 0;
    for (uint32_t q = 0; q < A.n0; q++) r += A.lab[q] < x;
    A.lrank[p] = r;
    A.plr[r] = p;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) A.C->clk0 = wall_clock64();
}

// ---------------------------------------------------------------------------
// per round
// ---------------------------------------------------------------------------
#define TAIL_WAVE_LOOP(k, count)                                                    \
  for (uint32_t k = blockIdx.x * kTailWaves + threadIdx.x / kWave; k < (count); \
       k += gridDim.x * kTailWaves)

// Step 1 (Alg. 4), answered from the table: per source s, the targets are
// the vertices v != s two arcs away through an affected out-neighbour with
// no memo entry (s, v); the search radius D_s is the longest such two-arc
// path; every target gets its entry.  Then pruning: an out-arc (s, v)
// heavier than the memoized dist(s, v) is deleted.  The searches read only
// the lists and weights, which pruning does not change, so they see the
// overlay as it was at the start of the round.  One wave per source.
__global__ void __launch_bounds__(kTailBlock) k_tail_search(TailArgs A) {
  TailCtr *C = A.C;
  if (C->done) return;
  const uint32_t cur = C->rounds & 1u;
  const uint32_t nw = C->cntW[cur];
  const uint16_t *lw = cur ? A.lw1 : A.lw0;
  const uint32_t *af = cur ? A.af1 : A.af0;
  __shared__ uint32_t s_new[kTailWaves][kTailMaxN / 32];
  uint32_t *nb = s_new[threadIdx.x / kWave];
  const int l = lane_id();
  const uint32_t n0 = A.n0, rw = A.rw;
  for (uint32_t i = l; i < rw; i += kWave) nb[i] = 0;
  wave_sync();
  uint64_t rows = 0, arcs = 0, probes = 0, targets = 0, pruned = 0;
  TAIL_WAVE_LOOP(k, nw) {
    const uint32_t s = lw[k];
    const uint16_t *os = A.ol + (size_t)s * n0;
    const uint32_t ds = A.olen[s];
    const uint32_t *es = A.eb + (size_t)s * rw;
    uint32_t dmax = 0;
    for (uint32_t b0 = 0; b0 < ds; b0 += kWave) {
      const uint32_t e = b0 + l;
      uint32_t u = 0, rl = 0, wsu = 0;
      if (e < ds) {
        u = os[e];
        if (af[u]) {
          rl = A.olen[u];
          wsu = A.W[(size_t)s * n0 + u];
          rows++;
        }
      }
      const uint32_t incl = gscan_incl<kWave>(rl);
      const uint32_t total = __shfl(incl, kWave - 1, kWave);
      // kTailPaths paths per lane: their list entries, then their memo
      // words and weights, are loaded together before any is used
      for (uint32_t i0 = 0; i0 < total; i0 += kWave * kTailPaths) {
        uint32_t v[kTailPaths], su[kTailPaths], sw[kTailPaths];
        bool ok[kTailPaths];
#pragma unroll
        for (int q = 0; q < kTailPaths; q++) {
          const uint32_t idx = i0 + q * kWave + l;
          ok[q] = false;
          v[q] = su[q] = sw[q] = 0;
          if (i0 + q * kWave < total) {  // uniform across the wave
            const int src = gfind<kWave>(incl, idx);
            su[q] = __shfl(u, src, kWave);
            sw[q] = __shfl(wsu, src, kWave);
            const uint32_t sinc = __shfl(incl, src, kWave), srl = __shfl(rl, src, kWave);
            if (idx < total) {
              v[q] = A.ol[(size_t)su[q] * n0 + (idx - (sinc - srl))];
              ok[q] = true;
            }
          }
        }
        uint32_t ew[kTailPaths], wv2[kTailPaths];
#pragma unroll
        for (int q = 0; q < kTailPaths; q++) {
          ew[q] = wv2[q] = 0;
          if (!ok[q]) continue;
          arcs++;
          if (v[q] == s) {
            ok[q] = false;
            continue;
          }
          probes++;
          ew[q] = es[v[q] >> 5];
          wv2[q] = A.W[(size_t)su[q] * n0 + v[q]];
        }
#pragma unroll
        for (int q = 0; q < kTailPaths; q++) {
          if (!ok[q] || ((ew[q] >> (v[q] & 31)) & 1u)) continue;
          dmax = max(dmax, tvia(sw[q], wv2[q]));
          atomicOr(&nb[v[q] >> 5], 1u << (v[q] & 31));
        }
      }
    }
    wave_sync();
    uint32_t nt = 0;
    for (uint32_t i = l; i < rw; i += kWave) nt += __popc(nb[i]);
    nt = gsum<kWave>(nt);
    dmax = gmax<kWave>(dmax);
    if (nt && dmax > SP_MAXW && l == 0) atomicOr(A.err, kErrOverflow);
    targets += l == 0 ? nt : 0;
    // pruning against the entries, the new ones included
    for (uint32_t e = l; e < ds; e += kWave) {
      const uint32_t v = os[e];
      const bool has = ((es[v >> 5] | nb[v >> 5]) >> (v & 31)) & 1u;
      if (!has) continue;
      const uint32_t w = A.W[(size_t)s * n0 + v], d = A.D[(size_t)s * A.N + v];
      if (w == SP_INF32 || d == SP_INF32 || w <= d) continue;
      tclear(A.ob, rw, s, v);
      tclear(A.ib, rw, v, s);
      pruned++;
    }
    wave_sync();
    if (nt) {
      uint32_t *esw = A.eb + (size_t)s * rw;
      for (uint32_t i = l; i < rw; i += kWave) {
        const uint32_t x = nb[i];
        if (x) esw[i] |= x;
      }
    }
    for (uint32_t i = l; i < rw; i += kWave) nb[i] = 0;
    wave_sync();
  }
  rows = gsum64<kWave>(rows);
  arcs = gsum64<kWave>(arcs);
  probes = gsum64<kWave>(probes);
  targets = gsum64<kWave>(targets);
  pruned = gsum64<kWave>(pruned);
  if (l == 0) {
    if (rows) atomicAdd(&C->rows, (unsigned long long)rows);
    if (arcs) atomicAdd(&C->arcs, (unsigned long long)arcs);
    if (probes) atomicAdd(&C->probes, (unsigned long long)probes);
    if (targets) atomicAdd(&C->targets, (unsigned long long)targets);
    if (pruned) atomicAdd(&C->pruned, (unsigned long long)pruned);
  }
}

// Pair (i, j) of N_in(u) x N_out(u) is a shortcut candidate when both arcs
// are live, the ends differ and the path through u is no longer than the
// memoized distance (or there is no entry).  kTailPairs pairs per thread,
// p0 + q * stride, with the loads of each kind issued together.
constexpr int kTailPairs = 4;
struct TailPairs {
  uint32_t a[kTailPairs], b[kTailPairs], via[kTailPairs];
  bool cand[kTailPairs];
};
__device__ __forceinline__ void tail_pairs(const TailArgs &A, uint32_t u, uint32_t p0,
                                           uint32_t stride, uint32_t np, uint32_t dout,
                                           TailPairs &r) {
  const size_t rowu = (size_t)u * A.n0;
  const uint32_t *ibu = A.ib + (size_t)u * A.rw, *obu = A.ob + (size_t)u * A.rw;
  bool act[kTailPairs];
#pragma unroll
  for (int q = 0; q < kTailPairs; q++) {
    const uint32_t p = p0 + q * stride;
    act[q] = p < np;
    r.a[q] = r.b[q] = 0;
    if (act[q]) {
      const uint32_t i = p / dout, j = p - i * dout;
      r.a[q] = A.il[rowu + i];
      r.b[q] = A.ol[rowu + j];
    }
  }
  uint32_t wa[kTailPairs], wb[kTailPairs], ew[kTailPairs];
  bool live[kTailPairs];
#pragma unroll
  for (int q = 0; q < kTailPairs; q++) {
    const uint32_t a = r.a[q], b = r.b[q];
    live[q] = act[q] && a != b && ((ibu[a >> 5] >> (a & 31)) & 1u) && ((obu[b >> 5] >> (b & 31)) & 1u);
  }
#pragma unroll
  for (int q = 0; q < kTailPairs; q++) {
    wa[q] = wb[q] = ew[q] = 0;
    if (live[q]) {
      wa[q] = A.W[(size_t)r.a[q] * A.n0 + u];
      wb[q] = A.W[rowu + r.b[q]];
      ew[q] = A.eb[(size_t)r.a[q] * A.rw + (r.b[q] >> 5)];
    }
  }
  uint32_t d[kTailPairs];
#pragma unroll
  for (int q = 0; q < kTailPairs; q++) {
    d[q] = SP_INF32;
    if (live[q] && ((ew[q] >> (r.b[q] & 31)) & 1u)) d[q] = A.D[(size_t)r.a[q] * A.N + r.b[q]];
  }
#pragma unroll
  for (int q = 0; q < kTailPairs; q++) {
    const uint64_t via = (uint64_t)wa[q] + wb[q];
    r.via[q] = via > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)via;
    // no entry (d stays SP_INF32) or a path through u no longer than it
    r.cand[q] = live[q] && (d[q] == SP_INF32 || via <= d[q]);
  }
}

// Step 2 (Alg. 5): edge difference of every affected vertex, one block each.
__global__ void __launch_bounds__(kTailBlock) k_tail_score(TailArgs A) {
  TailCtr *C = A.C;
  if (C->done) return;
  const uint32_t cur = C->rounds & 1u;
  const uint32_t na = C->cntA[cur];
  const uint16_t *la = cur ? A.la1 : A.la0;
  __shared__ uint32_t s_red[kTailWaves][3];
  const int l = lane_id();
  const uint32_t wv = threadIdx.x / kWave;
  for (uint32_t k = blockIdx.x; k < na; k += gridDim.x) {
    const uint32_t u = la[k];
    const uint32_t din = A.ilen[u], dout = A.olen[u];
    const uint32_t np = din * dout;
    uint32_t pairs = 0;
    for (uint32_t p0 = threadIdx.x; p0 < np; p0 += kTailBlock * kTailPairs) {
      TailPairs r;
      tail_pairs(A, u, p0, kTailBlock, np, dout, r);
#pragma unroll
      for (int q = 0; q < kTailPairs; q++) pairs += r.cand[q];
    }
    uint32_t cout = 0, only_in = 0;
    const size_t rowu = (size_t)u * A.n0;
    for (uint32_t e = threadIdx.x; e < dout; e += kTailBlock)
      cout += tbit(A.ob, A.rw, u, A.ol[rowu + e]);
    for (uint32_t e = threadIdx.x; e < din; e += kTailBlock) {
      const uint32_t a = A.il[rowu + e];
      if (tbit(A.ib, A.rw, u, a)) only_in += !tbit(A.ob, A.rw, u, a);
    }
    pairs = gsum<kWave>(pairs);
    cout = gsum<kWave>(cout);
    only_in = gsum<kWave>(only_in);
    if (l == 0) {
      s_red[wv][0] = pairs;
      s_red[wv][1] = cout;
      s_red[wv][2] = only_in;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t p = 0;
#pragma unroll
      for (int x = 0; x < kTailWaves; x++)
        p += (int64_t)s_red[x][0] - (int64_t)s_red[x][1] - (int64_t)s_red[x][2];
      p = p > INT32_MAX ? INT32_MAX : (p < INT32_MIN ? INT32_MIN : p);
      A.P[u] = (int32_t)p;
    }
    __syncthreads();
  }
}

// Steps 3 and 4 (Alg. 6 and 7) in one launch.  Select: u is selected iff
// its key (priority, label) is below every live neighbour's; a wave decides
// for one vertex.  Contract, by the whole block for each vertex its waves
// selected: live out-arcs go to the upward set and live in-arcs to the
// downward set, the neighbours join the next V_A, and every candidate pair
// lowers SC[a][b]; its first candidate lists the pair, and a joins V_S (so
// the next V_W; sflag marks V_S).  Contraction clears no bit: the twins of
// the moved arcs stay set until the compaction drops every entry to a dead
// vertex, so the selections in this launch all see the same overlay, and
// the rows a contraction reads (its own) change in no way meanwhile.
__global__ void __launch_bounds__(kTailBlock) k_tail_selcon(TailArgs A,
                                                            uint32_t round0, ArcOut up, ArcOut dn,
                                                            uint64_t up_base, uint64_t dn_base,
                                                            uint64_t up_cap, uint64_t dn_cap,
                                                            uint32_t *__restrict__ level,
                                                            int32_t *__restrict__ score,
                                                            uint8_t *__restrict__ alive_g) {
  TailCtr *C = A.C;
  if (C->done) return;
  const uint32_t cur = C->rounds & 1u, round = round0 + C->rounds;
  const uint32_t nxt = cur ^ 1u;
  uint32_t *afn = nxt ? A.af1 : A.af0;
  uint32_t *wfn = nxt ? A.wf1 : A.wf0;
  uint16_t *lan = nxt ? A.la1 : A.la0;
  uint16_t *lwn = nxt ? A.lw1 : A.lw0;
  __shared__ uint32_t s_sel[kTailWaves];
  const int l = lane_id();
  const uint32_t wv = threadIdx.x / kWave;
  const uint64_t below = l == 0 ? 0ull : ((1ull << l) - 1ull);
  const uint32_t n0 = A.n0, rw = A.rw;
  auto key = [&](uint32_t x) {
    return ((uint64_t)((uint32_t)A.P[x] ^ 0x80000000u) << 32) | A.lab[x];
  };
  for (uint32_t base = blockIdx.x * kTailWaves; base < n0; base += gridDim.x * kTailWaves) {
    const uint32_t u = base + wv;
    bool sel = false;
    if (u < n0 && A.alive[u]) {
      const uint64_t ku = key(u);
      const size_t rowu = (size_t)u * n0;
      bool beaten = false;
      for (uint32_t e = l; e < A.olen[u]; e += kWave) {
        const uint32_t v = A.ol[rowu + e];
        beaten |= tbit(A.ob, rw, u, v) && key(v) < ku;
      }
      for (uint32_t e = l; e < A.ilen[u]; e += kWave) {
        const uint32_t a = A.il[rowu + e];
        beaten |= tbit(A.ib, rw, u, a) && key(a) < ku;
      }
      sel = !gany<kWave>(beaten);
    }
    if (l == 0) s_sel[wv] = sel ? u : 0xFFFFFFFFu;
    __syncthreads();
    for (int x = 0; x < kTailWaves; x++) {
      const uint32_t cu = s_sel[x];
      if (cu == 0xFFFFFFFFu) continue;  // uniform over the block
      const uint32_t gu = A.gidp[cu];
      const size_t rowu = (size_t)cu * n0;
      if (threadIdx.x == 0) {
        level[gu] = round;
        score[gu] = A.P[cu];
        alive_g[gu] = 0;
        A.alive[cu] = 0;
        atomicAdd(&C->nf, 1u);
      }
      const uint32_t dout = A.olen[cu], din = A.ilen[cu];
      for (uint32_t b0 = wv * kWave; b0 < dout; b0 += kTailBlock) {
        const uint32_t e = b0 + l;
        uint32_t v = 0;
        bool live = false;
        if (e < dout) {
          v = A.ol[rowu + e];
          live = tbit(A.ob, rw, cu, v);
        }
        const uint64_t msk = __ballot(live);
        unsigned long long at0 = 0;
        if (l == 0 && msk) at0 = atomicAdd(&C->up_n, (unsigned long long)__popcll(msk));
        at0 = __shfl(at0, 0, kWave);
        if (live) {
          const uint64_t at = up_base + at0 + __popcll(msk & below);
          if (at < up_cap) {
            up.t[at] = gu;
            up.h[at] = A.gidp[v];
            up.w[at] = A.W[rowu + v];
            up.m[at] = A.MID[rowu + v];
          } else {
            atomicOr(A.err, kErrCapacity);
          }
          tmark(afn, lan, &C->cntA[nxt], v);
        }
      }
      for (uint32_t b0 = wv * kWave; b0 < din; b0 += kTailBlock) {
        const uint32_t e = b0 + l;
        uint32_t a = 0;
        bool live = false;
        if (e < din) {
          a = A.il[rowu + e];
          live = tbit(A.ib, rw, cu, a);
        }
        const uint64_t msk = __ballot(live);
        unsigned long long at0 = 0;
        if (l == 0 && msk) at0 = atomicAdd(&C->dn_n, (unsigned long long)__popcll(msk));
        at0 = __shfl(at0, 0, kWave);
        if (live) {
          const uint64_t at = dn_base + at0 + __popcll(msk & below);
          if (at < dn_cap) {
            dn.t[at] = A.gidp[a];
            dn.h[at] = gu;
            dn.w[at] = A.W[(size_t)a * n0 + cu];
            dn.m[at] = A.MID[(size_t)a * n0 + cu];
          } else {
            atomicOr(A.err, kErrCapacity);
          }
          tmark(afn, lan, &C->cntA[nxt], a);
        }
      }
      const uint32_t np = din * dout;
      const uint32_t lr = A.lrank[cu];
      for (uint32_t p0 = threadIdx.x; p0 < np; p0 += kTailBlock * kTailPairs) {
        TailPairs r;
        tail_pairs(A, cu, p0, kTailBlock, np, dout, r);
#pragma unroll
        for (int q = 0; q < kTailPairs; q++) {
          if (!r.cand[q]) continue;
          if (r.via[q] > SP_MAXW) {
            atomicOr(A.err, kErrOverflow);
            continue;
          }
          const unsigned long long val = ((unsigned long long)r.via[q] << 12) | lr;
          if (atomicMin(&A.SC[(size_t)r.a[q] * n0 + r.b[q]], val) == SP_EMPTY64)
            A.touched[atomicAdd(&C->ntouched, 1u)] = (r.a[q] << 12) | r.b[q];
          A.sflag[r.a[q]] = 1;
          tmark(wfn, lwn, &C->cntW[nxt], r.a[q]);
        }
      }
    }
    __syncthreads();  // s_sel is rewritten next
  }
}

// Drops the dead entries (pruned arcs, arcs to contracted vertices) from
// the lists of the live vertices; the live in-neighbours of a V_S vertex
// join the next V_W.
__global__ void __launch_bounds__(kTailBlock) k_tail_compact(TailArgs A) {
  TailCtr *C = A.C;
  if (C->done) return;
  const uint32_t cur = C->rounds & 1u;
  const uint32_t nxt = cur ^ 1u;
  uint32_t *wfn = nxt ? A.wf1 : A.wf0;
  uint16_t *lwn = nxt ? A.lw1 : A.lw0;
  const int l = lane_id();
  const uint64_t below = l == 0 ? 0ull : ((1ull << l) - 1ull);
  TAIL_WAVE_LOOP(u, A.n0) {
    if (!A.alive[u]) continue;
    const size_t rowu = (size_t)u * A.n0;
    const bool in_s = A.sflag[u] != 0;
    for (int side = 0; side < 2; side++) {
      uint16_t *lst = (side ? A.il : A.ol) + rowu;
      const uint32_t *bm = side ? A.ib : A.ob;
      uint32_t *len = side ? &A.ilen[u] : &A.olen[u];
      const uint32_t n = *len;
      uint32_t kept = 0;
      for (uint32_t b0 = 0; b0 < n; b0 += kWave) {
        const uint32_t e = b0 + l;
        uint32_t x = 0;
        bool keep = false;
        if (e < n) {
          x = lst[e];
          keep = tbit(bm, A.rw, u, x) && A.alive[x];
        }
        const uint64_t msk = __ballot(keep);
        if (keep) {
          lst[kept + __popcll(msk & below)] = (uint16_t)x;
          if (side && in_s) tmark(wfn, lwn, &C->cntW[nxt], x);
        }
        kept += (uint32_t)__popcll(msk);
        wave_sync();
      }
      if (l == 0) *len = kept;
    }
  }
}

// Overlay rebuild: each E+ pair (a, b) with its minimal (weight, label) --
// a live arc (a, b) takes the shortcut's weight and middle vertex only if
// the shortcut is lighter (a tie keeps the arc); otherwise the pair becomes
// a new arc, and a joins the next V_W when b is in V_S.  SC is emptied for
// the next round.  The last block to finish ends the round: its record,
// this round's flags cleared (they serve the round after next), the
// counters of the next round, and the stop condition.  A round with an
// error is not recorded.
__global__ void __launch_bounds__(kTailBlock) k_tail_merge_end(TailArgs A, uint32_t max_rounds,
                                                               TailRound *__restrict__ rec,
                                                               uint32_t rec_cap) {
  TailCtr *C = A.C;
  if (C->done) return;
  // the last block increments C->rounds only after every block has finished
  const uint32_t cur = C->rounds & 1u;
  const uint32_t nxt = cur ^ 1u;
  uint32_t *wfn = nxt ? A.wf1 : A.wf0;
  uint16_t *lwn = nxt ? A.lw1 : A.lw0;
  const uint32_t nt = C->ntouched;
  const uint32_t stride = gridDim.x * blockDim.x;
  uint64_t added = 0;
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < nt; t += stride) {
    const uint32_t pr = A.touched[t];
    const uint32_t a = pr >> 12, b = pr & 0xFFFu;
    const size_t ab = (size_t)a * A.n0 + b;
    const unsigned long long val = A.SC[ab];
    A.SC[ab] = SP_EMPTY64;
    const uint32_t w = (uint32_t)(val >> 12);
    const uint32_t mid = A.gidp[A.plr[(uint32_t)(val & 0xFFFu)]];
    if (tbit(A.ob, A.rw, a, b)) {
      if (w < A.W[ab]) {
        A.W[ab] = w;
        A.MID[ab] = mid;
      }
      continue;
    }
    A.W[ab] = w;
    A.MID[ab] = mid;
    tset(A.ob, A.rw, a, b);
    tset(A.ib, A.rw, b, a);
    A.ol[(size_t)a * A.n0 + atomicAdd(&A.olen[a], 1u)] = (uint16_t)b;
    A.il[(size_t)b * A.n0 + atomicAdd(&A.ilen[b], 1u)] = (uint16_t)a;
    if (A.sflag[b]) tmark(wfn, lwn, &C->cntW[nxt], a);
    added++;
  }
  added = gsum64<kWave>(added);
  if (lane_id() == 0 && added) atomicAdd(&C->added, (unsigned long long)added);

  // ---- end of the round, by the last block
  __shared__ uint32_t s_last;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    s_last = atomicAdd(&C->blocks, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  uint32_t *af = cur ? A.af1 : A.af0;
  uint32_t *wf = cur ? A.wf1 : A.wf0;
  const uint16_t *la = cur ? A.la1 : A.la0;
  const uint16_t *lw = cur ? A.lw1 : A.lw0;
  const uint32_t na = C->cntA[cur], nw = C->cntW[cur];
  for (uint32_t i = threadIdx.x; i < na; i += blockDim.x) af[la[i]] = 0;
  for (uint32_t i = threadIdx.x; i < nw; i += blockDim.x) wf[lw[i]] = 0;
  for (uint32_t i = threadIdx.x; i < A.n0; i += blockDim.x) A.sflag[i] = 0;
  __syncthreads();
  if (threadIdx.x != 0) return;
  C->blocks = 0;
  if (*A.err || C->nf == 0 || C->rounds >= rec_cap) {
    if (C->nf == 0 || C->rounds >= rec_cap) atomicOr(A.err, kErrCapacity);
    C->done = 1;
    return;
  }
  const unsigned long long moved = (C->up_n - C->up_prev) + (C->dn_n - C->dn_prev);
  const unsigned long long m2 = C->m - C->pruned - moved + C->added;
  TailRound r;
  r.alive_before = C->live;
  r.n_sources = nw;
  r.n_affected = na;
  r.n_selected = C->nf;
  r.n_targets = C->targets;
  r.n_pruned = C->pruned;
  r.n_shortcuts = C->ntouched;
  r.overlay_arcs = m2;
  r.rows = C->rows;
  r.arcs = C->arcs;
  r.probes = C->probes;
  r.clk = wall_clock64();
  rec[C->rounds] = r;
  C->live -= C->nf;
  C->m = m2;
  C->rounds++;
  C->nf = C->ntouched = 0;
  C->targets = C->pruned = C->rows = C->arcs = C->probes = C->added = 0;
  C->up_prev = C->up_n;
  C->dn_prev = C->dn_n;
  C->cntA[cur] = C->cntW[cur] = 0;
  if (C->live == 0 || C->rounds >= max_rounds) C->done = 1;
}

#undef TAIL_WAVE_LOOP

}  // namespace sp
