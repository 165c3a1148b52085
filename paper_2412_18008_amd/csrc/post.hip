// post.hip -- Postprocessing (re-index by level, then score) and the batched
// s-t query on the finished contraction hierarchy, for gfx950.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <map>
#include <mutex>
#include <type_traits>
#include <string>

#include "builder.hpp"
#include "common.hpp"

namespace sp {

#define HIP_TRY(expr)                                   \
  do {                                                  \
    hipError_t e_ = (expr);                             \
    if (e_ != hipSuccess) return hip_error(e_, #expr);  \
  } while (0)
#define TRY(expr)               \
  do {                          \
    int r_ = (expr);            \
    if (r_ != CH_OK) return r_; \
  } while (0)

// Default level window of the query: none.  With the searches pruned by the
// shortest path met so far and by stall-on-demand, expanding every flagged
// vertex at once is fastest (road1m, 182 levels: 17.2 ms per 100k queries,
// 18.9-24.6 ms with windows of 128 down to 16 levels; road24m, 412 levels:
// 1.00 s per 1M before the core table, 1.08-2.10 s with windows).  A
// hierarchy deeper than kQShallow levels starts its first query batch in
// the second tier, which also holds the core table: started in the first
// tier, about 36% of the road24m queries outgrow its tables (1.11 s per 1M
// then, against 1.00 s).
constexpr uint32_t kQShallow = 256;

static int bits_for(uint32_t n) {
  int b = 1;
  while (b < 32 && (1ull << b) < (uint64_t)n) b++;
  return b;
}

// ===========================================================================
// postprocess kernels
// ===========================================================================
__global__ void k_label_keys(uint32_t n, const uint32_t *__restrict__ label,
                             uint64_t *__restrict__ key, uint32_t *__restrict__ val) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    key[v] = label[v];
    val[v] = v;
  }
}

// (level, score) key of the vertex at each position of the label order.
__global__ void k_level_keys(uint32_t n, const uint32_t *__restrict__ order,
                             const uint32_t *__restrict__ level, const int32_t *__restrict__ score,
                             uint64_t *__restrict__ key) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const uint32_t v = order[i];
    key[i] = ((uint64_t)level[v] << 32) | ((uint32_t)score[v] ^ 0x80000000u);
  }
}

__global__ void k_graph_keys(uint32_t n, const uint32_t *__restrict__ order,
                             const uint32_t *__restrict__ gof, uint64_t *__restrict__ key) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) key[i] = gof[order[i]];
}

__global__ void k_rank_from_order(uint32_t n, const uint32_t *__restrict__ order,
                                  uint32_t *__restrict__ rank) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) rank[order[i]] = i;
}

// key = (rank[a] << kb) | rank[b] for arc list (a[i], b[i]).
__global__ void k_arc_rank_keys(uint64_t m, const uint32_t *__restrict__ a,
                                const uint32_t *__restrict__ b, const uint32_t *__restrict__ rank,
                                int kb, uint64_t *__restrict__ key, uint32_t *__restrict__ val) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
    key[i] = ((uint64_t)rank[a[i]] << kb) | rank[b[i]];
    val[i] = (uint32_t)i;
  }
}

__global__ void k_gather4(uint64_t m, const uint32_t *__restrict__ perm, const uint32_t *__restrict__ s0,
                          const uint32_t *__restrict__ s1, const uint32_t *__restrict__ s2,
                          const uint32_t *__restrict__ s3, uint32_t *__restrict__ d0,
                          uint32_t *__restrict__ d1, uint32_t *__restrict__ d2,
                          uint32_t *__restrict__ d3) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
    const uint32_t p = perm[i];
    d0[i] = s0[p];
    d1[i] = s1[p];
    d2[i] = s2[p];
    d3[i] = s3[p];
  }
}

// Query index from arcs sorted by key = (row rank << kb) | other rank.
__global__ void k_index(uint32_t n, uint64_t m, int kb, const uint64_t *__restrict__ key,
                        const uint32_t *__restrict__ w, uint32_t *__restrict__ off,
                        uint2 *__restrict__ arc) {
  const uint64_t lowmask = (1ull << kb) - 1ull;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += stride) {
    const uint64_t target = (uint64_t)i << kb;
    uint64_t lo = 0, hi = m;
    while (lo < hi) {
      const uint64_t md = (lo + hi) >> 1;
      if (key[md] < target) lo = md + 1;
      else hi = md;
    }
    off[i] = (uint32_t)lo;
  }
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride)
    arc[i] = make_uint2((uint32_t)(key[i] & lowmask), w[i]);
}

unsigned gridn(uint64_t items);
unsigned gridn(uint64_t items) {
  uint64_t g = (items + 255) / 256;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return (unsigned)g;
}

// Sorts one arc set (t, h, w, mid) by (rank[row side], rank[other side]) and
// builds its query index.  up = true: row = tail; up = false: row = head.
static int sort_arcs(ch_s *ch, bool up, DBuf &k1, DBuf &k2, DBuf &v1, DBuf &v2, DBuf &tmp,
                     bool make_index) {
  hipStream_t st = ch->stream;
  const uint64_t m = up ? ch->nup : ch->ndown;
  DBuf &t = up ? ch->up_t : ch->dn_t;
  DBuf &h = up ? ch->up_h : ch->dn_h;
  DBuf &w = up ? ch->up_w : ch->dn_w;
  DBuf &mid = up ? ch->up_m : ch->dn_m;
  const int kb = bits_for(ch->n);
  if (m >= 0xFFFFFFFFull) return set_error(CH_E_UNSUPPORTED, "too many CH arcs");
  const size_t m1 = std::max<uint64_t>(m, 1);
  HIP_TRY(k1.ensure(m1 * 8));
  HIP_TRY(k2.ensure(m1 * 8));
  HIP_TRY(v1.ensure(m1 * 4));
  HIP_TRY(v2.ensure(m1 * 4));
  if (m) {
    k_arc_rank_keys<<<gridn(m), 256, 0, st>>>(m, up ? t.as<uint32_t>() : h.as<uint32_t>(),
                                              up ? h.as<uint32_t>() : t.as<uint32_t>(),
                                              ch->rank.as<uint32_t>(), kb, k1.as<uint64_t>(),
                                              v1.as<uint32_t>());
    HIP_TRY(hipGetLastError());
    HIP_TRY(radix_sort_u64(k1.as<uint64_t>(), v1.as<uint32_t>(), k2.as<uint64_t>(),
                           v2.as<uint32_t>(), (uint32_t)m, 2 * kb, tmp, st));
  }
  DBuf nt, nh, nw, nm;
  HIP_TRY(nt.ensure(m1 * 4));
  HIP_TRY(nh.ensure(m1 * 4));
  HIP_TRY(nw.ensure(m1 * 4));
  HIP_TRY(nm.ensure(m1 * 4));
  if (m) {
    k_gather4<<<gridn(m), 256, 0, st>>>(m, v1.as<uint32_t>(), t.as<uint32_t>(), h.as<uint32_t>(),
                                        w.as<uint32_t>(), mid.as<uint32_t>(), nt.as<uint32_t>(),
                                        nh.as<uint32_t>(), nw.as<uint32_t>(), nm.as<uint32_t>());
    HIP_TRY(hipGetLastError());
  }
  HIP_TRY(hipStreamSynchronize(st));
  t.release();
  h.release();
  w.release();
  mid.release();
  t = nt;
  h = nh;
  w = nw;
  mid = nm;
  if (make_index) {
    DBuf &off = up ? ch->q_upoff : ch->q_dnoff;
    DBuf &arc = up ? ch->q_uparc : ch->q_dnarc;
    HIP_TRY(off.ensure(((size_t)ch->n + 1) * 4));
    HIP_TRY(arc.ensure(m1 * 8));
    k_index<<<gridn(std::max<uint64_t>(m, (uint64_t)ch->n + 1)), 256, 0, st>>>(
        ch->n, m, kb, k1.as<uint64_t>(), w.as<uint32_t>(), off.as<uint32_t>(), arc.as<uint2>());
    HIP_TRY(hipGetLastError());
  }
  return CH_OK;
}

// Level of the vertex at each rank.
__global__ void k_level_by_rank(uint32_t n, const uint32_t *__restrict__ rank,
                                const uint32_t *__restrict__ level, uint32_t *__restrict__ lvr) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
    lvr[rank[v]] = level[v];
}

// lstart[L] = the first rank whose level is >= L, for L <= nlev (levels do
// not decrease along the ranks).
__global__ void k_level_starts(uint32_t n, const uint32_t *__restrict__ lvr, uint32_t nlev,
                               uint32_t *__restrict__ lstart) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t L = blockIdx.x * blockDim.x + threadIdx.x; L <= nlev; L += stride) {
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
      const uint32_t md = (lo + hi) >> 1;
      if (lvr[md] < L) lo = md + 1;
      else hi = md;
    }
    lstart[L] = lo;
  }
}

// End of the level window of `win` levels that starts at each rank: the
// first rank of level level(v) + win + 1 (n past the last level).  Always
// above the rank itself.
__global__ void k_window_ends(uint32_t n, const uint32_t *__restrict__ rank,
                              const uint32_t *__restrict__ level,
                              const uint32_t *__restrict__ lstart, uint32_t nlev, uint32_t win,
                              uint32_t *__restrict__ wend) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    const uint64_t e = (uint64_t)level[v] + win + 1;
    wend[rank[v]] = lstart[e < nlev ? e : nlev];
  }
}

// First rank of every level, for the query's level window.
static int level_starts(ch_s *ch) {
  hipStream_t st = ch->stream;
  const uint32_t nlev = ch->rounds + 1;  // covers every level
  DBuf lvr;
  HIP_TRY(lvr.ensure((size_t)std::max<uint32_t>(ch->n, 1) * 4));
  HIP_TRY(ch->q_lstart.ensure(((size_t)nlev + 1) * 4));
  // level-window ends, filled by the first query batch that uses a window
  HIP_TRY(ch->q_wend.ensure((size_t)std::max<uint32_t>(ch->n, 1) * 4));
  ch->q_first_tier = ch->rounds > kQShallow ? 2 : 1;
  if (ch->n)
    k_level_by_rank<<<gridn(ch->n), 256, 0, st>>>(ch->n, ch->rank.as<uint32_t>(),
                                                  ch->level.as<uint32_t>(), lvr.as<uint32_t>());
  k_level_starts<<<gridn((uint64_t)nlev + 1), 256, 0, st>>>(ch->n, lvr.as<uint32_t>(), nlev,
                                                            ch->q_lstart.as<uint32_t>());
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(st));
  lvr.release();
  ch->q_nlev = nlev;
  ch->q_wend_win = 0;
  return CH_OK;
}

// Query index of a CH whose arc lists are already sorted by rank.
int build_index(ch_s *ch) {
  hipStream_t st = ch->stream;
  const int kb = bits_for(ch->n);
  DBuf k1, v1;
  for (int dir = 0; dir < 2; dir++) {
    const bool up = dir == 0;
    const uint64_t m = up ? ch->nup : ch->ndown;
    const size_t m1 = std::max<uint64_t>(m, 1);
    DBuf &off = up ? ch->q_upoff : ch->q_dnoff;
    DBuf &arc = up ? ch->q_uparc : ch->q_dnarc;
    HIP_TRY(k1.ensure(m1 * 8));
    HIP_TRY(v1.ensure(m1 * 4));
    HIP_TRY(off.ensure(((size_t)ch->n + 1) * 4));
    HIP_TRY(arc.ensure(m1 * 8));
    if (m) {
      k_arc_rank_keys<<<gridn(m), 256, 0, st>>>(
          m, up ? ch->up_t.as<uint32_t>() : ch->dn_h.as<uint32_t>(),
          up ? ch->up_h.as<uint32_t>() : ch->dn_t.as<uint32_t>(), ch->rank.as<uint32_t>(), kb,
          k1.as<uint64_t>(), v1.as<uint32_t>());
      HIP_TRY(hipGetLastError());
    }
    k_index<<<gridn(std::max<uint64_t>(m, (uint64_t)ch->n + 1)), 256, 0, st>>>(
        ch->n, m, kb, k1.as<uint64_t>(), up ? ch->up_w.as<uint32_t>() : ch->dn_w.as<uint32_t>(),
        off.as<uint32_t>(), arc.as<uint2>());
    HIP_TRY(hipGetLastError());
  }
  HIP_TRY(hipStreamSynchronize(st));
  k1.release();
  v1.release();
  const int rc = level_starts(ch);
  if (rc != CH_OK) return rc;
  ch->has_index = true;
  return CH_OK;
}

// Postprocessing: vertices are ordered by level, then by score at
// contraction (low to high), then by label; the CH arcs are re-keyed to the
// new ranks and sorted.
int postprocess(ch_s *ch, bool make_index, const uint32_t *gof, uint32_t kgraphs) {
  hipStream_t st = ch->stream;
  const uint32_t n = ch->n;
  const size_t n1 = std::max<uint32_t>(n, 1);
  DBuf k1, k2, v1, v2, tmp;
  int rc = CH_OK;
  do {
    hipError_t e;
    if ((e = k1.ensure(n1 * 8)) != hipSuccess || (e = k2.ensure(n1 * 8)) != hipSuccess ||
        (e = v1.ensure(n1 * 4)) != hipSuccess ||
        (e = v2.ensure(n1 * 4)) != hipSuccess || (e = ch->rank.ensure(n1 * 4)) != hipSuccess) {
      rc = hip_error(e, "postprocess alloc");
      break;
    }
    if (n) {
      k_label_keys<<<gridn(n), 256, 0, st>>>(n, ch->label.as<uint32_t>(), k1.as<uint64_t>(),
                                             v1.as<uint32_t>());
      if ((e = radix_sort_u64(k1.as<uint64_t>(), v1.as<uint32_t>(), k2.as<uint64_t>(),
                              v2.as<uint32_t>(), n, 32, tmp, st)) != hipSuccess) {
        rc = hip_error(e, "rank sort");
        break;
      }
      k_level_keys<<<gridn(n), 256, 0, st>>>(n, v1.as<uint32_t>(), ch->level.as<uint32_t>(),
                                             ch->score.as<int32_t>(), k1.as<uint64_t>());
      const int lb = bits_for(ch->rounds + 1);
      if ((e = radix_sort_u64(k1.as<uint64_t>(), v1.as<uint32_t>(), k2.as<uint64_t>(),
                              v2.as<uint32_t>(), n, 32 + lb, tmp, st)) != hipSuccess) {
        rc = hip_error(e, "rank sort");
        break;
      }
      if (gof && kgraphs > 1) {  // disjoint-union batch: graph id is the major key
        k_graph_keys<<<gridn(n), 256, 0, st>>>(n, v1.as<uint32_t>(), gof, k1.as<uint64_t>());
        if ((e = radix_sort_u64(k1.as<uint64_t>(), v1.as<uint32_t>(), k2.as<uint64_t>(),
                                v2.as<uint32_t>(), n, bits_for(kgraphs), tmp, st)) != hipSuccess) {
          rc = hip_error(e, "rank sort");
          break;
        }
      }
      k_rank_from_order<<<gridn(n), 256, 0, st>>>(n, v1.as<uint32_t>(), ch->rank.as<uint32_t>());
      if ((e = hipGetLastError()) != hipSuccess) {
        rc = hip_error(e, "rank");
        break;
      }
    }
    if ((rc = sort_arcs(ch, true, k1, k2, v1, v2, tmp, make_index)) != CH_OK) break;
    if ((rc = sort_arcs(ch, false, k1, k2, v1, v2, tmp, make_index)) != CH_OK) break;
    if (make_index && (rc = level_starts(ch)) != CH_OK) break;
    ch->has_index = make_index;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) rc = hip_error(e, "postprocess");
  } while (0);
  k1.release();
  k2.release();
  v1.release();
  v2.release();
  tmp.release();
  return rc;
}

// ===========================================================================
// query: one wave per query; upward closures of s (upward arcs) and of t
// (downward arcs, walked backwards) in two vertex -> distance tables, then
// the minimum of d_s(v) + d_t(v) over common vertices.  Label-correcting
// relaxation gives exact closure distances in any order, and because every
// tentative value is the length of a real path, the minimum is exact.
// ===========================================================================
enum : uint32_t { kQFront = 1u };

// Vertex -> distance table of one search direction.  DistT is uint32_t in
// LDS (a sum above 0xFFFFFFFE marks the query for the 64-bit path) or
// unsigned long long in the global-memory fallback.
template <typename IdxT, typename DistT, bool GL>
struct QTab {
  uint32_t *key;
  DistT *dist;
  uint32_t *flag;
  IdxT *order, *fr0, *fr1;
  uint32_t *ctr;  // used, |fr0|, |fr1|, overflow
  uint32_t cap, shift, limit;

  __device__ __forceinline__ uint32_t ld(const uint32_t *p) const {
    if constexpr (GL) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else return *p;
  }
  __device__ __forceinline__ void st(uint32_t *p, uint32_t v) const {
    if constexpr (GL) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else *p = v;
  }
  __device__ __forceinline__ DistT ldd(const DistT *p) const {
    if constexpr (GL) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else return *p;
  }
  __device__ __forceinline__ void std_(DistT *p, DistT v) const {
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
  __device__ __forceinline__ int insert(uint32_t v) const {
    uint32_t h = (v * 0x9E3779B1u) >> shift;
    for (uint32_t probes = 0; probes < cap; probes++) {
      uint32_t k = ld(&key[h]);
      if (k == v) return (int)h;
      if (k == SP_EMPTY32) {
        uint32_t prev = atomicCAS(&key[h], SP_EMPTY32, v);
        if (prev == SP_EMPTY32) {
          uint32_t idx = atomicAdd(&ctr[0], 1u);
          if (idx < limit) sti(&order[idx], (IdxT)h);
          else atomicOr(&ctr[3], 1u);
          return (int)h;
        }
        if (prev == v) return (int)h;
      }
      h = (h + 1) & (cap - 1);
    }
    atomicOr(&ctr[3], 1u);
    return -1;
  }
  __device__ __forceinline__ int find(uint32_t v) const {
    uint32_t h = (v * 0x9E3779B1u) >> shift;
    for (uint32_t probes = 0; probes < cap; probes++) {
      uint32_t k = ld(&key[h]);
      if (k == v) return (int)h;
      if (k == SP_EMPTY32) return -1;
      h = (h + 1) & (cap - 1);
    }
    return -1;
  }
};

template <typename IdxT, typename DistT, bool GL>
__device__ void qtab_reset(const QTab<IdxT, DistT, GL> &T) {
  const int l = lane_id();
  T.sync();
  uint32_t used = T.ld(&T.ctr[0]);
  if (used > T.limit) used = T.limit;
  for (uint32_t i = l; i < used; i += kWave) {
    IdxT s = T.ldi(&T.order[i]);
    T.st(&T.key[s], SP_EMPTY32);
    T.std_(&T.dist[s], (DistT)~(DistT)0);
    T.st(&T.flag[s], 0u);
  }
  T.sync();
  if (used >= T.limit) {
    for (uint32_t i = l; i < T.cap; i += kWave) {
      T.st(&T.key[i], SP_EMPTY32);
      T.std_(&T.dist[i], (DistT)~(DistT)0);
      T.st(&T.flag[i], 0u);
    }
  }
  if (l < 4) T.st(&T.ctr[l], 0u);
  T.sync();
}

// Upward closure from `src` over (off, arc).  Returns false on overflow of
// the table or of the distance type.
template <typename IdxT, typename DistT, bool GL>
__device__ bool closure(const QTab<IdxT, DistT, GL> &T, const uint32_t *__restrict__ off,
                        const uint2 *__restrict__ arc, uint32_t src, uint32_t &nrows,
                        uint32_t &narcs) {
  const int l = lane_id();
  constexpr unsigned long long kMax = sizeof(DistT) == 4 ? 0xFFFFFFFEull : 0xFFFFFFFFFFFFFFFEull;
  T.sync();
  if (l == 0) {
    const int s = T.insert(src);
    if (s >= 0) {
      T.std_(&T.dist[s], (DistT)0);
      T.st(&T.flag[s], kQFront);
      T.sti(&T.fr0[0], (IdxT)s);
      T.st(&T.ctr[1], 1u);
    }
  }
  T.sync();
  int cur = 0;
  while (!T.ld(&T.ctr[3])) {
    IdxT *fc = cur ? T.fr1 : T.fr0;
    IdxT *fn = cur ? T.fr0 : T.fr1;
    uint32_t *nc = &T.ctr[cur ? 2 : 1];
    uint32_t *nn = &T.ctr[cur ? 1 : 2];
    const uint32_t ncur = T.ld(nc);
    if (ncur == 0) break;
    T.sync();
    if (l == 0) T.st(nn, 0u);
    T.sync();
    for (uint32_t fb = 0; fb < ncur; fb += kWave) {
      const uint32_t i = fb + l;
      uint32_t rs = 0, rl = 0;
      unsigned long long dx = 0;
      if (i < ncur) {
        const IdxT x = T.ldi(&fc[i]);
        atomicAnd(&T.flag[x], ~kQFront);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        dx = T.ldd(&T.dist[x]);
        const uint32_t vx = T.ld(&T.key[x]);
        rs = off[vx];
        rl = off[vx + 1] - rs;
        nrows++;
        narcs += rl;
      }
      const uint32_t incl = gscan_incl<kWave>(rl);
      const uint32_t total = __shfl(incl, kWave - 1, kWave);
      for (uint32_t i0 = 0; i0 < total; i0 += kWave) {
        const uint32_t idx = i0 + l;
        const int srcl = gfind<kWave>(incl, idx);
        const uint32_t srs = __shfl(rs, srcl, kWave), sinc = __shfl(incl, srcl, kWave);
        const uint32_t srl = __shfl(rl, srcl, kWave);
        const unsigned long long sdx = __shfl(dx, srcl, kWave);
        if (idx < total) {
          const uint2 b = arc[srs + (idx - (sinc - srl))];
          const unsigned long long nd = sdx + b.y;
          if (nd > kMax) {
            atomicOr(&T.ctr[3], 1u);
          } else {
            const int y = T.insert(b.x);
            if (y >= 0) {
              const DistT old = atomicMin(&T.dist[y], (DistT)nd);
              if ((DistT)nd < old) {
                const uint32_t f = atomicOr(&T.flag[y], kQFront);
                if (!(f & kQFront)) {
                  const uint32_t p = atomicAdd(nn, 1u);
                  if (p < T.cap) T.sti(&fn[p], (IdxT)y);
                }
              }
            }
          }
        }
        T.sync();
        if (T.ld(&T.ctr[3])) break;
      }
      if (T.ld(&T.ctr[3])) break;
    }
    T.sync();
    cur ^= 1;
  }
  T.sync();
  return !T.ld(&T.ctr[3]);
}

template <typename IdxT, typename DistT, bool GL>
__device__ unsigned long long meet(const QTab<IdxT, DistT, GL> &Fw, const QTab<IdxT, DistT, GL> &Bw) {
  const int l = lane_id();
  unsigned long long best = SP_INF64;
  const uint32_t used = Fw.ld(&Fw.ctr[0]);
  for (uint32_t i = l; i < used; i += kWave) {
    const IdxT s = Fw.ldi(&Fw.order[i]);
    const int b = Bw.find(Fw.ld(&Fw.key[s]));
    if (b >= 0) {
      const unsigned long long c =
          (unsigned long long)Fw.ldd(&Fw.dist[s]) + (unsigned long long)Bw.ldd(&Bw.dist[b]);
      best = c < best ? c : best;
    }
  }
  return gmin64<kWave>(best);
}

// ---------------------------------------------------------------------------
// Bitmap-frontier query: both upward closures of one query at once.  Each
// direction has TOP + CAP distance slots and one frontier bit per slot: the
// TOP highest ranks (the top of the hierarchy, which most upward searches
// reach) have a slot each, indexed by rank - (n - TOP); every other vertex
// goes to an open-addressing table of CAP (vertex, distance) slots.  A step
// takes up to LIST flagged slots of both directions (clearing their bits),
// expands them, and flags each slot whose distance dropped; the closures are
// complete when no bit is set.  With a level window of W levels a step
// expands, per direction, only the flagged vertices whose CH level is at most
// W above the lowest flagged level (ranks are ordered by level, so this is a
// rank bound: the window end of the lowest flagged rank); the others stay
// flagged.  All in-arcs of a vertex come from lower levels, so vertices are
// rarely expanded before their distance is final, at the price of more
// steps.  Results do not depend on W or LIST: every tentative distance is a
// path length, and the search ends only when no distance can drop.  Arc
// loads of a step are issued kQUnroll deep per lane before any is used.
// A query moves to the next tier when a table passes 7/8 of CAP or a
// distance passes 32 bits.  NW waves share one query's tables, which live in
// LDS (GM = false) or in global memory (GM = true: one table set per block,
// reached through L2).
// ---------------------------------------------------------------------------
constexpr int kQUnroll = 8;

template <uint32_t CAP, uint32_t TOP = 0, uint32_t LIST = 2 * (CAP * 7 / 8)>
struct QLds {
  static constexpr uint32_t kSlots = TOP + CAP;
  using Entry = typename std::conditional<(2 * kSlots <= 65536), uint16_t, uint32_t>::type;
  static constexpr uint32_t kLimit = CAP * 7 / 8;
  static constexpr uint32_t kWords = kSlots / 32;
  static constexpr uint32_t kShift = 32 - __builtin_ctz(CAP);
  static constexpr uint32_t kTop = TOP;
  static constexpr uint32_t kList = LIST;
  uint32_t key[2][CAP];      // hashed part
  uint32_t dist[2][kSlots];  // dense top part, then hashed part
  uint32_t bits[2][kWords];
  Entry list[LIST];          // flagged slots of one step: dir * kSlots + slot
  uint32_t used[2];          // hashed entries
  uint32_t usedt[2];         // dense entries
  uint32_t ovf;
  uint32_t next[2];    // index of the block's current query (low, high word)
  uint32_t wsum[16];
  uint32_t wsum2[16];  // a second scan within one step
  unsigned long long wmin[16];
  unsigned long long mu;  // shortest s-t path length met so far (pruning bound)
};
// Tier 1: a slot per rank for the 2048 highest ranks, 512-slot tables for
// the rest (on a road-like 1M CH at most about 250 vertices of a search
// space lie below the top 2048 ranks); five blocks per CU.
using QTier1 = QLds<512, 2048, 2048>;
using QTier2 = QLds<4096, 8192, 4096>;
constexpr uint32_t kQCore = 4096;  // core ranks of tier 2 (within its 8192 rank slots)
constexpr uint64_t kQCoreBatch = 4096;  // smallest batch that builds a core table
constexpr uint32_t kQCore1 = 1024;  // core ranks of tier 1 (within its 2048 rank slots)
using QTier3 = QLds<16384>;
constexpr int kQTier1PerCU = 5;
static_assert(sizeof(QTier1) * kQTier1PerCU <= 163840, "five tier-1 query blocks per CU");
static_assert(sizeof(QTier2) + 8 * 16 <= 163840, "one tier-2 query block per CU");

// Table accessors: plain LDS accesses, or device-coherent ones for tables in
// global memory (written by other waves' atomics, which bypass the CU's
// vector L1).
template <bool GM>
__device__ __forceinline__ uint32_t qld(const uint32_t *p) {
  if constexpr (GM) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
template <bool GM>
__device__ __forceinline__ void qst(uint32_t *p, uint32_t v) {
  if constexpr (GM) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else *p = v;
}
template <bool GM>
__device__ __forceinline__ unsigned long long qld64(const unsigned long long *p) {
  if constexpr (GM) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
template <bool GM>
__device__ __forceinline__ void qst64(unsigned long long *p, unsigned long long v) {
  if constexpr (GM) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
template <bool GM, typename E>
__device__ __forceinline__ E qlde(const E *p) {
  if constexpr (GM) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else return *p;
}
template <bool GM, typename E>
__device__ __forceinline__ void qste(E *p, E v) {
  if constexpr (GM) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else *p = v;
}

template <int NW, bool GM>
__device__ __forceinline__ void qsync() {
  if constexpr (GM) __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "agent");
  if constexpr (NW == 1) wave_sync();
  else __syncthreads();
}

// Slot of v in direction d (inserted if absent); *fresh = 1 when inserted
// here; -1 when the table is full.
template <bool GM, typename L>
__device__ __forceinline__ int qins(L &S, uint32_t d, uint32_t v, uint32_t *fresh) {
  constexpr uint32_t CAP = sizeof(S.key[0]) / 4;
  uint32_t h = (v * 0x9E3779B1u) >> L::kShift;
  for (uint32_t probes = 0; probes < CAP; probes++) {
    const uint32_t k = qld<GM>(&S.key[d][h]);
    if (k == v) return (int)h;
    if (k == SP_EMPTY32) {
      const uint32_t prev = atomicCAS(&S.key[d][h], SP_EMPTY32, v);
      if (prev == SP_EMPTY32) {
        *fresh = 1;
        return (int)h;
      }
      if (prev == v) return (int)h;
    }
    h = (h + 1) & (CAP - 1);
  }
  return -1;
}

template <bool GM, typename L>
__device__ __forceinline__ int qfind(const L &S, uint32_t d, uint32_t v) {
  constexpr uint32_t CAP = sizeof(S.key[0]) / 4;
  uint32_t h = (v * 0x9E3779B1u) >> L::kShift;
  for (uint32_t probes = 0; probes < CAP; probes++) {
    const uint32_t k = qld<GM>(&S.key[d][h]);
    if (k == v) return (int)h;
    if (k == SP_EMPTY32) return -1;
    h = (h + 1) & (CAP - 1);
  }
  return -1;
}

// Block-wide exclusive prefix of c over NW waves; *total = the block sum.
template <int NW, bool GM, typename L>
__device__ __forceinline__ uint32_t qscan(L &S, uint32_t c, uint32_t *total, uint32_t *ws) {
  const uint32_t incl = gscan_incl<kWave>(c);
  if constexpr (NW == 1) {
    *total = __shfl(incl, kWave - 1, kWave);
    return incl - c;
  } else {
    const int wv = threadIdx.x / kWave;
    if (lane_id() == kWave - 1) qst<GM>(&ws[wv], incl);
    qsync<NW, GM>();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < NW; i++) {
      const uint32_t x = qld<GM>(&ws[i]);
      before += i < wv ? x : 0u;
      all += x;
    }
    // wsum is written again only after the step's later barriers
    *total = all;
    return before + incl - c;
  }
}

// qscan that also returns the block minima of m0 and m1 (through wmin,
// which is free until the end of a query).
template <int NW, bool GM, typename L>
__device__ __forceinline__ uint32_t qscan_min(L &S, uint32_t c, uint32_t m0, uint32_t m1,
                                              uint32_t *total, uint32_t *M0, uint32_t *M1) {
  const uint32_t incl = gscan_incl<kWave>(c);
  m0 = gmin<kWave>(m0);
  m1 = gmin<kWave>(m1);
  if constexpr (NW == 1) {
    *total = __shfl(incl, kWave - 1, kWave);
    *M0 = m0;
    *M1 = m1;
    return incl - c;
  } else {
    const int wv = threadIdx.x / kWave;
    uint32_t *wm = reinterpret_cast<uint32_t *>(S.wmin);
    if (lane_id() == kWave - 1) {
      qst<GM>(&S.wsum[wv], incl);
      qst<GM>(&wm[2 * wv], m0);
      qst<GM>(&wm[2 * wv + 1], m1);
    }
    qsync<NW, GM>();
    uint32_t before = 0, all = 0, a0 = SP_EMPTY32, a1 = SP_EMPTY32;
#pragma unroll
    for (int i = 0; i < NW; i++) {
      const uint32_t x = qld<GM>(&S.wsum[i]);
      before += i < wv ? x : 0u;
      all += x;
      a0 = min(a0, qld<GM>(&wm[2 * i]));
      a1 = min(a1, qld<GM>(&wm[2 * i + 1]));
    }
    *total = all;
    *M0 = a0;
    *M1 = a1;
    return before + incl - c;
  }
}

template <bool GM, typename L>
__device__ __forceinline__ void qclear(L &S, uint32_t tid, uint32_t nt) {
  constexpr uint32_t CAP = sizeof(S.key[0]) / 4;
  for (uint32_t i = tid; i < CAP; i += nt) {
    qst<GM>(&S.key[0][i], SP_EMPTY32);
    qst<GM>(&S.key[1][i], SP_EMPTY32);
  }
  for (uint32_t i = tid; i < L::kSlots; i += nt) {
    qst<GM>(&S.dist[0][i], SP_INF32);
    qst<GM>(&S.dist[1][i], SP_INF32);
  }
  for (uint32_t i = tid; i < 2 * L::kWords; i += nt)
    qst<GM>(&S.bits[i / L::kWords][i % L::kWords], 0u);
  if (tid < 2) {
    qst<GM>(&S.used[tid], 0u);
    qst<GM>(&S.usedt[tid], 0u);
  }
  if (tid == 0) qst<GM>(&S.ovf, 0u);
}

// Queries: list ? list[i] for i < *nlist : i for i < q, taken one at a time
// by the blocks from the counter *work (so blocks that draw large queries
// take fewer).  Queries that do not fit go to ovf_list (count in
// *ovf_count).  GM: gtab holds one L per block.
// Core table (tiers 1 and 2): a query does not expand the CORE highest ranks; it
// takes min over pairs (a, b) of core vertices reached from s and from t of
// d_s(a) + D[a][b] + d_t(b), with D the exact distances among them (the CH
// arcs among the highest ranks keep those distances: a shortest up-down path
// between two of them climbs from the lower one).  A shortest s-t path whose
// highest vertex is in the core enters it at some a and leaves it at some b,
// and its two ends are found exactly below the core; every other path is met
// as before.  CORE = 0: no core (kQCore1 and kQCore, the core sizes, are
// defined with the tier tables).

template <int NW, typename L, bool GM, int CORE = 0>
__global__ void __launch_bounds__(64 * NW) k_query(
    uint64_t q, uint32_t n, const uint32_t *__restrict__ list,
    const uint32_t *__restrict__ nlist, uint32_t *__restrict__ bad,
    const uint32_t *__restrict__ qs, const uint32_t *__restrict__ qt,
    const uint32_t *__restrict__ rank, const uint32_t *__restrict__ upoff,
    const uint2 *__restrict__ uparc, const uint32_t *__restrict__ dnoff,
    const uint2 *__restrict__ dnarc, unsigned long long *__restrict__ dist,
    uint32_t *__restrict__ visited, uint32_t *__restrict__ ovf_list,
    uint32_t *__restrict__ ovf_count, const uint32_t *__restrict__ wend,
    unsigned long long *__restrict__ work, L *__restrict__ gtab,
    unsigned long long *__restrict__ qcount, uint32_t prune,
    const uint32_t *__restrict__ coreD = nullptr, uint32_t core0 = 0xFFFFFFFFu,
    uint32_t coreN = 0, uint32_t coreK = 0) {
  using E = typename L::Entry;
  constexpr uint32_t CAP = sizeof(((L *)nullptr)->key[0]) / 4;
  constexpr uint32_t TOP = L::kTop, NS = L::kSlots;
  constexpr bool kLds = !GM;
  __shared__ typename std::conditional<kLds, L, char>::type sh;
  L &S = *(GM ? gtab + blockIdx.x : reinterpret_cast<L *>(&sh));
  constexpr uint32_t NT = 64 * NW;
  constexpr uint32_t kW2 = 2 * L::kWords;  // bitmap words of both directions
  const uint32_t tid = threadIdx.x;
  const int l = lane_id();
  const uint32_t wv = tid / kWave;
  const uint64_t nq = list ? (uint64_t)*nlist : q;
  // ranks >= tbase have a dense slot (rank - tbase)
  const uint32_t tbase = TOP ? (n > TOP ? n - TOP : 0u) : 0xFFFFFFFFu;
  // slot of v in direction d, inserted into the hashed part if absent
  // (*fresh = 1 then); -1 when the hashed part is full
  auto slot_of = [&](uint32_t d, uint32_t v, uint32_t *fresh) -> int {
    if (TOP && v >= tbase) return (int)(v - tbase);
    const int h = qins<GM>(S, d, v, fresh);
    return h < 0 ? -1 : (int)TOP + h;
  };
  auto rank_of = [&](uint32_t d, uint32_t slot) -> uint32_t {
    return (TOP && slot < TOP) ? tbase + slot : qld<GM>(&S.key[d][slot - TOP]);
  };
  // Stall-on-demand (pruned searches only).  Vertex x, reached in direction
  // d at distance dx, is not expanded when some higher-ranked u with a CH arc
  // between them that points along the search (u -> x for the search from s,
  // x -> u for the one from t) gives d(u) + w < dx: d(u) is a real path
  // length, so dx is not the distance of x, and every path that leaves x
  // upward is beaten by the one through u.  The vertices of a shortest
  // up-down path are never stalled at their exact distance (no real path is
  // shorter), so they still expand and the result stays exact; x is checked
  // again whenever its distance drops.  The arcs checked are x's arcs of the
  // other direction, read by the whole wave as in an expansion; a lane that
  // finds a stall sets its entry's bit in the wave's mask.  Called by every
  // lane of a wave (wave-uniform loop bounds).
  // rows and arcs read (expansions and stall checks; stats batches)
  uint32_t nrows = 0, narcs = 0;
  __shared__ unsigned long long s_stall[NW];
  auto stall_check = [&](bool cand, uint32_t vx, uint32_t dx, uint32_t dr) -> bool {
    uint32_t ss = 0, sl = 0;
    if (cand) {
      const uint32_t *o = dr ? upoff : dnoff;
      ss = o[vx];
      sl = o[vx + 1] - ss;
      nrows++;
      narcs += sl;
    }
    const uint32_t incl = gscan_incl<kWave>(sl);
    const uint32_t T = __shfl(incl, kWave - 1, kWave);
    if (T == 0) return false;
    for (uint32_t i0 = 0; i0 < T; i0 += kWave * kQUnroll) {
      uint2 a[kQUnroll];
      uint32_t sd[kQUnroll], sdr[kQUnroll], src[kQUnroll];
#pragma unroll
      for (int u = 0; u < kQUnroll; u++) {
        const uint32_t idx = i0 + u * kWave + l;
        a[u] = make_uint2(SP_EMPTY32, 0u);
        sd[u] = 0;
        sdr[u] = 0;
        src[u] = 0;
        if (i0 + u * kWave < T) {  // uniform across the wave
          const int sl2 = gfind<kWave>(incl, idx);
          const uint32_t sss = __shfl(ss, sl2, kWave), sinc = __shfl(incl, sl2, kWave);
          const uint32_t ssl = __shfl(sl, sl2, kWave);
          sd[u] = __shfl(dx, sl2, kWave);
          sdr[u] = __shfl(dr, sl2, kWave);
          src[u] = (uint32_t)sl2;
          if (idx < T) a[u] = (sdr[u] ? uparc : dnarc)[sss + (idx - (sinc - ssl))];
        }
      }
#pragma unroll
      for (int u = 0; u < kQUnroll; u++) {
        if (a[u].x == SP_EMPTY32 || a[u].y >= sd[u]) continue;
        uint32_t du = SP_INF32;
        if (TOP && a[u].x >= tbase) {
          du = qld<GM>(&S.dist[sdr[u]][a[u].x - tbase]);
        } else {
          const int h = qfind<GM>(S, sdr[u], a[u].x);
          if (h >= 0) du = qld<GM>(&S.dist[sdr[u]][TOP + h]);
        }
        if (du != SP_INF32 && (unsigned long long)du + a[u].y < sd[u])
          atomicOr(&s_stall[wv], 1ull << src[u]);
      }
    }
    wave_sync();
    const bool st = (s_stall[wv] >> l) & 1ull;
    wave_sync();
    if (l == 0) s_stall[wv] = 0ull;
    wave_sync();
    return st;
  };
  if (tid < NW) s_stall[tid] = 0ull;
  qclear<GM>(S, tid, NT);
  qsync<NW, GM>();
  for (;;) {
    // every thread has read the previous index (it passed a barrier since)
    if (tid == 0) {
      const unsigned long long w = atomicAdd(work, 1ull);
      qst<GM>(&S.next[0], (uint32_t)w);
      qst<GM>(&S.next[1], (uint32_t)(w >> 32));
    }
    qsync<NW, GM>();
    const uint64_t qi = (uint64_t)qld<GM>(&S.next[0]) | ((uint64_t)qld<GM>(&S.next[1]) << 32);
    if (qi >= nq) break;
    const uint64_t k = list ? (uint64_t)list[qi] : qi;
    if (qs[k] >= n || qt[k] >= n) {  // the same k in every thread
      if (tid == 0) {
        atomicOr(bad, 1u);
        dist[k] = SP_INF64;
      }
      qsync<NW, GM>();
      continue;
    }
    if (tid < 2) {
      const uint32_t v = rank[tid ? qt[k] : qs[k]];
      uint32_t fresh = 0;
      const int a = slot_of(tid, v, &fresh);  // an empty table has room
      qst<GM>(&S.dist[tid][a], 0u);
      qst<GM>(&S.bits[tid][a >> 5], 1u << (a & 31));
      if (TOP && (uint32_t)a < TOP) qst<GM>(&S.usedt[tid], 1u);
      else qst<GM>(&S.used[tid], 1u);
      if (tid == 0) qst64<GM>(&S.mu, qs[k] == qt[k] ? 0ull : SP_INF64);
    }
    qsync<NW, GM>();
    for (;;) {
      // flagged slots of both directions (words tid, tid + NT, ...): their
      // count and, with a window, the lowest flagged rank of each direction
      uint32_t c = 0, mk0 = SP_EMPTY32, mk1 = SP_EMPTY32;
      for (uint32_t wi = tid; wi < kW2; wi += NT) {
        const uint32_t d = wi / L::kWords, wd = wi % L::kWords;
        uint32_t x = qld<GM>(&S.bits[d][wd]);
        c += __popc(x);
        if (wend) {
          while (x) {
            const uint32_t b = __builtin_ctz(x);
            x &= x - 1;
            const uint32_t r = rank_of(d, wd * 32 + b);
            if (d) mk1 = min(mk1, r);
            else mk0 = min(mk0, r);
          }
        }
      }
      uint32_t F, M0 = SP_EMPTY32, M1 = SP_EMPTY32;
      uint32_t p = wend ? qscan_min<NW, GM>(S, c, mk0, mk1, &F, &M0, &M1)
                        : qscan<NW, GM>(S, c, &F, S.wsum);
      if (F == 0) break;
      // ranks >= T[d] stay flagged for a later step (the minima are the same
      // in every lane, so these are scalar loads)
      uint32_t T0 = SP_EMPTY32, T1 = SP_EMPTY32;
      if (wend) {
        M0 = __builtin_amdgcn_readfirstlane(M0);
        M1 = __builtin_amdgcn_readfirstlane(M1);
        if (M0 != SP_EMPTY32) T0 = wend[M0];
        if (M1 != SP_EMPTY32) T1 = wend[M1];
      }
      // the flagged slots go to the list (in word order) and leave the
      // bitmap; when there are more than LIST, only slots inside the window
      // are taken (counted and placed by a second scan), so a step always
      // expands the lowest flagged rank of each direction, and the first
      // LIST of them are taken, the rest stay flagged
      const bool part = F > L::kList;
      if (part) {
        uint32_t c2 = 0;
        for (uint32_t wi = tid; wi < kW2; wi += NT) {
          const uint32_t d = wi / L::kWords, wd = wi % L::kWords;
          uint32_t x = qld<GM>(&S.bits[d][wd]);
          const uint32_t Td = d ? T1 : T0;
          while (x) {
            const uint32_t b = __builtin_ctz(x);
            x &= x - 1;
            c2 += rank_of(d, wd * 32 + b) < Td;
          }
        }
        p = qscan<NW, GM>(S, c2, &F, S.wsum2);
      }
      for (uint32_t wi = tid; wi < kW2; wi += NT) {
        const uint32_t d = wi / L::kWords, wd = wi % L::kWords;
        uint32_t x = qld<GM>(&S.bits[d][wd]);
        if (!x) continue;
        const uint32_t Td = d ? T1 : T0;
        uint32_t keep = 0;
        while (x) {
          const uint32_t b = __builtin_ctz(x);
          x &= x - 1;
          if (part && rank_of(d, wd * 32 + b) >= Td) {
            keep |= 1u << b;
            continue;
          }
          if (p < L::kList) qste<GM>(&S.list[p], (E)(d * NS + wd * 32 + b));
          else keep |= 1u << b;
          p++;
        }
        qst<GM>(&S.bits[d][wd], keep);
      }
      if (F > L::kList) F = L::kList;
      qsync<NW, GM>();
      uint32_t fresh0 = 0, fresh1 = 0, ft0 = 0, ft1 = 0;
      // entries dealt to the waves in turn, so a small step still uses all
      for (uint32_t cb = 0; cb < F; cb += NT) {
        const uint32_t i = cb + (uint32_t)l * NW + wv;
        uint32_t rs = 0, rl = 0, dx = 0, dr = 0, vx = 0;
        bool cand = false;
        if (i < F) {
          const uint32_t e = qlde<GM>(&S.list[i]);
          dr = e / NS;
          const uint32_t slot = e - dr * NS;
          vx = rank_of(dr, slot);
          dx = qld<GM>(&S.dist[dr][slot]);
          if (vx >= (dr ? T1 : T0)) {
            atomicOr(&S.bits[dr][slot >> 5], 1u << (slot & 31));
          } else if (prune && dx >= qld64<GM>(&S.mu)) {
            // no path through x is shorter than one already met
          } else if (CORE && coreD && vx >= core0) {
            // a core vertex: its paths come from the core table at the end
          } else {
            cand = true;
          }
        }
        if (prune && stall_check(cand, vx, dx, dr)) cand = false;
        if (cand) {
          const uint32_t *o = dr ? dnoff : upoff;
          rs = o[vx];
          rl = o[vx + 1] - rs;
          nrows++;
          narcs += rl;
        }
        const uint32_t incl = gscan_incl<kWave>(rl);
        const uint32_t T = __shfl(incl, kWave - 1, kWave);
        for (uint32_t i0 = 0; i0 < T; i0 += kWave * kQUnroll) {
          const unsigned long long mub = prune ? qld64<GM>(&S.mu) : SP_INF64;
          uint2 a[kQUnroll];
          uint32_t sd[kQUnroll], sdr[kQUnroll];
#pragma unroll
          for (int u = 0; u < kQUnroll; u++) {
            const uint32_t idx = i0 + u * kWave + l;
            a[u] = make_uint2(SP_EMPTY32, 0u);
            sd[u] = 0;
            sdr[u] = 0;
            if (i0 + u * kWave < T) {  // uniform across the wave
              const int src = gfind<kWave>(incl, idx);
              const uint32_t srs = __shfl(rs, src, kWave), sinc = __shfl(incl, src, kWave);
              const uint32_t srl = __shfl(rl, src, kWave);
              sd[u] = __shfl(dx, src, kWave);
              sdr[u] = __shfl(dr, src, kWave);
              if (idx < T) a[u] = (sdr[u] ? dnarc : uparc)[srs + (idx - (sinc - srl))];
            }
          }
#pragma unroll
          for (int u = 0; u < kQUnroll; u++) {
            if (a[u].x == SP_EMPTY32) continue;
            const unsigned long long nd = (unsigned long long)sd[u] + a[u].y;
            if (nd >= mub) continue;  // pruned: not shorter than a path already met
            if (nd > 0xFFFFFFFEull) {
              atomicOr(&S.ovf, 1u);
              continue;
            }
            uint32_t fr = 0;
            const int y = slot_of(sdr[u], a[u].x, &fr);
            if (y < 0) {
              atomicOr(&S.ovf, 1u);
              continue;
            }
            if (sdr[u]) fresh1 += fr;
            else fresh0 += fr;
            const uint32_t old = atomicMin(&S.dist[sdr[u]][y], (uint32_t)nd);
            if ((uint32_t)nd < old) {
              atomicOr(&S.bits[sdr[u]][y >> 5], 1u << (y & 31));
              if (TOP && (uint32_t)y < TOP && old == SP_INF32) {  // first reach of a dense slot
                if (sdr[u]) ft1++;
                else ft0++;
              }
              if (prune) {  // met by the other direction: a path s -> y -> t
                const uint32_t od = sdr[u] ^ 1u;
                int yo = -1;  // y's slot in the other direction's table
                if (TOP && (uint32_t)y < TOP) {
                  yo = y;
                } else {
                  const int h = qfind<GM>(S, od, a[u].x);
                  if (h >= 0) yo = (int)TOP + h;
                }
                if (yo >= 0) {
                  const uint32_t dv2 = qld<GM>(&S.dist[od][yo]);
                  if (dv2 != SP_INF32) atomicMin(&S.mu, nd + dv2);
                }
              }
            }
          }
          // a full table fails every further insert only after probing all
          // of it: leave the step once an overflow is flagged (the query
          // goes to the next tier anyway)
          if (__builtin_amdgcn_readfirstlane(qld<GM>(&S.ovf))) break;
        }
        if (__builtin_amdgcn_readfirstlane(qld<GM>(&S.ovf))) break;
      }
      fresh0 = gsum<kWave>(fresh0);
      fresh1 = gsum<kWave>(fresh1);
      if (TOP) {
        ft0 = gsum<kWave>(ft0);
        ft1 = gsum<kWave>(ft1);
      }
      if (l == 0) {
        const uint32_t u0 = atomicAdd(&S.used[0], fresh0) + fresh0;
        const uint32_t u1 = atomicAdd(&S.used[1], fresh1) + fresh1;
        if (u0 > L::kLimit || u1 > L::kLimit) atomicOr(&S.ovf, 1u);
        if (TOP) {
          atomicAdd(&S.usedt[0], ft0);
          atomicAdd(&S.usedt[1], ft1);
        }
      }
      qsync<NW, GM>();
      if (qld<GM>(&S.ovf)) break;
    }
    qsync<NW, GM>();
    const bool ok = qld<GM>(&S.ovf) == 0;
    if (ok) {
      unsigned long long best = SP_INF64;
      for (uint32_t i = tid; i < TOP; i += NT) {  // dense part: the same slot
        const uint32_t a = qld<GM>(&S.dist[0][i]), b = qld<GM>(&S.dist[1][i]);
        if (a != SP_INF32 && b != SP_INF32) {
          const unsigned long long c2 = (unsigned long long)a + b;
          best = c2 < best ? c2 : best;
        }
      }
      for (uint32_t i = tid; i < CAP; i += NT) {
        const uint32_t v = qld<GM>(&S.key[0][i]);
        if (v == SP_EMPTY32) continue;
        const int b = qfind<GM>(S, 1, v);
        if (b >= 0) {
          const unsigned long long c2 = (unsigned long long)qld<GM>(&S.dist[0][TOP + i]) +
                                        (unsigned long long)qld<GM>(&S.dist[1][TOP + b]);
          best = c2 < best ? c2 : best;
        }
      }
      if (prune) {  // a met path that the scan no longer sees is still a path
        const unsigned long long m = qld64<GM>(&S.mu);
        best = m < best ? m : best;
      }
      if constexpr (CORE > 0) {
        if (coreD) {
          // core entries of each direction (dense slots from cb on), listed
          // by a block scan in the hashed keys' space (read for the last
          // time above), then every pair through the core table
          static_assert(2 * CORE * sizeof(uint16_t) <= sizeof(S.key), "core lists fit the keys");
          qsync<NW, GM>();
          uint16_t(*s_core)[CORE] = reinterpret_cast<uint16_t(*)[CORE]>(&S.key[0][0]);
          const uint32_t cb = core0 - tbase;
          uint32_t cnt[2];
#pragma unroll
          for (int d = 0; d < 2; d++) {
            uint32_t c = 0;
            for (uint32_t i = tid; i < coreK; i += NT) c += qld<GM>(&S.dist[d][cb + i]) != SP_INF32;
            uint32_t p = qscan<NW, GM>(S, c, &cnt[d], d ? S.wsum2 : S.wsum);
            for (uint32_t i = tid; i < coreK; i += NT)
              if (qld<GM>(&S.dist[d][cb + i]) != SP_INF32) s_core[d][p++] = (uint16_t)i;
          }
          qsync<NW, GM>();
          const uint32_t n1 = cnt[1];
          const uint64_t np = (uint64_t)cnt[0] * n1;
          for (uint64_t pp = tid; pp < np; pp += NT) {
            const uint32_t i = s_core[0][pp / n1], j = s_core[1][pp % n1];
            const uint32_t w = coreD[(size_t)i * coreN + j];
            narcs++;  // one table read (stats batches)
            if (w == SP_INF32) continue;
            const unsigned long long c2 = (unsigned long long)qld<GM>(&S.dist[0][cb + i]) + w +
                                          qld<GM>(&S.dist[1][cb + j]);
            best = c2 < best ? c2 : best;
          }
        }
      }
      best = gmin64<kWave>(best);
      if constexpr (NW > 1) {
        if (l == 0) {
          qst<GM>(reinterpret_cast<uint32_t *>(&S.wmin[wv]), (uint32_t)best);
          qst<GM>(reinterpret_cast<uint32_t *>(&S.wmin[wv]) + 1, (uint32_t)(best >> 32));
        }
        qsync<NW, GM>();
        for (int i = 0; i < NW; i++) {
          const uint32_t *wp = reinterpret_cast<const uint32_t *>(&S.wmin[i]);
          const unsigned long long x =
              (unsigned long long)qld<GM>(wp) | ((unsigned long long)qld<GM>(wp + 1) << 32);
          best = x < best ? x : best;
        }
      }
      if (tid == 0) {
        dist[k] = best;
        if (visited)
          visited[k] = qld<GM>(&S.used[0]) + qld<GM>(&S.used[1]) + qld<GM>(&S.usedt[0]) +
                       qld<GM>(&S.usedt[1]);
      }
    } else if (tid == 0) {
      const uint32_t p2 = atomicAdd(ovf_count, 1u);
      ovf_list[p2] = (uint32_t)k;
    }
    qsync<NW, GM>();
    qclear<GM>(S, tid, NT);
    qsync<NW, GM>();
  }
  if (qcount) {
    const uint64_t r = gsum64<kWave>(nrows), a = gsum64<kWave>(narcs);
    if (l == 0) {
      atomicAdd(&qcount[0], (unsigned long long)r);
      atomicAdd(&qcount[1], (unsigned long long)a);
    }
  }
}

// Queries whose closures outgrow LDS or 32-bit distances: tables of cap
// slots in global memory with 64-bit distances.  With limit < cap a query
// whose table passes limit entries goes to ovf_list; with cap >= 2n slots
// and limit = cap no query overflows.
__global__ void __launch_bounds__(64) k_query_global(
    uint32_t nlist, const uint32_t *__restrict__ list, const uint32_t *__restrict__ qs,
    const uint32_t *__restrict__ qt, const uint32_t *__restrict__ rank,
    const uint32_t *__restrict__ upoff, const uint2 *__restrict__ uparc,
    const uint32_t *__restrict__ dnoff, const uint2 *__restrict__ dnarc,
    unsigned long long *__restrict__ dist, uint32_t *__restrict__ visited,
    uint32_t *__restrict__ tabs, uint32_t cap, uint32_t limit, uint32_t *__restrict__ ovf_list,
    uint32_t *__restrict__ ovf_count, unsigned long long *__restrict__ qcount) {
  // per direction: key[cap], dist[cap] (2 words each), flag[cap], order, fr0,
  // fr1 [cap] and 4 counters = 8 cap + 4 words
  const size_t per = (size_t)cap * 8 + 4;
  uint32_t *base = tabs + (size_t)blockIdx.x * 2 * per;
  QTab<uint32_t, unsigned long long, true> T[2];
  for (int d = 0; d < 2; d++) {
    uint32_t *b = base + d * per;
    T[d].key = b;
    T[d].dist = reinterpret_cast<unsigned long long *>(b + cap);
    T[d].flag = b + 3 * (size_t)cap;
    T[d].order = b + 4 * (size_t)cap;
    T[d].fr0 = b + 5 * (size_t)cap;
    T[d].fr1 = b + 6 * (size_t)cap;
    T[d].ctr = b + 8 * (size_t)cap;
    T[d].cap = cap;
    T[d].shift = 32 - __builtin_ctz(cap);
    T[d].limit = limit;
  }
  uint32_t nrows = 0, narcs = 0;  // expansions and relaxations (stats batches)
  for (uint32_t i = blockIdx.x; i < nlist; i += gridDim.x) {
    const uint32_t k = list[i];
    const uint32_t rs = rank[qs[k]], rt = rank[qt[k]];
    bool ok = closure(T[0], upoff, uparc, rs, nrows, narcs);
    if (ok) ok = closure(T[1], dnoff, dnarc, rt, nrows, narcs);
    if (ok) {
      const unsigned long long mu = meet(T[0], T[1]);
      if (lane_id() == 0) {
        dist[k] = mu;
        if (visited) visited[k] = T[0].ld(&T[0].ctr[0]) + T[1].ld(&T[1].ctr[0]);
      }
    } else if (lane_id() == 0) {
      const uint32_t p = atomicAdd(ovf_count, 1u);
      ovf_list[p] = k;
    }
    qtab_reset(T[0]);
    qtab_reset(T[1]);
  }
  if (qcount) {
    const uint64_t r = gsum64<kWave>(nrows), a = gsum64<kWave>(narcs);
    if (lane_id() == 0) {
      atomicAdd(&qcount[0], (unsigned long long)r);
      atomicAdd(&qcount[1], (unsigned long long)a);
    }
  }
}

// Words of the per-batch query counters (see query_tiers).
constexpr uint32_t kQCtrWords = 32;

// The tiers of one batch on device arrays (ds, dt, dd, dv).  Scratch comes
// from `sc`: sc.ctr (16 words), sc.ovf1 / sc.ovf2 (q entries each),
// sc.tier3(n3, &tabs, &blocks) and sc.tier4(n4, &tabs, &cap, &limit, &ntab)
// (tables for the global-memory tiers, requested only when a query needs
// them); tier4 sets *limit < *cap when its tables can fill, and a query
// that still overflows then makes the call fail with CH_E_LIMIT.
// Core matrix entries from the CH arcs of the core rows c0 .. n-1 (row
// index = rank - c0): upward arcs of a row go to higher ranks, downward arcs
// of a row come from higher ranks, so every such arc joins two core
// vertices.  *maxw = the largest weight seen.
__global__ void k_core_arcs(uint32_t c0, uint32_t n, uint32_t N, const uint32_t *__restrict__ upoff,
                            const uint2 *__restrict__ uparc, const uint32_t *__restrict__ dnoff,
                            const uint2 *__restrict__ dnarc, uint32_t *__restrict__ D,
                            uint32_t *__restrict__ maxw) {
  const uint32_t stride = gridDim.x * blockDim.x;
  uint32_t mx = 0;
  for (uint32_t r = c0 + blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
    const uint32_t i = r - c0;
    for (uint32_t e = upoff[r]; e < upoff[r + 1]; e++) {
      const uint2 a = uparc[e];
      if (a.x < c0 || a.x >= n) continue;
      atomicMin(&D[(size_t)i * N + (a.x - c0)], a.y);
      mx = max(mx, a.y);
    }
    for (uint32_t e = dnoff[r]; e < dnoff[r + 1]; e++) {
      const uint2 a = dnarc[e];
      if (a.x < c0 || a.x >= n) continue;
      atomicMin(&D[(size_t)(a.x - c0) * N + i], a.y);
      mx = max(mx, a.y);
    }
  }
  if (mx) atomicMax(maxw, mx);
}

// A core table of a CH (once per CH and tier, at the tier's first pruned
// batch of at least kQCoreBatch queries): the kmax highest ranks (all of
// them on smaller CHs), their arcs, then the all-pairs closure.  Not used
// when a core distance could pass 32 bits (largest core arc weight x core
// size above 0xFFFFFFFE).
static int core_table(ch_s *ch, uint32_t kmax, DBuf &tab, uint32_t &k_out, uint32_t &n_out,
                      int &state, hipStream_t st) {
  if (state) return CH_OK;
  state = 2;
  const uint32_t n = ch->n;
  const uint32_t K = std::min<uint32_t>(kmax, n);
  if (K == 0) return CH_OK;
  const uint32_t N = (K + 63) / 64 * 64, c0 = n - K;
  HIP_TRY(tab.ensure((size_t)N * N * 4));
  HIP_TRY(ch->q_core_max.ensure(4));
  uint32_t *D = tab.as<uint32_t>(), *mx = ch->q_core_max.as<uint32_t>();
  HIP_TRY(fw_init(D, N, st));
  HIP_TRY(fill_u32(mx, 0u, 1, st));
  k_core_arcs<<<(K + 255) / 256, 256, 0, st>>>(c0, n, N, ch->q_upoff.as<uint32_t>(),
                                               ch->q_uparc.as<uint2>(), ch->q_dnoff.as<uint32_t>(),
                                               ch->q_dnarc.as<uint2>(), D, mx);
  HIP_TRY(hipGetLastError());
  uint32_t hmx = 0;
  HIP_TRY(hipMemcpyAsync(&hmx, mx, 4, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if ((uint64_t)hmx * K > 0xFFFFFFFEull) return CH_OK;
  HIP_TRY(fw_close(D, N, st));
  k_out = K;
  n_out = N;
  state = 1;
  return CH_OK;
}

template <typename Scratch>
static int query_tiers(ch_s *ch, const uint32_t *ds, const uint32_t *dt, uint64_t q,
                       unsigned long long *dd, uint32_t *dv, uint32_t flags, hipStream_t st,
                       Scratch &sc) {
  // Tiers: 1 = a slot per rank for the 2048 highest ranks plus 512-slot
  // tables per direction for the others (five blocks per CU),
  // 2 = a slot per rank for the 8192 highest ranks plus 4096-slot tables per
  // direction for the others (one block of 16 waves per CU), 3 = 16384-slot
  // tables in global memory, 4 = tables of at least 2n slots with 64-bit
  // distances (never overflow).  Each tier takes the previous one's overflow
  // list; the first tier is the one where most queries of the previous batch
  // ended.
  // counters: [0] tier-1 overflows, [1] bad ids, [2] tier-2 overflows,
  // [4] tier-3 overflows, [6] tier-4 overflows, 64-bit work counters of
  // tiers 1-3 at [8], [10], [12]
  uint32_t *ctr = sc.ctr;
  // cleared by a fill kernel, not a memset (the scratch may be in use by a
  // captured sequence of this stream); words 16-19: two 64-bit counters of
  // expanded vertices and relaxed arcs (stats batches)
  HIP_TRY(fill_u32(ctr, 0u, kQCtrWords, st));
  // a stats batch (visited counts) expands both upward search spaces
  // completely, so its counts do not depend on timing; other batches skip
  // what cannot be shorter than a path already met
  const uint32_t prune = (dv || (flags & CH_Q_FULL_CLOSURE)) ? 0u : 1u;
  unsigned long long *qcount = (dv || (flags & CH_Q_COUNT))
                                   ? reinterpret_cast<unsigned long long *>(ctr + 16)
                                   : nullptr;
  ch_query_stats_t qsn{};
  qsn.queries = q;
  const uint32_t forced = (flags >> 22) & 3u;  // CH_Q_FIRST_TIER; 0 = adaptive
  qsn.first_tier = forced ? forced : (uint32_t)ch->q_first_tier;
  qsn.counted = qcount ? 1u : 0u;
  // tier timing: events 2t and 2t+1 around tier t (ch_query_batch only)
  // the events come from a pool per host thread and device, made once and
  // kept to the end of the process (creating and destroying eight events
  // per CH cost about 2 ms per CH in a 512-graph batch)
  hipEvent_t *ev = nullptr;
  if (sc.timed) {
    static thread_local std::map<int, std::array<hipEvent_t, 8>> pool;
    auto &a = pool[ch->device];
    if (!a[0])
      for (int i = 0; i < 8; i++) HIP_TRY(hipEventCreate(&a[i]));
    ev = a.data();
  }
  auto mark = [&](int i) -> hipError_t { return ev ? hipEventRecord(ev[i], st) : hipSuccess; };
  int cus = 256;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ch->device);
  const uint32_t *rank = ch->rank.as<uint32_t>();
  const uint32_t *upoff = ch->q_upoff.as<uint32_t>(), *dnoff = ch->q_dnoff.as<uint32_t>();
  const uint2 *uparc = ch->q_uparc.as<uint2>(), *dnarc = ch->q_dnarc.as<uint2>();
  uint32_t *ovf1 = sc.ovf1, *ovf2 = sc.ovf2;
  const int first = forced ? (int)forced : ch->q_first_tier;
  const uint32_t wf = (flags >> 12) & 0xFFu;  // 0: default window, 255: none
  uint32_t win = (wf == 0 || wf == 255) ? 0u : wf;
  if (win >= ch->rounds) win = 0;  // a window over every level: the plain path
  if (win && win != ch->q_wend_win) {
    // q_wend is allocated with the query index
    if (ch->q_wend.cap < (size_t)std::max<uint32_t>(ch->n, 1) * 4)
      return set_error(CH_E_DEVICE, "query window array missing (internal error)");
    if (ch->n)
      k_window_ends<<<gridn(ch->n), 256, 0, st>>>(ch->n, rank, ch->level.as<uint32_t>(),
                                                  ch->q_lstart.as<uint32_t>(), ch->q_nlev, win,
                                                  ch->q_wend.as<uint32_t>());
    HIP_TRY(hipGetLastError());
    ch->q_wend_win = win;
  }
  const uint32_t *wend = win ? ch->q_wend.as<uint32_t>() : nullptr;
  if (first <= 1) {
    qsn.tier_queries[0] = q;
    HIP_TRY(mark(0));
    const uint64_t g = std::min<uint64_t>(q, (uint64_t)cus * kQTier1PerCU);
    const uint32_t nw = (flags >> 8) & 0xFu;  // 0: four waves per query
    // the first tier's core table (the kQCore1 highest ranks, within its
    // rank slots), made like the second tier's
    const bool use_core1 = prune && !(flags & CH_Q_NO_CORE);
    if (use_core1 && ch->q_core1_state == 0 && sc.can_alloc && q >= kQCoreBatch)
      TRY(core_table(ch, kQCore1, ch->q_core1, ch->q_core1_k, ch->q_core1_n, ch->q_core1_state,
                     st));
    const bool core1 = use_core1 && ch->q_core1_state == 1;
    const uint32_t *c1D = core1 ? ch->q_core1.as<uint32_t>() : nullptr;
    const uint32_t c1lo = core1 ? ch->n - ch->q_core1_k : 0xFFFFFFFFu;
#define SP_QUERY_LAUNCH(NW)                                                                    \
  k_query<NW, QTier1, false, kQCore1><<<(unsigned)g, 64 * NW, 0, st>>>(                         \
      q, ch->n, nullptr, nullptr, ctr + 1, ds, dt, rank, upoff, uparc, dnoff, dnarc, dd, dv,   \
      ovf1, ctr, wend, reinterpret_cast<unsigned long long *>(ctr + 8), nullptr, qcount, prune, \
      c1D, c1lo, ch->q_core1_n, ch->q_core1_k)
    if (nw == 1) SP_QUERY_LAUNCH(1);
    else if (nw == 2) SP_QUERY_LAUNCH(2);
    else if (nw == 8) SP_QUERY_LAUNCH(8);
    else SP_QUERY_LAUNCH(4);
#undef SP_QUERY_LAUNCH
    HIP_TRY(hipGetLastError());
    HIP_TRY(mark(1));
  }
  if (first <= 2) {
    HIP_TRY(mark(2));
    // the core table: pruned batches only (full closures expand everything),
    // made on the first such batch with at least kQCoreBatch queries in this
    // tier when the scratch may allocate (its closure, about 7 ms at 4096
    // ranks, is amortised over the batch and the CH's later ones).  After
    // the first tier only its overflows come here: their count is read first
    const bool use_core = prune && !(flags & CH_Q_NO_CORE);
    if (use_core && ch->q_core_state == 0 && sc.can_alloc && q >= kQCoreBatch) {
      uint32_t in2 = 0xFFFFFFFFu;
      if (first <= 1) {
        HIP_TRY(hipMemcpyAsync(&in2, ctr, 4, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
      }
      if (in2 >= kQCoreBatch)
        TRY(core_table(ch, kQCore, ch->q_core, ch->q_core_k, ch->q_core_n, ch->q_core_state,
                       st));
    }
    const bool core = use_core && ch->q_core_state == 1;
    k_query<16, QTier2, false, kQCore><<<(unsigned)std::min<uint64_t>(q, cus), 1024, 0, st>>>(
        q, ch->n, first <= 1 ? ovf1 : nullptr, ctr, ctr + 1, ds, dt, rank, upoff, uparc, dnoff,
        dnarc, dd, dv, ovf2, ctr + 2, wend, reinterpret_cast<unsigned long long *>(ctr + 10),
        nullptr, qcount, prune, core ? ch->q_core.as<uint32_t>() : nullptr,
        core ? ch->n - ch->q_core_k : 0xFFFFFFFFu, ch->q_core_n, ch->q_core_k);
    HIP_TRY(hipGetLastError());
    HIP_TRY(mark(3));
  }
  uint32_t hc[4] = {0, 0, 0, 0};
  HIP_TRY(hipMemcpyAsync(hc, ctr, 16, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (hc[1]) return set_error(CH_E_INVALID, "a query vertex id is >= n");
  const uint64_t into2 = first <= 1 ? hc[0] : q;
  if (first <= 2) qsn.tier_queries[1] = into2;
  uint64_t n3 = first <= 2 ? hc[2] : q;
  uint32_t *list3 = first <= 2 ? ovf2 : nullptr;
  uint32_t n4 = 0;
  if (n3) {
    QTier3 *tabs = nullptr;
    uint64_t nb = std::min<uint64_t>(n3, (uint64_t)cus * 4);
    TRY(sc.tier3(n3, &tabs, &nb));
    // overflows into ctr[4]; the input count is tier 2's, on the device
    qsn.tier_queries[2] = n3;
    HIP_TRY(mark(4));
    k_query<8, QTier3, true><<<(unsigned)nb, 512, 0, st>>>(
        q, ch->n, list3, ctr + 2, ctr + 1, ds, dt, rank, upoff, uparc, dnoff, dnarc, dd, dv,
        ovf1, ctr + 4, wend, reinterpret_cast<unsigned long long *>(ctr + 12), tabs, qcount,
        prune);
    HIP_TRY(hipGetLastError());
    HIP_TRY(mark(5));
    uint32_t h2[4] = {0, 0, 0, 0};  // ctr[1..4]
    HIP_TRY(hipMemcpyAsync(h2, ctr + 1, 16, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (h2[0]) return set_error(CH_E_INVALID, "a query vertex id is >= n");
    n4 = h2[3];
  }
  if (n4) {
    uint32_t *tabs = nullptr, cap = 0, limit = 0;
    size_t ntab = 0;
    TRY(sc.tier4(n4, cus, &tabs, &cap, &limit, &ntab));
    // keys and dists all ones; flag, order, fronts, counters zero
    for (size_t k = 0; k < 2 * ntab; k++) {
      uint32_t *b = tabs + k * ((size_t)cap * 8 + 4);
      HIP_TRY(fill_u32(b, SP_EMPTY32, 3ull * cap, st));
      HIP_TRY(fill_u32(b + 3ull * cap, 0u, (size_t)cap * 5 + 4, st));
    }
    qsn.tier_queries[3] = n4;
    HIP_TRY(mark(6));
    k_query_global<<<(unsigned)ntab, 64, 0, st>>>(n4, ovf1, ds, dt, rank, upoff, uparc, dnoff,
                                                 dnarc, dd, dv, tabs, cap, limit, ovf2, ctr + 6,
                                                 qcount);
    HIP_TRY(hipGetLastError());
    HIP_TRY(mark(7));
    if (limit < cap) {
      uint32_t n5 = 0;
      HIP_TRY(hipMemcpyAsync(&n5, ctr + 6, 4, hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      if (n5)
        return set_error(CH_E_LIMIT, "a query's upward search space outgrew the largest table "
                                     "of ch_query_batch_noalloc; use ch_query_batch");
    }
  }
  // where the next batch starts (adaptive batches only)
  if (!forced && first <= 1 && hc[0] * 2 > q) ch->q_first_tier = 2;
  if (!forced && first <= 2 && into2 && (uint64_t)hc[2] * 2 > into2) ch->q_first_tier = 3;
  // counters and tier times of this batch (one more wait, for the copies)
  if (qcount || ev) {
    unsigned long long qc[2] = {0, 0};
    if (qcount) HIP_TRY(hipMemcpyAsync(qc, qcount, 16, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    qsn.rows = qc[0];
    qsn.arcs = qc[1];
    for (int t = 0; ev && t < 4; t++)
      if (qsn.tier_queries[t]) HIP_TRY(hipEventElapsedTime(&qsn.tier_ms[t], ev[2 * t], ev[2 * t + 1]));
  }
  ch->qstats = qsn;
  return CH_OK;
}

// Scratch of ch_query_batch: buffers of the CH, grown on demand.
struct QScratchCH {
  ch_s *ch;
  uint32_t *ctr = nullptr, *ovf1 = nullptr, *ovf2 = nullptr;
  bool timed = true;
  bool can_alloc = true;  // may build the CH's core table
  int tier3(uint64_t, QTier3 **tabs, uint64_t *nb) {
    HIP_TRY(ch->q_tab.ensure(*nb * sizeof(QTier3)));
    *tabs = reinterpret_cast<QTier3 *>(ch->q_tab.p);
    return CH_OK;
  }
  int tier4(uint32_t n4, int cus, uint32_t **tabs, uint32_t *cap, uint32_t *limit,
            size_t *ntab) {
    uint64_t c = 1;
    while (c < 2ull * ch->n + 2) c <<= 1;
    *cap = *limit = (uint32_t)std::min<uint64_t>(c, 1ull << 31);
    const size_t per = ((size_t)*cap * 8 + 4) * 4 * 2;
    *ntab = std::max<size_t>(
        1, std::min<size_t>({(size_t)n4, (size_t)cus * 2, (size_t)(4ull << 30) / per}));
    HIP_TRY(ch->q_gtab.ensure(*ntab * per));
    *tabs = ch->q_gtab.as<uint32_t>();
    return CH_OK;
  }
};

int query_batch(const ch_s *chc, const uint32_t *s, const uint32_t *t, uint64_t q, uint64_t *dist,
                uint32_t *visited, uint32_t flags, hipStream_t st) {
  ch_s *ch = const_cast<ch_s *>(chc);
  if (!ch->has_index) return set_error(CH_E_INVALID, "the CH was built without a query index");
  if (q == 0) return CH_OK;
  if (!st) st = ch->stream;
  const bool on_dev = flags & CH_Q_ON_DEVICE;
  const uint32_t *ds = s, *dt = t;
  unsigned long long *dd = reinterpret_cast<unsigned long long *>(dist);
  HIP_TRY(ch->q_ctr.ensure(kQCtrWords * 4));
  if (!on_dev) {
    HIP_TRY(ch->q_s.ensure(q * 4));
    HIP_TRY(ch->q_t.ensure(q * 4));
    HIP_TRY(ch->q_d.ensure(q * 8));
    HIP_TRY(hipMemcpyAsync(ch->q_s.p, s, q * 4, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(ch->q_t.p, t, q * 4, hipMemcpyHostToDevice, st));
    ds = ch->q_s.as<uint32_t>();
    dt = ch->q_t.as<uint32_t>();
    dd = ch->q_d.as<unsigned long long>();
  }
  uint32_t *dv = visited;
  if (visited && !on_dev) {
    HIP_TRY(ch->q_v.ensure(q * 4));
    dv = ch->q_v.as<uint32_t>();
  }
  HIP_TRY(ch->q_ovf.ensure(q * 4));
  HIP_TRY(ch->q_ovf2.ensure(q * 4));
  QScratchCH sc{ch, ch->q_ctr.as<uint32_t>(), ch->q_ovf.as<uint32_t>(), ch->q_ovf2.as<uint32_t>()};
  TRY(query_tiers(ch, ds, dt, q, dd, dv, flags, st, sc));
  if (!on_dev) HIP_TRY(hipMemcpyAsync(dist, dd, q * 8, hipMemcpyDeviceToHost, st));
  if (visited && !on_dev) HIP_TRY(hipMemcpyAsync(visited, dv, q * 4, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return CH_OK;
}

// ---------------------------------------------------------------------------
// Query batch without allocations (ch_query_batch_noalloc).  Every scratch
// array of the tiers lives in `scratch`, one fixed array per GPU: counters,
// two overflow lists of a pass of kNaChunk queries, kNaT3Blocks tier-3
// tables and one tier-4 table set of kNaT4Cap slots per direction.  Host
// code never uses the array's name as an address: the device address comes
// from hipGetSymbolAddress, once per device.
// ---------------------------------------------------------------------------
constexpr uint64_t kNaChunk = 1ull << 20;  // queries per pass
constexpr uint32_t kNaT3Blocks = 64;
constexpr uint32_t kNaT4Cap = 1u << 20;   // never fills on a CH of <= 524,287 vertices
constexpr size_t na_align(size_t x) { return (x + 255) & ~(size_t)255; }
constexpr size_t kNaOvf1 = 256;
static_assert(kQCtrWords * 4 <= kNaOvf1, "query counters in the scratch array");
constexpr size_t kNaOvf2 = kNaOvf1 + kNaChunk * 4;
constexpr size_t kNaT3 = na_align(kNaOvf2 + kNaChunk * 4);
constexpr size_t kNaT4 = na_align(kNaT3 + (size_t)kNaT3Blocks * sizeof(QTier3));
constexpr size_t kNaEnd = kNaT4 + 2 * ((size_t)kNaT4Cap * 8 + 4) * 4;
static_assert(kNaEnd <= CH_NOALLOC_SCRATCH_BYTES, "no-allocation query scratch too small");
static_assert(alignof(QTier3) <= 256, "tier-3 tables in the scratch array");

static __device__ __align__(256) uint8_t scratch[CH_NOALLOC_SCRATCH_BYTES];

constexpr int kNaMaxDevices = 64;
static std::mutex g_na_mu;
static uint8_t *g_na_ptr[kNaMaxDevices] = {};

// Device address of `scratch` on `dev`, looked up on the first call for that
// device with it current.
static int na_scratch(int dev, uint8_t **out) {
  if (dev < 0 || dev >= kNaMaxDevices)
    return set_error(CH_E_DEVICE, "device index out of range for the query scratch");
  std::lock_guard<std::mutex> lock(g_na_mu);
  if (!g_na_ptr[dev]) {
    int cur = -1;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != dev) HIP_TRY(hipSetDevice(dev));
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess) return hip_error(e, "hipGetSymbolAddress(scratch)");
    if (!p) return set_error(CH_E_DEVICE, "no device address for the query scratch");
    g_na_ptr[dev] = static_cast<uint8_t *>(p);
  }
  *out = g_na_ptr[dev];
  return CH_OK;
}

struct QScratchFixed {
  uint8_t *base;
  uint32_t n;
  uint32_t *ctr, *ovf1, *ovf2;
  bool timed = false;  // creating events is left to ch_query_batch
  bool can_alloc = false;  // uses a core table only if one was built before
  int tier3(uint64_t, QTier3 **tabs, uint64_t *nb) {
    *nb = std::min<uint64_t>(*nb, kNaT3Blocks);
    *tabs = reinterpret_cast<QTier3 *>(base + kNaT3);
    return CH_OK;
  }
  int tier4(uint32_t, int, uint32_t **tabs, uint32_t *cap, uint32_t *limit, size_t *ntab) {
    *tabs = reinterpret_cast<uint32_t *>(base + kNaT4);
    *cap = kNaT4Cap;
    // a table of >= 2n + 2 slots never fills; else a query stops at 7/8
    *limit = 2ull * n + 2 <= kNaT4Cap ? kNaT4Cap : kNaT4Cap - kNaT4Cap / 8;
    *ntab = 1;
    return CH_OK;
  }
};

int query_batch_noalloc(const ch_s *chc, const uint32_t *s, const uint32_t *t, uint64_t q,
                        uint64_t *dist, uint32_t *visited, uint32_t flags, hipStream_t st) {
  ch_s *ch = const_cast<ch_s *>(chc);
  if (!ch->has_index) return set_error(CH_E_INVALID, "the CH was built without a query index");
  if (!(flags & CH_Q_ON_DEVICE))
    return set_error(CH_E_INVALID, "ch_query_batch_noalloc takes device arrays (CH_Q_ON_DEVICE)");
  if (q == 0) return CH_OK;
  if (!st) st = ch->stream;
  uint8_t *base = nullptr;
  TRY(na_scratch(ch->device, &base));
  QScratchFixed sc{base, ch->n, reinterpret_cast<uint32_t *>(base),
                   reinterpret_cast<uint32_t *>(base + kNaOvf1),
                   reinterpret_cast<uint32_t *>(base + kNaOvf2)};
  for (uint64_t c0 = 0; c0 < q; c0 += kNaChunk) {
    const uint64_t qc = std::min<uint64_t>(kNaChunk, q - c0);
    TRY(query_tiers(ch, s + c0, t + c0, qc, reinterpret_cast<unsigned long long *>(dist + c0),
                    visited ? visited + c0 : nullptr, flags, st, sc));
  }
  HIP_TRY(hipStreamSynchronize(st));
  return CH_OK;
}

}  // namespace sp
