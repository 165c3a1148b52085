// phast.hip -- one-to-all and many-to-many distances on a finished CH, by
// the two sweeps the paper describes for SSSP on a CH (Sec. "Query on
// Contraction Hierarchies": vertices grouped by level as in PHAST; a forward
// search on the upward edges, then a backward "decontraction" on the
// downward edges layer by layer).
//
// Every CH arc joins two different levels (the vertices contracted in one
// round form an independent set), so:
//   upward sweep:   levels bottom to top; every reached vertex of the level
//                   pushes d + w along its upward arcs (atomic minimum);
//                   each level's distances are final before it pushes;
//   downward sweep: levels top to bottom; every vertex pulls
//                   d(v) = min(d_up(v), min over downward arcs u -> v of
//                   d(u) + w) from the higher levels, already final.
// The result is the exact distance from the source to every vertex (the
// shortest path is an upward path to its highest vertex, then a downward
// one).  KC sources run together: distances are stored rank-major, KC per
// vertex, one lane per source.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "builder.hpp"
#include "common.hpp"

namespace sp {

#define HIP_TRY(expr)                                   \
  do {                                                  \
    hipError_t e_ = (expr);                             \
    if (e_ != hipSuccess) return hip_error(e_, #expr);  \
  } while (0)

constexpr unsigned long long kPhInf = ~0ull;

template <int KC>
__global__ void __launch_bounds__(256) k_phast_init(uint64_t words, unsigned long long *__restrict__ d) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride)
    d[i] = kPhInf;
}

// d[rank(s_i)][i] = 0 for the chunk's sources (ids already checked < n).
template <int KC>
__global__ void k_phast_sources(uint32_t kc, const uint32_t *__restrict__ s,
                                const uint32_t *__restrict__ rank,
                                unsigned long long *__restrict__ d) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kc) d[(size_t)rank[s[i]] * KC + i] = 0ull;
}

// One level of the upward sweep: ranks [r0, r1), KC lanes per vertex.
template <int KC>
__global__ void __launch_bounds__(256) k_phast_up(uint32_t r0, uint32_t r1,
                                                  const uint32_t *__restrict__ upoff,
                                                  const uint2 *__restrict__ uparc,
                                                  unsigned long long *__restrict__ d) {
  const uint32_t gl = threadIdx.x % KC;
  const uint32_t ng = gridDim.x * (blockDim.x / KC);
  for (uint32_t v = r0 + blockIdx.x * (blockDim.x / KC) + threadIdx.x / KC; v < r1; v += ng) {
    const unsigned long long x = d[(size_t)v * KC + gl];
    if (x == kPhInf) continue;
    const uint32_t e1 = upoff[v + 1];
    for (uint32_t e = upoff[v]; e < e1; e++) {
      const uint2 a = uparc[e];
      atomicMin(&d[(size_t)a.x * KC + gl], x + a.y);
    }
  }
}

// One level of the downward sweep: every vertex takes the minimum over its
// downward arcs from higher-ranked vertices (stored at the lower end).
template <int KC>
__global__ void __launch_bounds__(256) k_phast_down(uint32_t r0, uint32_t r1,
                                                    const uint32_t *__restrict__ dnoff,
                                                    const uint2 *__restrict__ dnarc,
                                                    unsigned long long *__restrict__ d) {
  const uint32_t gl = threadIdx.x % KC;
  const uint32_t ng = gridDim.x * (blockDim.x / KC);
  for (uint32_t v = r0 + blockIdx.x * (blockDim.x / KC) + threadIdx.x / KC; v < r1; v += ng) {
    unsigned long long best = d[(size_t)v * KC + gl];
    const uint32_t e1 = dnoff[v + 1];
    for (uint32_t e = dnoff[v]; e < e1; e++) {
      const uint2 a = dnarc[e];
      const unsigned long long y = d[(size_t)a.x * KC + gl];
      if (y != kPhInf && y + a.y < best) best = y + a.y;
    }
    d[(size_t)v * KC + gl] = best;
  }
}

// out[i * nt + j] = distance from the chunk's source i to target j (t[j], or
// vertex j when t is null), in original ids.
template <int KC>
__global__ void __launch_bounds__(256) k_phast_out(uint32_t kc, uint32_t nt,
                                                   const uint32_t *__restrict__ t,
                                                   const uint32_t *__restrict__ rank,
                                                   const unsigned long long *__restrict__ d,
                                                   unsigned long long *__restrict__ out) {
  const uint64_t total = (uint64_t)kc * nt;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += stride) {
    const uint32_t i = (uint32_t)(k / nt), j = (uint32_t)(k % nt);
    const uint32_t v = t ? t[j] : j;
    out[k] = d[(size_t)rank[v] * KC + i];
  }
}

// Id check: *bad |= 1 when some id >= n.
__global__ void k_phast_check(uint64_t cnt, const uint32_t *__restrict__ ids, uint32_t n,
                              uint32_t *__restrict__ bad) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += stride)
    if (ids[i] >= n) atomicOr(bad, 1u);
}

static unsigned ph_grid(uint64_t threads) {
  return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((threads + 255) / 256, 16384));
}

template <int KC>
static int phast_chunks(ch_s *ch, const uint32_t *ds, uint32_t ks, const uint32_t *dt,
                        uint32_t nt, unsigned long long *dd, const std::vector<uint32_t> &ls,
                        hipStream_t st) {
  const uint32_t n = ch->n;
  HIP_TRY(ch->q_phast.ensure((size_t)n * KC * 8));
  unsigned long long *d = ch->q_phast.as<unsigned long long>();
  const uint32_t *rank = ch->rank.as<uint32_t>();
  const uint32_t *upoff = ch->q_upoff.as<uint32_t>(), *dnoff = ch->q_dnoff.as<uint32_t>();
  const uint2 *uparc = ch->q_uparc.as<uint2>(), *dnarc = ch->q_dnarc.as<uint2>();
  const uint32_t nlev = (uint32_t)ls.size() - 1;
  for (uint32_t c0 = 0; c0 < ks; c0 += KC) {
    const uint32_t kc = std::min<uint32_t>(KC, ks - c0);
    k_phast_init<KC><<<ph_grid((uint64_t)n * KC), 256, 0, st>>>((uint64_t)n * KC, d);
    k_phast_sources<KC><<<1, 64, 0, st>>>(kc, ds + c0, rank, d);
    HIP_TRY(hipGetLastError());
    for (uint32_t L = 0; L < nlev; L++) {  // upward: bottom level first
      if (ls[L + 1] <= ls[L]) continue;
      k_phast_up<KC><<<ph_grid((uint64_t)(ls[L + 1] - ls[L]) * KC), 256, 0, st>>>(
          ls[L], ls[L + 1], upoff, uparc, d);
    }
    HIP_TRY(hipGetLastError());
    for (uint32_t L = nlev; L-- > 0;) {  // downward: top level first
      if (ls[L + 1] <= ls[L]) continue;
      k_phast_down<KC><<<ph_grid((uint64_t)(ls[L + 1] - ls[L]) * KC), 256, 0, st>>>(
          ls[L], ls[L + 1], dnoff, dnarc, d);
    }
    HIP_TRY(hipGetLastError());
    k_phast_out<KC><<<ph_grid((uint64_t)kc * nt), 256, 0, st>>>(kc, nt, dt, rank, d,
                                                                 dd + (size_t)c0 * nt);
    HIP_TRY(hipGetLastError());
  }
  return CH_OK;
}

int one_to_all(const ch_s *chc, const uint32_t *s, uint32_t ks, const uint32_t *t, uint32_t kt,
               uint64_t *dist, uint32_t flags, hipStream_t st) {
  ch_s *ch = const_cast<ch_s *>(chc);
  if (!ch->has_index) return set_error(CH_E_INVALID, "the CH was built without a query index");
  if (ks == 0) return CH_OK;
  if (!st) st = ch->stream;
  const uint32_t n = ch->n;
  const uint32_t nt = t ? kt : n;
  const bool on_dev = flags & CH_Q_ON_DEVICE;
  const uint64_t outn = (uint64_t)ks * nt;
  DBuf hs, ht, hd, bad;
  const uint32_t *ds = s, *dt = t;
  unsigned long long *dd = reinterpret_cast<unsigned long long *>(dist);
  if (!on_dev) {
    HIP_TRY(hs.ensure((size_t)ks * 4));
    HIP_TRY(hipMemcpyAsync(hs.p, s, (size_t)ks * 4, hipMemcpyHostToDevice, st));
    ds = hs.as<uint32_t>();
    if (t && kt) {
      HIP_TRY(ht.ensure((size_t)kt * 4));
      HIP_TRY(hipMemcpyAsync(ht.p, t, (size_t)kt * 4, hipMemcpyHostToDevice, st));
      dt = ht.as<uint32_t>();
    }
    HIP_TRY(hd.ensure(std::max<uint64_t>(outn, 1) * 8));
    dd = hd.as<unsigned long long>();
  }
  // ids < n, checked on the device before any sweep
  HIP_TRY(bad.ensure(4));
  HIP_TRY(fill_u32(bad.as<uint32_t>(), 0u, 1, st));
  k_phast_check<<<ph_grid(ks), 256, 0, st>>>(ks, ds, n, bad.as<uint32_t>());
  if (t && kt) k_phast_check<<<ph_grid(kt), 256, 0, st>>>(kt, dt, n, bad.as<uint32_t>());
  HIP_TRY(hipGetLastError());
  uint32_t hbad = 0;
  std::vector<uint32_t> ls(ch->q_nlev + 1);
  HIP_TRY(hipMemcpyAsync(&hbad, bad.p, 4, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(ls.data(), ch->q_lstart.p, ls.size() * 4, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (hbad) return set_error(CH_E_INVALID, "a source or target id is >= n");
  if (nt) {
    int rc;
    // sources per pass (lanes per vertex): enough for the batch, at most 64
    if (ks >= 16) rc = phast_chunks<64>(ch, ds, ks, dt, nt, dd, ls, st);
    else if (ks >= 4) rc = phast_chunks<16>(ch, ds, ks, dt, nt, dd, ls, st);
    else if (ks >= 2) rc = phast_chunks<4>(ch, ds, ks, dt, nt, dd, ls, st);
    else rc = phast_chunks<1>(ch, ds, ks, dt, nt, dd, ls, st);
    if (rc != CH_OK) return rc;
  }
  if (!on_dev && outn) HIP_TRY(hipMemcpyAsync(dist, dd, outn * 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return CH_OK;
}

}  // namespace sp
