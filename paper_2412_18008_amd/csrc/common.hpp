// common.hpp -- device helpers shared by the gfx950 kernels of the CH library.
//
// Wave size is 64.  Many kernels split a wave into "groups" of G lanes
// (G in {4, 8, 16, 32, 64}); each group works on one item (a vertex, a
// search source, a query) and its lanes cooperate through shuffles that stay
// inside the group.  Group lanes are converged whenever a group collective
// is called.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define SP_INF32 0xFFFFFFFFu
#define SP_MAXW 0xFFFFFFFEu
#define SP_NOMID 0xFFFFFFFFu
#define SP_EMPTY32 0xFFFFFFFFu
#define SP_EMPTY64 0xFFFFFFFFFFFFFFFFull
#define SP_INF64 0xFFFFFFFFFFFFFFFFull

namespace sp {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Orders LDS accesses between lanes of one wave (the wave executes in
// lockstep, but the compiler must not move LDS operations across this point).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int G>
__device__ __forceinline__ int glane() { return lane_id() & (G - 1); }

template <int G>
__device__ __forceinline__ uint64_t group_mask_bits() {
  return G == 64 ? ~0ull : (((1ull << G) - 1ull) << (lane_id() & ~(G - 1)));
}

// Ballot restricted to this lane's group, shifted down to bit 0.
template <int G>
__device__ __forceinline__ uint64_t gballot(bool p) {
  uint64_t b = __ballot(p);
  if constexpr (G == 64) return b;
  else return (b >> (lane_id() & ~(G - 1))) & ((1ull << G) - 1ull);
}

template <int G>
__device__ __forceinline__ bool gany(bool p) { return gballot<G>(p) != 0; }

template <int G, typename T>
__device__ __forceinline__ T gshfl(T v, int src) { return __shfl(v, src, G); }

template <int G>
__device__ __forceinline__ uint32_t gsum(uint32_t v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
  return v;
}

template <int G>
__device__ __forceinline__ uint64_t gsum64(uint64_t v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
  return v;
}

template <int G>
__device__ __forceinline__ uint32_t gmax(uint32_t v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor(v, o, G));
  return v;
}

template <int G>
__device__ __forceinline__ uint32_t gmin(uint32_t v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v = min(v, (uint32_t)__shfl_xor(v, o, G));
  return v;
}

template <int G>
__device__ __forceinline__ uint64_t gmin64(uint64_t v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) {
    uint64_t x = __shfl_xor(v, o, G);
    v = x < v ? x : v;
  }
  return v;
}

// Inclusive prefix sum over the group.
template <int G>
__device__ __forceinline__ uint32_t gscan_incl(uint32_t v) {
  const int l = glane<G>();
#pragma unroll
  for (int o = 1; o < G; o <<= 1) {
    uint32_t x = __shfl_up(v, o, G);
    if (l >= o) v += x;
  }
  return v;
}

// Lowest group lane whose inclusive prefix exceeds idx (binary search over
// the group's prefix values; every group lane must call it).
template <int G>
__device__ __forceinline__ int gfind(uint32_t incl, uint32_t idx) {
  int lo = 0;
#pragma unroll
  for (int step = G / 2; step > 0; step >>= 1) {
    int probe = lo + step - 1;
    uint32_t pv = __shfl(incl, probe, G);
    if (pv <= idx) lo += step;
  }
  return lo;
}

// Published integer hashes (own implementations):
//  - fmix32: the 32-bit finaliser of Appleby's MurmurHash3 (a bijection);
//  - lowbias32: Wellons' "hash-prospector" 32-bit mixer.
__host__ __device__ __forceinline__ uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

__host__ __device__ __forceinline__ uint32_t lowbias32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

// ---------------------------------------------------------------------------
// Memo: open addressing over 16-byte slots {key = (s << 32) | v, value},
// grouped in buckets of 16 slots (256 bytes).  The probe sequence of a pair
// visits bucket 0 in the region of its source s (W adjacent buckets starting
// at a bucket chosen by s, the one inside it chosen by v), then buckets
// chosen by the pair; inside a bucket it starts at a pair-dependent slot and
// wraps.  So the entries of one source share W buckets, and the builder
// sizes W (a power of two, `wmask` = W - 1) from the entries per live source
// whenever it rebuilds the table: W = 1 while sources hold a few entries
// (all of a source's lookups touch one bucket), larger once they hold
// hundreds (a lookup still resolves in its first bucket).  `bmask` = number
// of buckets - 1.
// ---------------------------------------------------------------------------
struct MemoSlot {
  uint64_t key;
  uint32_t val;
  uint32_t pad;
};

struct MemoRef {
  MemoSlot *t;
  uint64_t bmask;
  uint64_t wmask;
};

constexpr uint32_t kMemoBucket = 16;

// splitmix64 finaliser (Steele, Lea and Flood).
__host__ __device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// Hash of the pair's target: the low 4 bits pick the first slot inside a
// bucket, the rest the bucket inside the source's region.
__device__ __forceinline__ uint32_t memo_vhash(uint32_t v) { return lowbias32(v ^ 0x9e3779b9u); }

__device__ __forceinline__ uint64_t memo_bucket(const MemoRef &m, uint64_t k, uint32_t s,
                                                uint32_t hv, uint32_t i) {
  return (i == 0 ? mix64(s) + ((hv >> 4) & m.wmask)
                 : mix64(k ^ (0x9E3779B97F4A7C15ull * i))) & m.bmask;
}

// Returns the stored value or SP_INF32 when the pair is absent.  Slots are
// read four at a time (independent loads inside one bucket), then checked
// in probe order.  The probe sequence starts at slot j0 of the first bucket
// (the earlier slots known to hold neither the pair nor an empty slot).
__device__ __forceinline__ uint32_t memo_get_from(const MemoRef &m, uint32_t s, uint32_t v,
                                                  uint32_t j0, uint32_t *probes) {
  const uint64_t k = ((uint64_t)s << 32) | v;
  const uint32_t hv = memo_vhash(v);
  const uint32_t o = hv & (kMemoBucket - 1);
  for (uint32_t i = 0;; i++) {
    const MemoSlot *b = m.t + memo_bucket(m, k, s, hv, i) * kMemoBucket;
    for (uint32_t j = i == 0 ? j0 : 0; j < kMemoBucket; j += 4) {
      ulonglong2 e[4];
#pragma unroll
      for (int q = 0; q < 4; q++)
        e[q] = *reinterpret_cast<const ulonglong2 *>(&b[(o + j + q) & (kMemoBucket - 1)]);
      // first slot in probe order holding the pair or empty; selects keep
      // e[] in registers (an indexed read would move it to scratch)
      uint32_t r = SP_INF32;
      bool done = false;
#pragma unroll
      for (int q = 0; q < 4; q++) {
        if (done) continue;
        (*probes)++;
        if (e[q].x == k) {
          r = (uint32_t)e[q].y;
          done = true;
        } else if (e[q].x == SP_EMPTY64) {
          done = true;
        }
      }
      if (done) return r;
    }
  }
}

__device__ __forceinline__ uint32_t memo_get(const MemoRef &m, uint32_t s, uint32_t v,
                                             uint32_t *probes) {
  return memo_get_from(m, s, v, 0, probes);
}

// Lookups per lane batched by the pair loops of score, contract and prune.
constexpr int kPairBatch = 4;

// K lookups at once: the first four slots of every lookup are loaded before
// any is examined (4K independent loads in flight), the rare lookups that
// need more slots continue one by one.  out[k] = SP_INF32 for inactive k.
template <int K>
__device__ __forceinline__ void memo_get_batch(const MemoRef &m, const uint32_t (&s)[K],
                                               const uint32_t (&v)[K], const bool (&act)[K],
                                               uint32_t (&out)[K], uint32_t *probes) {
  ulonglong2 e[K][4];
  uint64_t key[K];
#pragma unroll
  for (int k = 0; k < K; k++) {
    key[k] = ((uint64_t)s[k] << 32) | v[k];
    const uint32_t hv = memo_vhash(v[k]);
    const uint32_t o = hv & (kMemoBucket - 1);
    const MemoSlot *b = m.t + memo_bucket(m, key[k], s[k], hv, 0) * kMemoBucket;
#pragma unroll
    for (int q = 0; q < 4; q++) {
      e[k][q] = make_ulonglong2(SP_EMPTY64, 0ull);
      if (act[k]) e[k][q] = *reinterpret_cast<const ulonglong2 *>(&b[(o + q) & (kMemoBucket - 1)]);
    }
  }
#pragma unroll
  for (int k = 0; k < K; k++) {
    uint32_t r = SP_INF32;
    bool done = !act[k];
#pragma unroll
    for (int q = 0; q < 4; q++) {
      if (done) continue;
      (*probes)++;
      if (e[k][q].x == key[k]) {
        r = (uint32_t)e[k][q].y;
        done = true;
      } else if (e[k][q].x == SP_EMPTY64) {
        done = true;
      }
    }
    if (!done) r = memo_get_from(m, s[k], v[k], 4, probes);
    out[k] = r;
  }
}

// Insert (s, v) -> val if the pair is absent (first writer wins).  The
// table is kept at most half full, so an empty slot is always reached.
__device__ __forceinline__ void memo_put(const MemoRef &m, uint32_t s, uint32_t v, uint32_t val) {
  const uint64_t k = ((uint64_t)s << 32) | v;
  const uint32_t hv = memo_vhash(v);
  const uint32_t o = hv & (kMemoBucket - 1);
  for (uint32_t i = 0;; i++) {
    MemoSlot *b = m.t + memo_bucket(m, k, s, hv, i) * kMemoBucket;
    for (uint32_t j = 0; j < kMemoBucket; j++) {
      MemoSlot *slot = &b[(o + j) & (kMemoBucket - 1)];
      uint64_t cur = __hip_atomic_load(&slot->key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (cur == k) return;
      if (cur == SP_EMPTY64) {
        uint64_t prev = atomicCAS((unsigned long long *)&slot->key,
                                  (unsigned long long)SP_EMPTY64, (unsigned long long)k);
        if (prev == SP_EMPTY64) {
          slot->val = val;
          return;
        }
        if (prev == k) return;
      }
    }
  }
}

// Device-side error flags (bit set by any kernel, read by the host).
enum : uint32_t {
  kErrOverflow = 1u,  // search bound or shortcut weight above 0xFFFFFFFE
  kErrCapacity = 2u,  // an internal buffer bound was exceeded (a bug)
};

}  // namespace sp
