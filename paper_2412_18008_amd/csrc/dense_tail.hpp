// dense_tail.hpp -- witness distances from an all-pairs table once the
// overlay is small.
//
// Contraction preserves the distance between every two vertices that are
// still in the overlay (a shortcut replaces exactly the path it removes,
// pruning only deletes arcs longer than a known distance), so the exact
// witness distance of a live pair (s, v) in any round is the overlay
// distance at any earlier round.  When the overlay has n0 <= the threshold
// vertices, the build computes all n0^2 distances once (blocked
// Floyd-Warshall over 64 x 64 tiles in LDS); every later round in exact
// mode answers its searches from the table: the same targets, radius D_s,
// memo entries (target distances <= D_s) and reached-vertex count as the
// search of Alg. 4 would give.
#pragma once

#include "common.hpp"
#include "search.hpp"

namespace sp {

constexpr int kFwTile = 64;     // tile edge
constexpr int kFwThreads = 256; // 16 entries of a tile per thread (4 x 4)

// a + b clamped to 0xFFFFFFFF: a distance above 0xFFFFFFFE (or through an
// absent entry) is stored as "none"; no witness radius reaches it.
__device__ __forceinline__ uint32_t sat_add(uint32_t a, uint32_t b) {
  return __builtin_elementwise_add_sat(a, b);  // one clamped 32-bit add
}

// Dense matrix N x N (N a multiple of kFwTile, row-major): none everywhere,
// 0 on the diagonal (padding rows included).
__global__ void k_fw_init(uint32_t *__restrict__ D, uint32_t N) {
  const uint64_t total = (uint64_t)N * N;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride)
    D[i] = (i / N == i % N) ? 0u : SP_INF32;
}

// Arcs of the overlay (local ids = matrix rows), and the position <-> original
// id maps of the table.
__global__ void k_fw_arcs(Overlay ov, uint32_t N, uint32_t *__restrict__ D,
                          uint32_t *__restrict__ pos_of_gid, uint32_t *__restrict__ gid_of_pos) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < ov.n; u += stride) {
    pos_of_gid[ov.gid[u]] = u;
    gid_of_pos[u] = ov.gid[u];
    for (uint32_t e = ov.foff[u]; e < ov.foff[u + 1]; e++) {
      const uint2 a = ov.farc[e];
      if (a.y != SP_INF32) atomicMin(&D[(size_t)u * N + a.x], a.y);
    }
  }
}

__device__ __forceinline__ void fw_load(uint32_t (*T)[kFwTile + 1], const uint32_t *D, uint32_t N,
                                        uint32_t ti, uint32_t tj) {
  for (int e = threadIdx.x; e < kFwTile * kFwTile; e += kFwThreads) {
    const int i = e / kFwTile, j = e % kFwTile;
    T[i][j] = D[(size_t)(ti * kFwTile + i) * N + tj * kFwTile + j];
  }
}

__device__ __forceinline__ void fw_store(const uint32_t (*T)[kFwTile + 1], uint32_t *D, uint32_t N,
                                         uint32_t ti, uint32_t tj) {
  for (int e = threadIdx.x; e < kFwTile * kFwTile; e += kFwThreads) {
    const int i = e / kFwTile, j = e % kFwTile;
    D[(size_t)(ti * kFwTile + i) * N + tj * kFwTile + j] = T[i][j];
  }
}

// acc[a][b] (entry (ty*4 + a, tx*4 + b) of a tile, ty = thread / 16, tx =
// thread % 16) = min(acc, min over k of A[row][k] + B[k][col]).
__device__ __forceinline__ void fw_minplus_acc(uint32_t (&acc)[4][4],
                                               const uint32_t (*A)[kFwTile + 1],
                                               const uint32_t (*B)[kFwTile + 1]) {
  const int ty = threadIdx.x / 16, tx = threadIdx.x % 16;
  for (int k = 0; k < kFwTile; k++) {
    uint32_t av[4], bv[4];
#pragma unroll
    for (int a = 0; a < 4; a++) av[a] = A[ty * 4 + a][k];
#pragma unroll
    for (int b = 0; b < 4; b++) bv[b] = B[k][tx * 4 + b];
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
      for (int b = 0; b < 4; b++) {
        const uint32_t c = sat_add(av[a], bv[b]);
        acc[a][b] = c < acc[a][b] ? c : acc[a][b];
      }
  }
}

// The 16 entries of a tile that this thread owns, straight from / to D.
__device__ __forceinline__ void fw_acc_load(uint32_t (&acc)[4][4], const uint32_t *D, uint32_t N,
                                            uint32_t ti, uint32_t tj) {
  const int ty = threadIdx.x / 16, tx = threadIdx.x % 16;
#pragma unroll
  for (int a = 0; a < 4; a++)
#pragma unroll
    for (int b = 0; b < 4; b++)
      acc[a][b] = D[(size_t)(ti * kFwTile + ty * 4 + a) * N + tj * kFwTile + tx * 4 + b];
}

__device__ __forceinline__ void fw_acc_store(const uint32_t (&acc)[4][4], uint32_t *D, uint32_t N,
                                             uint32_t ti, uint32_t tj) {
  const int ty = threadIdx.x / 16, tx = threadIdx.x % 16;
#pragma unroll
  for (int a = 0; a < 4; a++)
#pragma unroll
    for (int b = 0; b < 4; b++)
      D[(size_t)(ti * kFwTile + ty * 4 + a) * N + tj * kFwTile + tx * 4 + b] = acc[a][b];
}

// Phase k, step 1: closure of the diagonal tile (k, k) over its own 64
// intermediate vertices: the Floyd-Warshall loop in LDS, one barrier per
// pivot t.  Row t and column t keep their values while pivot t is applied
// (the diagonal stays 0 with non-negative weights), so every thread can
// update its own entries in place.  1024 threads, four entries of one row
// each.
constexpr int kFwDiagThreads = 1024;

__global__ void __launch_bounds__(kFwDiagThreads) k_fw_diag(uint32_t *__restrict__ D, uint32_t N,
                                                            uint32_t k) {
  __shared__ uint32_t T[kFwTile][kFwTile + 1];
  constexpr int kPer = kFwTile * kFwTile / kFwDiagThreads;  // 4
  const int i = threadIdx.x / (kFwTile / kPer), j0 = (threadIdx.x % (kFwTile / kPer)) * kPer;
  const size_t base = (size_t)(k * kFwTile + i) * N + (size_t)k * kFwTile + j0;
  uint32_t r[kPer];
#pragma unroll
  for (int q = 0; q < kPer; q++) {
    r[q] = D[base + q];
    T[i][j0 + q] = r[q];
  }
  __syncthreads();
  for (int t = 0; t < kFwTile; t++) {
    const uint32_t a = T[i][t];
#pragma unroll
    for (int q = 0; q < kPer; q++) r[q] = min(r[q], sat_add(a, T[t][j0 + q]));
#pragma unroll
    for (int q = 0; q < kPer; q++) T[i][j0 + q] = r[q];
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < kPer; q++) D[base + q] = r[q];
}

// Phase k, step 2: block b < nb updates row tile (k, b) and block nb + b
// column tile (b, k), b != k, with the closed diagonal tile: (k, b) <-
// closure(k, k) (x) (k, b) and (b, k) <- (b, k) (x) closure(k, k) (min-plus
// products; the closure's zero diagonal keeps the old entries).
__global__ void __launch_bounds__(kFwThreads) k_fw_panels(uint32_t *__restrict__ D, uint32_t N,
                                                          uint32_t k) {
  __shared__ uint32_t Dk[kFwTile][kFwTile + 1];
  __shared__ uint32_t T[kFwTile][kFwTile + 1];
  const uint32_t nb = N / kFwTile;
  const bool col = blockIdx.x >= nb;
  const uint32_t b = col ? blockIdx.x - nb : blockIdx.x;
  if (b == k) return;
  fw_load(Dk, D, N, k, k);
  if (col) fw_load(T, D, N, b, k);
  else fw_load(T, D, N, k, b);
  __syncthreads();
  uint32_t acc[4][4];
  const int ty = threadIdx.x / 16, tx = threadIdx.x % 16;
#pragma unroll
  for (int a = 0; a < 4; a++)
#pragma unroll
    for (int c = 0; c < 4; c++) acc[a][c] = T[ty * 4 + a][tx * 4 + c];
  if (col) fw_minplus_acc(acc, T, Dk);
  else fw_minplus_acc(acc, Dk, T);
  if (col) fw_acc_store(acc, D, N, b, k);
  else fw_acc_store(acc, D, N, k, b);
}

// Phase k, step 3: tile (i, j), i, j != k: min with (i, k) (x) (k, j).  The
// tile's own entries stay in registers.
__global__ void __launch_bounds__(kFwThreads) k_fw_rest(uint32_t *__restrict__ D, uint32_t N,
                                                        uint32_t k) {
  __shared__ uint32_t A[kFwTile][kFwTile + 1];
  __shared__ uint32_t B[kFwTile][kFwTile + 1];
  const uint32_t nb = N / kFwTile;
  const uint32_t i = blockIdx.x / nb, j = blockIdx.x % nb;
  if (i == k || j == k) return;
  fw_load(A, D, N, i, k);
  fw_load(B, D, N, k, j);
  uint32_t acc[4][4];
  fw_acc_load(acc, D, N, i, j);
  __syncthreads();
  fw_minplus_acc(acc, A, B);
  fw_acc_store(acc, D, N, i, j);
}

// Table position of every vertex of the current overlay (local ids change
// every round).
__global__ void k_tab_posl(uint32_t n, const uint32_t *__restrict__ gid,
                           const uint32_t *__restrict__ pos_of_gid, uint32_t *__restrict__ posl) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += stride)
    posl[u] = pos_of_gid[gid[u]];
}

// Witness search of Alg. 4 answered from the table (exact mode): one group
// of 64 lanes per source.  Per group in LDS: a seen bit and the largest
// two-arc length per table position.
constexpr int kTabMaxN = 4096;  // largest table the lookup kernel serves

__global__ void __launch_bounds__(64) k_ls_table(
    Overlay ov, const uint32_t *__restrict__ vw, uint32_t nw, const uint8_t *__restrict__ aflag,
    MemoRef memo, LsCounters *__restrict__ cnt,
    const uint32_t *__restrict__ Dtab, uint32_t N, uint32_t n0,
    const uint32_t *__restrict__ pos_of_gid, const uint32_t *__restrict__ gid_of_pos,
    const uint32_t *__restrict__ posl, const uint8_t *__restrict__ alive_g,
    uint32_t *__restrict__ ws, uint32_t *__restrict__ err) {
  __shared__ uint32_t s_seen[kTabMaxN / 32];
  __shared__ uint32_t s_tgt[kTabMaxN / 32];
  __shared__ uint32_t s_via[kTabMaxN];  // 0xFFFFFFFF - largest via (atomicMin)
  __shared__ uint16_t s_cand[kTabMaxN];  // positions of the candidates
  const int l = lane_id();
  const uint32_t words = (n0 + 31) / 32;
  SearchStats ss;
  for (uint32_t k = blockIdx.x; k < nw; k += gridDim.x) {
    const uint32_t s = vw[k];
    const uint32_t gs = ov.gid[s];
    const uint32_t ps = posl[s];
    wave_sync();  // the previous source's LDS reads come first
    for (uint32_t i = l; i < words; i += kWave) {
      s_seen[i] = 0;
      s_tgt[i] = 0;
    }
    for (uint32_t i = l; i < n0; i += kWave) s_via[i] = 0xFFFFFFFFu;
    wave_sync();
    // ---- targets: out-neighbours v != s of affected out-neighbours u
    const uint32_t a0 = ov.foff[s], a1 = ov.foff[s + 1];
    for (uint32_t base = a0; base < a1; base += kWave) {
      const uint32_t e = base + l;
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
      const uint32_t incl = gscan_incl<kWave>(rl);
      const uint32_t total = __shfl(incl, kWave - 1, kWave);
      constexpr int U = 8;  // arcs per lane gathered before use
      for (uint32_t i0 = 0; i0 < total; i0 += kWave * U) {
        uint2 b[U];
        uint32_t sw[U], p[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
          const uint32_t idx = i0 + u * kWave + l;
          b[u] = make_uint2(s, 0u);  // s itself is skipped below
          sw[u] = 0;
          if (i0 + u * kWave < total) {  // uniform across the wave
            const int src = gfind<kWave>(incl, idx);
            const uint32_t srs = __shfl(rs, src, kWave), sinc = __shfl(incl, src, kWave);
            const uint32_t srl = __shfl(rl, src, kWave);
            sw[u] = __shfl(wsu, src, kWave);
            if (idx < total) {
              b[u] = ov.farc[srs + (idx - (sinc - srl))];
              ss.arcs++;
            }
          }
        }
#pragma unroll
        for (int u = 0; u < U; u++) p[u] = b[u].x != s ? posl[b[u].x] : 0u;
#pragma unroll
        for (int u = 0; u < U; u++) {
          if (b[u].x == s) continue;
          const uint64_t via = (uint64_t)sw[u] + b[u].y;
          const uint32_t viac = via > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)via;
          atomicOr(&s_seen[p[u] >> 5], 1u << (p[u] & 31));
          atomicMin(&s_via[p[u]], 0xFFFFFFFFu - viac);
        }
      }
    }
    wave_sync();
    // ---- candidates in position order (bitmap compaction), then the
    // targets: candidates without a memo entry; radius D over them
    uint32_t c = 0;
    for (uint32_t w = l; w < words; w += kWave) c += __popc(s_seen[w]);
    uint32_t nc;
    {
      const uint32_t incl = gscan_incl<kWave>(c);
      nc = __shfl(incl, kWave - 1, kWave);
      uint32_t p = incl - c;
      for (uint32_t w = l; w < words; w += kWave) {
        uint32_t bits = s_seen[w];
        s_tgt[w] = 0;
        while (bits) {
          s_cand[p++] = (uint16_t)(w * 32 + __builtin_ctz(bits));
          bits &= bits - 1;
        }
      }
    }
    wave_sync();
    uint32_t D = 0, nt = 0;
    for (uint32_t i0 = l; i0 < nc; i0 += kWave * kPairBatch) {
      uint32_t ks[kPairBatch], kv[kPairBatch], got[kPairBatch], pos[kPairBatch];
      bool act[kPairBatch];
#pragma unroll
      for (int q = 0; q < kPairBatch; q++) {
        const uint32_t i = i0 + q * kWave;
        act[q] = i < nc;
        pos[q] = act[q] ? s_cand[i] : 0u;
        ks[q] = gs;
        kv[q] = act[q] ? gid_of_pos[pos[q]] : 0u;
      }
      memo_get_batch<kPairBatch>(memo, ks, kv, act, got, &ss.probes);
#pragma unroll
      for (int q = 0; q < kPairBatch; q++) {
        if (!act[q] || got[q] != SP_INF32) continue;
        atomicOr(&s_tgt[pos[q] >> 5], 1u << (pos[q] & 31));
        D = max(D, 0xFFFFFFFFu - s_via[pos[q]]);
        nt++;
      }
    }
    wave_sync();
    D = gmax<kWave>(D);
    nt = gsum<kWave>(nt);
    if (nt == 0) continue;
    if (D > SP_MAXW) {
      if (l == 0) atomicOr(err, kErrOverflow);
      continue;
    }
    ss.targets += l == 0 ? nt : 0;
    ss.searched += l == 0 ? 1 : 0;
    // ---- memo entries for targets within D; reached-vertex count
    const uint32_t *row = Dtab + (size_t)ps * N;
    uint32_t ball = 0;
    for (uint32_t p0 = l; p0 < n0; p0 += kWave * 4) {
      uint32_t d[4], g[4];
#pragma unroll
      for (int q = 0; q < 4; q++) {  // four row loads in flight
        const uint32_t p = p0 + q * kWave;
        d[q] = p < n0 ? row[p] : SP_INF32;
      }
#pragma unroll
      for (int q = 0; q < 4; q++) {
        const uint32_t p = p0 + q * kWave;
        g[q] = d[q] <= D ? gid_of_pos[p] : 0u;
      }
#pragma unroll
      for (int q = 0; q < 4; q++) {
        const uint32_t p = p0 + q * kWave;
        if (d[q] > D) continue;
        if (alive_g[g[q]]) ball++;
        if ((s_tgt[p >> 5] >> (p & 31)) & 1u) {
          memo_put(memo, gs, g[q], d[q]);
          ss.inserts++;
        }
      }
    }
    ball = gsum<kWave>(ball);
    if (ws && l == 0) ws[gs] = ball;
  }
  flush_stats<64>(ss, cnt);
}

}  // namespace sp
