// prim.hip -- scan, compaction and radix sort for gfx950.
#include "common.hpp"
#include "prim.hpp"

namespace sp {

hipError_t DBuf::ensure(size_t bytes) {
  if (bytes <= cap) return hipSuccess;
  size_t nc = cap + cap / 2;
  if (nc < bytes) nc = bytes;
  if (nc < 256) nc = 256;
  if (p) {
    hipError_t e = hipFree(p);
    if (e != hipSuccess) return e;
    p = nullptr;
    cap = 0;
  }
  hipError_t e = hipMalloc(&p, nc);
  if (e != hipSuccess) {
    p = nullptr;
    return e;
  }
  cap = nc;
  return hipSuccess;
}

void DBuf::release() {
  if (p) (void)hipFree(p);
  p = nullptr;
  cap = 0;
}

// ---------------------------------------------------------------------------
// fills
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_fill(T *p, T v, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

__global__ void k_iota(uint32_t *p, uint32_t n) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t stride = gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = i;
}

static unsigned grid_for(size_t n, unsigned block = 256, unsigned maxg = 8192) {
  size_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > maxg) g = maxg;
  return (unsigned)g;
}

hipError_t fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t st) {
  if (!n) return hipSuccess;
  k_fill<uint32_t><<<grid_for(n), 256, 0, st>>>(p, v, n);
  return hipGetLastError();
}
hipError_t fill_u64(uint64_t *p, uint64_t v, size_t n, hipStream_t st) {
  if (!n) return hipSuccess;
  k_fill<uint64_t><<<grid_for(n), 256, 0, st>>>(p, v, n);
  return hipGetLastError();
}
hipError_t fill_u8(uint8_t *p, uint8_t v, size_t n, hipStream_t st) {
  if (!n) return hipSuccess;
  k_fill<uint8_t><<<grid_for(n), 256, 0, st>>>(p, v, n);
  return hipGetLastError();
}
hipError_t iota_u32(uint32_t *p, uint32_t n, hipStream_t st) {
  if (!n) return hipSuccess;
  k_iota<<<grid_for(n), 256, 0, st>>>(p, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// scan: tiles of 256 threads x 8 items; block sums scanned recursively
// ---------------------------------------------------------------------------
constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanBlock * kScanItems;

template <typename T>
__device__ T block_excl_scan(T v, T *total) {
  __shared__ T warp_tot[kScanBlock / kWave];
  const int lane = lane_id(), w = threadIdx.x / kWave;
  T incl = v;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    T x = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += x;
  }
  if (lane == kWave - 1) warp_tot[w] = incl;
  __syncthreads();
  T pre = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kScanBlock / kWave; i++) {
    if (i < w) pre += warp_tot[i];
    tot += warp_tot[i];
  }
  __syncthreads();
  *total = tot;
  return pre + incl - v;
}

template <typename T>
__global__ void k_tile_sum(const T *__restrict__ in, uint64_t n, T *__restrict__ sums) {
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
  T s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; k++) {
    uint64_t i = base + (uint64_t)k * kScanBlock + threadIdx.x;
    if (i < n) s += in[i];
  }
  T tot;
  (void)block_excl_scan<T>(s, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

template <typename T>
__global__ void k_tile_scan(const T *__restrict__ in, T *__restrict__ out, uint64_t n,
                            const T *__restrict__ offs, T *__restrict__ total) {
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
  T v[kScanItems];
  T s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; k++) {
    uint64_t i = base + k;
    v[k] = i < n ? in[i] : (T)0;
    s += v[k];
  }
  T tot;
  T pre = block_excl_scan<T>(s, &tot) + (offs ? offs[blockIdx.x] : (T)0);
#pragma unroll
  for (int k = 0; k < kScanItems; k++) {
    uint64_t i = base + k;
    if (i < n) out[i] = pre;
    pre += v[k];
  }
  if (total && blockIdx.x == gridDim.x - 1 && threadIdx.x == kScanBlock - 1) *total = pre;
}

template <typename T>
static hipError_t scan_impl(const T *in, T *out, uint64_t n, T *total, DBuf &tmp, size_t tmp_off,
                            hipStream_t st) {
  if (n == 0) {
    if (total) return hipMemsetAsync(total, 0, sizeof(T), st);
    return hipSuccess;
  }
  const uint64_t tiles = (n + kScanTile - 1) / kScanTile;
  if (tiles == 1) {
    k_tile_scan<T><<<1, kScanBlock, 0, st>>>(in, out, n, nullptr, total);
    return hipGetLastError();
  }
  // layout of tmp from tmp_off: sums[tiles] (recursion uses the space after)
  size_t need = tmp_off + (tiles + 64) * sizeof(T);
  if (need > tmp.cap) return hipErrorInvalidValue;
  T *sums = reinterpret_cast<T *>(static_cast<char *>(tmp.p) + tmp_off);
  k_tile_sum<T><<<(unsigned)tiles, kScanBlock, 0, st>>>(in, n, sums);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = scan_impl<T>(sums, sums, tiles, total, tmp, tmp_off + (tiles + 64) * sizeof(T), st);
  if (e != hipSuccess) return e;
  k_tile_scan<T><<<(unsigned)tiles, kScanBlock, 0, st>>>(in, out, n, sums, nullptr);
  return hipGetLastError();
}

template <typename T>
static size_t scan_tmp_bytes(uint64_t n) {
  size_t b = 0;
  while (n > (uint64_t)kScanTile) {
    n = (n + kScanTile - 1) / kScanTile;
    b += (n + 64) * sizeof(T);
  }
  return b + 256;
}

hipError_t scan_u32(const uint32_t *in, uint32_t *out, uint32_t n, uint32_t *total, DBuf &tmp,
                    hipStream_t st) {
  hipError_t e = tmp.ensure(scan_tmp_bytes<uint32_t>(n));
  if (e != hipSuccess) return e;
  return scan_impl<uint32_t>(in, out, n, total, tmp, 0, st);
}

hipError_t scan_u64(const uint64_t *in, uint64_t *out, uint64_t n, uint64_t *total, DBuf &tmp,
                    hipStream_t st) {
  hipError_t e = tmp.ensure(scan_tmp_bytes<uint64_t>(n));
  if (e != hipSuccess) return e;
  return scan_impl<uint64_t>(in, out, n, total, tmp, 0, st);
}

// ---------------------------------------------------------------------------
// select_flags: per-tile counts, scan, ordered scatter
// ---------------------------------------------------------------------------
__global__ void k_flag_count(const uint8_t *__restrict__ f, uint32_t n, uint32_t *__restrict__ cnt) {
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
  uint32_t c = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; k++) {
    uint64_t i = base + (uint64_t)k * kScanBlock + threadIdx.x;
    if (i < n && f[i]) c++;
  }
  uint32_t tot;
  (void)block_excl_scan<uint32_t>(c, &tot);
  if (threadIdx.x == 0) cnt[blockIdx.x] = tot;
}

__global__ void k_flag_scatter(const uint8_t *__restrict__ f, uint32_t n,
                               const uint32_t *__restrict__ offs, uint32_t *__restrict__ out) {
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
  uint32_t c = 0;
  uint8_t v[kScanItems];
#pragma unroll
  for (int k = 0; k < kScanItems; k++) {
    uint64_t i = base + k;
    v[k] = (i < n) ? f[i] : 0;
    c += v[k] != 0;
  }
  uint32_t tot;
  uint32_t pre = block_excl_scan<uint32_t>(c, &tot) + offs[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanItems; k++)
    if (v[k]) out[pre++] = (uint32_t)(base + k);
}

hipError_t select_flags(const uint8_t *flags, uint32_t n, uint32_t *out, uint32_t *count,
                        DBuf &tmp, hipStream_t st) {
  if (n == 0) return hipMemsetAsync(count, 0, sizeof(uint32_t), st);
  const uint32_t tiles = (n + kScanTile - 1) / kScanTile;
  hipError_t e = tmp.ensure((tiles + 64) * sizeof(uint32_t) + scan_tmp_bytes<uint32_t>(tiles));
  if (e != hipSuccess) return e;
  uint32_t *cnt = tmp.as<uint32_t>();
  k_flag_count<<<tiles, kScanBlock, 0, st>>>(flags, n, cnt);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  e = scan_impl<uint32_t>(cnt, cnt, tiles, count, tmp, (tiles + 64) * sizeof(uint32_t), st);
  if (e != hipSuccess) return e;
  k_flag_scatter<<<tiles, kScanBlock, 0, st>>>(flags, n, cnt, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// radix sort: 8-bit digits; per pass a tile histogram, a scan of the
// digit-major count table, and a stable scatter that ranks keys of equal
// digit within a tile with wave match masks.
// ---------------------------------------------------------------------------
constexpr int kSortBlock = 256;
constexpr int kSortItems = 16;  // rounds of 256 keys per tile
constexpr int kSortTile = kSortBlock * kSortItems;
constexpr int kWavesPerSortBlock = kSortBlock / kWave;

__global__ void k_sort_hist(const uint64_t *__restrict__ keys, uint32_t n, int shift,
                            uint32_t *__restrict__ hist, uint32_t tiles) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t base = (uint64_t)blockIdx.x * kSortTile;
  for (int k = 0; k < kSortItems; k++) {
    uint64_t i = base + (uint64_t)k * kSortBlock + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(uint64_t)threadIdx.x * tiles + blockIdx.x] = h[threadIdx.x];
}

// Lanes of this wave whose digit equals mine (over active lanes).
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid) {
  uint64_t m = __ballot(valid);
#pragma unroll
  for (int b = 0; b < 8; b++) {
    bool bit = (d >> b) & 1u;
    uint64_t bb = __ballot(bit && valid);
    m &= bit ? bb : ~bb;
  }
  return m;
}

__global__ void k_sort_scatter(const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin,
                               uint64_t *__restrict__ kout, uint32_t *__restrict__ vout,
                               uint32_t n, int shift, const uint32_t *__restrict__ offs,
                               uint32_t tiles) {
  __shared__ uint32_t run[256];                      // keys of each digit placed so far
  __shared__ uint32_t wcnt[kWavesPerSortBlock][256];  // per-wave digit counts this round
  const int lane = lane_id(), w = threadIdx.x / kWave;
  run[threadIdx.x] = offs[(uint64_t)threadIdx.x * tiles + blockIdx.x];
  for (int i = 0; i < kWavesPerSortBlock; i++) wcnt[i][threadIdx.x] = 0;
  __syncthreads();
  const uint64_t base = (uint64_t)blockIdx.x * kSortTile;
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int k = 0; k < kSortItems; k++) {
    const uint64_t i = base + (uint64_t)k * kSortBlock + threadIdx.x;
    const bool valid = i < n;
    uint64_t key = valid ? kin[i] : 0;
    uint32_t val = valid ? vin[i] : 0;
    uint32_t d = (uint32_t)(key >> shift) & 255u;
    uint64_t peers = match_digit(d, valid);
    uint32_t wrank = __popcll(peers & lt_mask);
    bool leader = valid && (peers & lt_mask) == 0;
    if (leader) wcnt[w][d] = __popcll(peers);
    __syncthreads();
    // thread t owns digit t: convert per-wave counts to exclusive offsets
    {
      uint32_t acc = run[threadIdx.x];
      for (int j = 0; j < kWavesPerSortBlock; j++) {
        uint32_t c = wcnt[j][threadIdx.x];
        wcnt[j][threadIdx.x] = acc;
        acc += c;
      }
      run[threadIdx.x] = acc;
    }
    __syncthreads();
    if (valid) {
      uint32_t pos = wcnt[w][d] + wrank;
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
    for (int j = 0; j < kWavesPerSortBlock; j++) wcnt[j][threadIdx.x] = 0;
    __syncthreads();
  }
}

hipError_t radix_sort_u64(uint64_t *keys, uint32_t *vals, uint64_t *keys_alt, uint32_t *vals_alt,
                          uint32_t n, int bits, DBuf &tmp, hipStream_t st) {
  if (n <= 1 || bits <= 0) return hipSuccess;
  const uint32_t tiles = (n + kSortTile - 1) / kSortTile;
  const uint64_t hn = (uint64_t)tiles * 256;
  hipError_t e = tmp.ensure(hn * sizeof(uint32_t) + scan_tmp_bytes<uint32_t>(hn) + 256);
  if (e != hipSuccess) return e;
  uint32_t *hist = tmp.as<uint32_t>();
  const size_t scan_off = ((hn * sizeof(uint32_t) + 255) / 256) * 256;
  uint64_t *ka = keys, *kb = keys_alt;
  uint32_t *va = vals, *vb = vals_alt;
  int passes = 0;
  for (int shift = 0; shift < bits; shift += 8, passes++) {
    k_sort_hist<<<tiles, kSortBlock, 0, st>>>(ka, n, shift, hist, tiles);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    e = scan_impl<uint32_t>(hist, hist, hn, nullptr, tmp, scan_off, st);
    if (e != hipSuccess) return e;
    k_sort_scatter<<<tiles, kSortBlock, 0, st>>>(ka, va, kb, vb, n, shift, hist, tiles);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    uint64_t *tk = ka;
    ka = kb;
    kb = tk;
    uint32_t *tv = va;
    va = vb;
    vb = tv;
  }
  if (passes & 1) {
    e = hipMemcpyAsync(keys, ka, (size_t)n * sizeof(uint64_t), hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(vals, va, (size_t)n * sizeof(uint32_t), hipMemcpyDeviceToDevice, st);
  }
  return e;
}

}  // namespace sp
