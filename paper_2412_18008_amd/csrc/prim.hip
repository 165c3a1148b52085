// prim.hip -- scan, compaction and radix sort for gfx950.
#include "common.hpp"
#include "prim.hpp"

#include <map>
#include <mutex>

namespace sp {

namespace {

struct BlockCache {
  std::mutex mu;
  std::multimap<std::pair<int, size_t>, void *> blocks;  // (device, size) -> block
  std::map<int, size_t> bytes;                            // cached bytes per device
  std::map<int, size_t> limit;                            // cap per device
};

// Cache cap of a device: a quarter of its memory (72 GB of the 288 GB of an
// MI355X), so that a batch of hundreds of CHs can be built, queried and
// freed repeatedly without hipMalloc / hipFree (each CH holds about 30
// buffers); an allocation that fails empties the cache and retries.
size_t cache_limit(BlockCache &c, int dev) {
  auto it = c.limit.find(dev);
  if (it != c.limit.end()) return it->second;
  hipDeviceProp_t prop;
  size_t lim = 32ull << 30;
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.totalGlobalMem)
    lim = prop.totalGlobalMem / 4;
  c.limit[dev] = lim;
  return lim;
}

BlockCache &block_cache() {
  static BlockCache *c = new BlockCache;  // lives until the process ends
  return *c;
}

// Allocation size class: whole MiB from 1 MiB up, else a power of two.
size_t size_class(size_t b) {
  if (b >= (1u << 20)) return (b + (1u << 20) - 1) & ~(size_t)((1u << 20) - 1);
  size_t c = 256;
  while (c < b) c <<= 1;
  return c;
}

// A cached block of device dev with at least `bytes` and at most twice that.
void *cache_take(int dev, size_t bytes, size_t *got) {
  BlockCache &c = block_cache();
  std::lock_guard<std::mutex> g(c.mu);
  auto it = c.blocks.lower_bound({dev, bytes});
  if (it == c.blocks.end() || it->first.first != dev || it->first.second > 2 * bytes)
    return nullptr;
  void *p = it->second;
  *got = it->first.second;
  c.bytes[dev] -= *got;
  c.blocks.erase(it);
  return p;
}

// Frees every cached block of device dev (before retrying an allocation).
void cache_flush(int dev) {
  BlockCache &c = block_cache();
  std::lock_guard<std::mutex> g(c.mu);
  for (auto it = c.blocks.begin(); it != c.blocks.end();) {
    if (it->first.first == dev) {
      (void)hipFree(it->second);
      it = c.blocks.erase(it);
    } else {
      ++it;
    }
  }
  c.bytes[dev] = 0;
}

}  // namespace

hipError_t DBuf::ensure(size_t bytes) {
  if (bytes <= cap) return hipSuccess;
  size_t nc = cap + cap / 2;
  if (nc < bytes) nc = bytes;
  nc = size_class(nc);
  release();
  int d = 0;
  hipError_t e = hipGetDevice(&d);
  if (e != hipSuccess) return e;
  size_t got = 0;
  if (void *q = cache_take(d, nc, &got)) {
    e = hipDeviceSynchronize();  // no kernel may still use the block
    if (e != hipSuccess) {
      (void)hipFree(q);
      return e;
    }
    p = q;
    cap = got;
    dev = d;
    return hipSuccess;
  }
  e = hipMalloc(&p, nc);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    cache_flush(d);
    e = hipMalloc(&p, nc);
  }
  if (e != hipSuccess) {
    p = nullptr;
    return e;
  }
  cap = nc;
  dev = d;
  return hipSuccess;
}

void DBuf::release() {
  if (!p) return;
  BlockCache &c = block_cache();
  bool kept = false;
  {
    std::lock_guard<std::mutex> g(c.mu);
    size_t &b = c.bytes[dev];
    if (b + cap <= cache_limit(c, dev)) {
      c.blocks.emplace(std::make_pair(dev, cap), p);
      b += cap;
      kept = true;
    }
  }
  if (!kept) (void)hipFree(p);
  p = nullptr;
  cap = 0;
  dev = -1;
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

// ---------------------------------------------------------------------------
// single-block primitives for small inputs (one launch each): 1024 threads x
// 8 consecutive items
// ---------------------------------------------------------------------------
constexpr int kSmallBlock = 1024;
constexpr int kSmallItems = 8;
constexpr uint32_t kSmallN = kSmallBlock * kSmallItems;

template <typename T>
__device__ T small_block_excl_scan(T v, T *total) {
  __shared__ T wt[kSmallBlock / kWave];
  const int lane = lane_id(), w = threadIdx.x / kWave;
  T incl = v;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    T x = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += x;
  }
  if (lane == kWave - 1) wt[w] = incl;
  __syncthreads();
  T pre = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kSmallBlock / kWave; i++) {
    pre += i < w ? wt[i] : (T)0;
    tot += wt[i];
  }
  __syncthreads();
  *total = tot;
  return pre + incl - v;
}

// Exclusive scans of up to three arrays of n <= kSmallN entries (in == out
// allowed); null `in` skips that array.
template <typename T>
__global__ void __launch_bounds__(kSmallBlock) k_scan_small(const T *in0, T *out0, T *tot0,
                                                            const T *in1, T *out1, T *tot1,
                                                            const T *in2, T *out2, T *tot2,
                                                            uint32_t n) {
  const T *ins[3] = {in0, in1, in2};
  T *outs[3] = {out0, out1, out2};
  T *tots[3] = {tot0, tot1, tot2};
  const uint32_t base = threadIdx.x * kSmallItems;
  for (int a = 0; a < 3; a++) {
    if (!ins[a]) {
      if (tots[a] && threadIdx.x == 0) *tots[a] = 0;
      continue;
    }
    T v[kSmallItems];
    T c = 0;
#pragma unroll
    for (int k = 0; k < kSmallItems; k++) {
      v[k] = base + k < n ? ins[a][base + k] : (T)0;
      c += v[k];
    }
    T tot;
    T pre = small_block_excl_scan<T>(c, &tot);
#pragma unroll
    for (int k = 0; k < kSmallItems; k++) {
      if (base + k < n) outs[a][base + k] = pre;
      pre += v[k];
    }
    if (tots[a] && threadIdx.x == 0) *tots[a] = tot;
  }
}

template <typename T>
static hipError_t scan_impl(const T *in, T *out, uint64_t n, T *total, DBuf &tmp, size_t tmp_off,
                            hipStream_t st) {
  if (n <= kSmallN) {  // one launch, also for n == 0 (total = 0)
    k_scan_small<T><<<1, kSmallBlock, 0, st>>>(in, out, total, nullptr, nullptr, nullptr,
                                               nullptr, nullptr, nullptr, (uint32_t)n);
    return hipGetLastError();
  }
  const uint64_t tiles = (n + kScanTile - 1) / kScanTile;
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
  if (n && (!in || !out)) return hipErrorInvalidValue;
  hipError_t e = tmp.ensure(scan_tmp_bytes<uint32_t>(n));
  if (e != hipSuccess) return e;
  return scan_impl<uint32_t>(in, out, n, total, tmp, 0, st);
}

hipError_t scan3_u32(const uint32_t *in0, uint32_t *out0, uint32_t *tot0, const uint32_t *in1,
                     uint32_t *out1, uint32_t *tot1, const uint32_t *in2, uint32_t *out2,
                     uint32_t *tot2, uint32_t n, DBuf &tmp, hipStream_t st) {
  if (n <= kSmallN) {
    k_scan_small<uint32_t><<<1, kSmallBlock, 0, st>>>(in0, out0, tot0, in1, out1, tot1, in2, out2,
                                                      tot2, n);
    return hipGetLastError();
  }
  // arrays with a null input are skipped, as in the single-block kernel
  const uint32_t *ins[3] = {in0, in1, in2};
  uint32_t *outs[3] = {out0, out1, out2}, *tots[3] = {tot0, tot1, tot2};
  for (int a = 0; a < 3; a++) {
    if (!ins[a]) continue;
    hipError_t e = scan_u32(ins[a], outs[a], n, tots[a], tmp, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t scan_u64(const uint64_t *in, uint64_t *out, uint64_t n, uint64_t *total, DBuf &tmp,
                    hipStream_t st) {
  if (n && (!in || !out)) return hipErrorInvalidValue;
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

__global__ void __launch_bounds__(kSmallBlock) k_flag_select_small(const uint8_t *__restrict__ f,
                                                                   uint32_t n,
                                                                   uint32_t *__restrict__ out,
                                                                   uint32_t *__restrict__ count) {
  const uint32_t base = threadIdx.x * kSmallItems;
  uint8_t v[kSmallItems];
  uint32_t c = 0;
#pragma unroll
  for (int k = 0; k < kSmallItems; k++) {
    v[k] = base + k < n ? f[base + k] : 0;
    c += v[k] != 0;
  }
  uint32_t tot;
  uint32_t pre = small_block_excl_scan<uint32_t>(c, &tot);
#pragma unroll
  for (int k = 0; k < kSmallItems; k++)
    if (v[k]) out[pre++] = base + k;
  if (threadIdx.x == 0) *count = tot;
}

// Two flag arrays at once: block 0 compacts (f0, out0, count0), block 1
// (f1, out1, count1).
__global__ void __launch_bounds__(kSmallBlock) k_flag_select_small2(
    const uint8_t *__restrict__ f0, const uint8_t *__restrict__ f1, uint32_t n,
    uint32_t *__restrict__ out0, uint32_t *__restrict__ out1, uint32_t *__restrict__ count0,
    uint32_t *__restrict__ count1) {
  const uint8_t *f = blockIdx.x ? f1 : f0;
  uint32_t *out = blockIdx.x ? out1 : out0;
  const uint32_t base = threadIdx.x * kSmallItems;
  uint8_t v[kSmallItems];
  uint32_t c = 0;
#pragma unroll
  for (int k = 0; k < kSmallItems; k++) {
    v[k] = base + k < n ? f[base + k] : 0;
    c += v[k] != 0;
  }
  uint32_t tot;
  uint32_t pre = small_block_excl_scan<uint32_t>(c, &tot);
#pragma unroll
  for (int k = 0; k < kSmallItems; k++)
    if (v[k]) out[pre++] = base + k;
  if (threadIdx.x == 0) *(blockIdx.x ? count1 : count0) = tot;
}

hipError_t select_flags2(const uint8_t *f0, const uint8_t *f1, uint32_t n, uint32_t *out0,
                         uint32_t *out1, uint32_t *count0, uint32_t *count1, DBuf &tmp,
                         hipStream_t st) {
  if (!count0 || !count1 || (n && (!f0 || !f1 || !out0 || !out1))) return hipErrorInvalidValue;
  if (n <= kSmallN) {
    k_flag_select_small2<<<2, kSmallBlock, 0, st>>>(f0, f1, n, out0, out1, count0, count1);
    return hipGetLastError();
  }
  hipError_t e = select_flags(f0, n, out0, count0, tmp, st);
  if (e != hipSuccess) return e;
  return select_flags(f1, n, out1, count1, tmp, st);
}

hipError_t select_flags(const uint8_t *flags, uint32_t n, uint32_t *out, uint32_t *count,
                        DBuf &tmp, hipStream_t st) {
  if (!count || (n && (!flags || !out))) return hipErrorInvalidValue;
  if (n <= kSmallN) {  // one launch, also for n == 0
    k_flag_select_small<<<1, kSmallBlock, 0, st>>>(flags, n, out, count);
    return hipGetLastError();
  }
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

// (key, index) sort of n <= kSmallSort entries in one block: bitonic network
// in LDS over the keys' low `bits` bits, ties by index (the order a stable
// sort gives); vals receive the original indices.
constexpr uint32_t kSmallSort = 4096;

__global__ void __launch_bounds__(kSmallBlock) k_sort_small_iota(uint64_t *__restrict__ keys,
                                                                 uint32_t *__restrict__ vals,
                                                                 uint32_t n, uint64_t mask) {
  __shared__ uint64_t sk[kSmallSort];
  __shared__ uint32_t sv[kSmallSort];
  uint32_t np = 1;
  while (np < n) np <<= 1;
  for (uint32_t i = threadIdx.x; i < np; i += kSmallBlock) {
    sk[i] = i < n ? keys[i] : ~0ull;
    sv[i] = i < n ? i : 0xFFFFFFFFu;
  }
  __syncthreads();
  // each step compares np / 2 pairs (i, i + j): pair p has i = p with a
  // zero bit inserted at bit log2(j), so no thread idles on the upper halves
  for (uint32_t k = 2; k <= np; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t p = threadIdx.x; p < (np >> 1); p += kSmallBlock) {
        const uint32_t i = ((p & ~(j - 1)) << 1) | (p & (j - 1));
        const uint32_t l = i | j;
        const uint64_t a = sk[i] & mask, b = sk[l] & mask;
        const bool gt = a > b || (a == b && sv[i] > sv[l]);
        const bool up = (i & k) == 0;
        if (gt == up) {
          const uint64_t tk = sk[i];
          sk[i] = sk[l];
          sk[l] = tk;
          const uint32_t tv = sv[i];
          sv[i] = sv[l];
          sv[l] = tv;
        }
      }
      __syncthreads();
    }
  }
  for (uint32_t i = threadIdx.x; i < n; i += kSmallBlock) {
    keys[i] = sk[i];
    vals[i] = sv[i];
  }
}

hipError_t sort_u64_index(uint64_t *keys, uint32_t *vals, uint64_t *keys_alt, uint32_t *vals_alt,
                          uint32_t n, int bits, DBuf &tmp, hipStream_t st) {
  if (n == 0) return hipSuccess;
  if (!keys || !vals || (n > kSmallSort && (!keys_alt || !vals_alt))) return hipErrorInvalidValue;
  if (n <= kSmallSort) {
    const uint64_t mask = bits >= 64 ? ~0ull : ((1ull << bits) - 1ull);
    k_sort_small_iota<<<1, kSmallBlock, 0, st>>>(keys, vals, n, mask);
    return hipGetLastError();
  }
  hipError_t e = iota_u32(vals, n, st);
  if (e != hipSuccess) return e;
  return radix_sort_u64(keys, vals, keys_alt, vals_alt, n, bits, tmp, st);
}

}  // namespace sp
