// prim.hpp -- device-wide primitives (scan, compaction, radix sort) used by
// the CH builder.  All run on a caller-given stream; scratch memory comes
// from a caller-owned Workspace.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace sp {

// Growable device buffer (grows by 1.5x, never shrinks).  Blocks come from
// and go back to a per-device cache of released blocks (at most a quarter
// of the device's memory), so repeated builds and queries do not pay hipMalloc / hipFree:
// taking a cached block first synchronises the device, so a block released
// while a kernel on another stream may still use it is never handed out
// early.
struct DBuf {
  void *p = nullptr;
  size_t cap = 0;
  int dev = -1;  // device of the allocation
  hipError_t ensure(size_t bytes);
  void release();
  template <typename T>
  T *as() const { return reinterpret_cast<T *>(p); }
};

// Exclusive scan of n uint32 values; out may alias in.  *total_dev (device
// pointer, may be null) receives the sum.
hipError_t scan_u32(const uint32_t *in, uint32_t *out, uint32_t n, uint32_t *total_dev,
                    DBuf &tmp, hipStream_t st);
// Same for uint64 values.
hipError_t scan_u64(const uint64_t *in, uint64_t *out, uint64_t n, uint64_t *total_dev,
                    DBuf &tmp, hipStream_t st);

// out[k] = i for the k-th i (ascending) with flags[i] != 0; *count_dev = k.
hipError_t select_flags(const uint8_t *flags, uint32_t n, uint32_t *out, uint32_t *count_dev,
                        DBuf &tmp, hipStream_t st);
// select_flags of two flag arrays of the same length (one launch when small).
hipError_t select_flags2(const uint8_t *f0, const uint8_t *f1, uint32_t n, uint32_t *out0,
                         uint32_t *out1, uint32_t *count0, uint32_t *count1, DBuf &tmp,
                         hipStream_t st);

// Stable LSD radix sort of (key, value) pairs on key bits [0, bits).
// Results end in keys/vals (the alt buffers are scratch of the same size).
hipError_t radix_sort_u64(uint64_t *keys, uint32_t *vals, uint64_t *keys_alt,
                          uint32_t *vals_alt, uint32_t n, int bits, DBuf &tmp, hipStream_t st);

// Fill helpers.
// Up to three exclusive scans of n entries each (one launch when n is
// small); an array with a null input is skipped.
hipError_t scan3_u32(const uint32_t *in0, uint32_t *out0, uint32_t *tot0, const uint32_t *in1,
                     uint32_t *out1, uint32_t *tot1, const uint32_t *in2, uint32_t *out2,
                     uint32_t *tot2, uint32_t n, DBuf &tmp, hipStream_t st);
// Sort keys by their low `bits` bits; vals receive each key's original
// index (ties in index order, as a stable sort).
hipError_t sort_u64_index(uint64_t *keys, uint32_t *vals, uint64_t *keys_alt, uint32_t *vals_alt,
                          uint32_t n, int bits, DBuf &tmp, hipStream_t st);
hipError_t fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t st);
hipError_t fill_u64(uint64_t *p, uint64_t v, size_t n, hipStream_t st);
hipError_t fill_u8(uint8_t *p, uint8_t v, size_t n, hipStream_t st);
hipError_t iota_u32(uint32_t *p, uint32_t n, hipStream_t st);

}  // namespace sp
