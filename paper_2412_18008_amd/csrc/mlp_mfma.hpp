// mlp_mfma.hpp -- the learned priority's network in bf16 on the gfx950
// matrix cores: forward (inference) and forward + backward + parameter
// gradients (training), with bf16 operands and fp32 accumulation
// (v_mfma_f32_16x16x32_bf16).  Included by mlp.hip, which holds the GELU and
// bf16 rounding helpers.
//
// One wave takes 32 samples at a time (two 16-row MFMA tiles):
//   h1 = x W1^T + b1     (K = 8, zero-padded to one 32-wide K block)
//   a1 = bf16(GELU(h1)), h2 = a1 W2^T + b2, a2 = bf16(GELU(h2)),
//   y  = a2 . W3 + b3    (vector ALUs: a sum over the 16 lanes of a row).
// Training adds, for the mean squared error over a batch of B samples,
//   dy = 2 (y - t) / B, d2 = dy W3 * GELU'(h2), d1 = (d2 W2) * GELU'(h1),
//   dW2 += d2^T a1 and dW1 += d1^T x (MFMA with K = the 32 samples),
//   and the bias and W3 gradients on the vector ALUs.
// A wave keeps its gradient sums in registers over all its tiles and writes
// them once; a second kernel adds the waves' sums in wave order, so a
// result does not depend on timing.
//
// Operand layout (16x16x32): lane l, group g = l / 16, r = l % 16 holds
// A[row r][8 values of K block g] and B[8 values of K block g][column r];
// D holds rows 4g .. 4g+3 of column r.  A and B assign K to (g, element)
// the same way, so the order of K inside a block does not matter.
#pragma once

#include <hip/hip_runtime.h>

namespace sp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short short8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kMfmaWaves = 4;  // waves per block
constexpr int kMfmaRows = 32;  // samples per wave step

// bf16 bits of f (round to nearest even, the same as to_bf16).
__device__ __forceinline__ uint16_t bf16_bits(float f) {
  return (uint16_t)(__float_as_uint(to_bf16(f)) >> 16);
}
__device__ __forceinline__ float bf16_val(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ bf16x8 pack8(const float *v) {
  short8 s;
#pragma unroll
  for (int e = 0; e < 8; e++) s[e] = (short)bf16_bits(v[e]);
  return __builtin_bit_cast(bf16x8, s);
}
__device__ __forceinline__ bf16x8 zero8() {
  short8 s = {0, 0, 0, 0, 0, 0, 0, 0};
  return __builtin_bit_cast(bf16x8, s);
}
// eight consecutive bf16 values from LDS (16-byte aligned)
__device__ __forceinline__ bf16x8 lds8(const uint16_t *p) {
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const short8 *>(p));
}
__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
// sum over the 16 lanes of a group (same g)
__device__ __forceinline__ float sum16(float v) {
#pragma unroll
  for (int o = 1; o < 16; o <<= 1) v += __shfl_xor(v, o, 64);
  return v;
}
// sum over the four groups (same r)
__device__ __forceinline__ float sum_groups(float v) {
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}

// Per-wave LDS: activations and deltas of one 32-sample step as bf16, in
// sample-major (rm: [32][64]) and unit-major (cm: [64][32]) order.
struct MfmaLds {
  uint16_t a1_rm[kMfmaRows * 64];
  uint16_t a1_cm[64 * kMfmaRows];
  uint16_t d2_rm[kMfmaRows * 64];
  uint16_t d2_cm[64 * kMfmaRows];
  uint16_t d1_cm[64 * kMfmaRows];
  uint16_t x_cm[16 * kMfmaRows];
};

// Inference needs the sample-major activations only.
struct MfmaLdsFwd {
  uint16_t a1_rm[kMfmaRows * 64];
};

// Weight operands of one wave (bf16), loaded once.
struct MfmaWeights {
  bf16x8 B1[4];      // layer 1: B[k][n] = W1[n][k] (k < 8), n tile t
  bf16x8 B2[2][4];   // layer 2: B[k][n] = W2[n][k], K block kb, n tile t
  bf16x8 B2T[2][4];  // backward: B[k][n] = W2[k][n]
  float b1[4], b2[4], w3[4];  // per column r of each n tile (bf16 values)
  float b3;
  __device__ void load(const float *__restrict__ w, bool train) {
    const int l = (int)(threadIdx.x % 64), g = l / 16, r = l % 16;
    const float *W1 = w, *bb1 = w + 512, *W2 = w + 576, *bb2 = w + 4672, *W3 = w + 4736;
#pragma unroll
    for (int t = 0; t < 4; t++) {
      const int n = 16 * t + r;
      B1[t] = g == 0 ? pack8(W1 + n * 8) : zero8();
#pragma unroll
      for (int kb = 0; kb < 2; kb++) {
        B2[kb][t] = pack8(W2 + n * 64 + 32 * kb + 8 * g);
        if (train) {
          float v[8];
#pragma unroll
          for (int e = 0; e < 8; e++) v[e] = W2[(32 * kb + 8 * g + e) * 64 + n];
          B2T[kb][t] = pack8(v);
        }
      }
      b1[t] = to_bf16(bb1[n]);
      b2[t] = to_bf16(bb2[n]);
      w3[t] = to_bf16(W3[n]);
    }
    b3 = to_bf16(w[4800]);
  }
};

// Forward of one 32-sample step.  x rows (8 floats, or zeros past the
// end) of sub-tile h are given by row_of(h, r).  Leaves h1, h2 (fp32, D
// layout), a1 in LDS and y of rows 4g+i of sub-tile h in y[h][i] (every lane
// of the group).
template <bool TRAIN, typename LdsT, typename RowFn>
__device__ __forceinline__ void mfma_forward(const MfmaWeights &W, LdsT &S, RowFn row_of,
                                             f32x4 (&h1)[2][4], f32x4 (&h2)[2][4],
                                             float (&y)[2][4]) {
  const int l = (int)(threadIdx.x % 64), g = l / 16, r = l % 16;
#pragma unroll
  for (int h = 0; h < 2; h++) {
    float xv[8];
    row_of(h, r, xv);
    const bf16x8 A1 = g == 0 ? pack8(xv) : zero8();
    if constexpr (TRAIN) {
      if (g == 0) {
#pragma unroll
        for (int k = 0; k < 8; k++) S.x_cm[k * kMfmaRows + 16 * h + r] = bf16_bits(xv[k]);
      }
    }
#pragma unroll
    for (int t = 0; t < 4; t++) {
      f32x4 c = {W.b1[t], W.b1[t], W.b1[t], W.b1[t]};
      h1[h][t] = mfma(A1, W.B1[t], c);
#pragma unroll
      for (int i = 0; i < 4; i++) {
        const uint16_t a = bf16_bits(gelu_pade(h1[h][t][i]));
        const int s = 16 * h + 4 * g + i, n = 16 * t + r;
        S.a1_rm[s * 64 + n] = a;
        if constexpr (TRAIN) S.a1_cm[n * kMfmaRows + s] = a;
      }
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
  for (int h = 0; h < 2; h++) {
    const bf16x8 A20 = lds8(&S.a1_rm[(16 * h + r) * 64 + 8 * g]);
    const bf16x8 A21 = lds8(&S.a1_rm[(16 * h + r) * 64 + 32 + 8 * g]);
    float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < 4; t++) {
      f32x4 c = {W.b2[t], W.b2[t], W.b2[t], W.b2[t]};
      c = mfma(A20, W.B2[0][t], c);
      c = mfma(A21, W.B2[1][t], c);
      h2[h][t] = c;
#pragma unroll
      for (int i = 0; i < 4; i++) part[i] = part[i] + W.w3[t] * to_bf16(gelu_pade(c[i]));
    }
#pragma unroll
    for (int i = 0; i < 4; i++) y[h][i] = sum16(part[i]) + W.b3;
  }
}

// Inference: y and priority of n samples (rows of X).
__global__ void __launch_bounds__(64 * kMfmaWaves) k_mlp_forward_mfma(
    const float *__restrict__ X, uint64_t n, const float *__restrict__ w, float *__restrict__ yout,
    int32_t *__restrict__ prio) {
  __shared__ __align__(16) MfmaLdsFwd lds[kMfmaWaves];
  MfmaLdsFwd &S = lds[threadIdx.x / 64];
  MfmaWeights W;
  W.load(w, false);
  const int l = (int)(threadIdx.x % 64), g = l / 16, r = l % 16;
  const uint64_t nw = (uint64_t)gridDim.x * kMfmaWaves;
  const uint64_t steps = (n + kMfmaRows - 1) / kMfmaRows;
  for (uint64_t k = (uint64_t)blockIdx.x * kMfmaWaves + threadIdx.x / 64; k < steps; k += nw) {
    const uint64_t s0 = k * kMfmaRows;
    f32x4 h1[2][4], h2[2][4];
    float y[2][4];
    mfma_forward<false>(W, S, [&](int h, int rr, float *xv) {
      const uint64_t s = s0 + 16 * h + rr;
#pragma unroll
      for (int e = 0; e < 8; e++) xv[e] = s < n ? X[s * 8 + e] : 0.0f;
    }, h1, h2, y);
    if (r == 0) {
#pragma unroll
      for (int h = 0; h < 2; h++)
#pragma unroll
        for (int i = 0; i < 4; i++) {
          const uint64_t s = s0 + 16 * h + 4 * g + i;
          if (s < n) {
            if (yout) yout[s] = y[h][i];
            if (prio) prio[s] = priority_of(y[h][i]);
          }
        }
    }
    // the next step rewrites the LDS tiles
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// Gradient sums of one wave over its 32-sample steps of the batch (samples
// idx[0 .. B-1] of X, T), written to part + wave * kMlpParams; the wave's
// sum of squared errors to lossp[wave].
__global__ void __launch_bounds__(64 * kMfmaWaves) k_mlp_grad_mfma(
    const float *__restrict__ X, const float *__restrict__ T, const uint32_t *__restrict__ idx,
    uint32_t B, const float *__restrict__ w, float *__restrict__ part,
    float *__restrict__ lossp) {
  __shared__ __align__(16) MfmaLds lds[kMfmaWaves];
  MfmaLds &S = lds[threadIdx.x / 64];
  MfmaWeights W;
  W.load(w, true);
  const int l = (int)(threadIdx.x % 64), g = l / 16, r = l % 16;
  const uint32_t wave = blockIdx.x * kMfmaWaves + threadIdx.x / 64;
  const uint32_t nw = gridDim.x * kMfmaWaves;
  const uint32_t steps = (B + kMfmaRows - 1) / kMfmaRows;
  const float inv2B = 2.0f / (float)B;
  f32x4 gW2[4][4], gW1[4];
  float gb1[4], gb2[4], gw3[4], gb3 = 0.f, sq = 0.f;
#pragma unroll
  for (int a = 0; a < 4; a++) {
    gW1[a] = f32x4{0.f, 0.f, 0.f, 0.f};
    gb1[a] = gb2[a] = gw3[a] = 0.f;
#pragma unroll
    for (int b = 0; b < 4; b++) gW2[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
  for (uint32_t k = wave; k < steps; k += nw) {
    const uint32_t s0 = k * kMfmaRows;
    f32x4 h1[2][4], h2[2][4];
    float y[2][4];
    mfma_forward<true>(W, S, [&](int h, int rr, float *xv) {
      const uint32_t b = s0 + 16 * h + rr;
      const size_t row = b < B ? (size_t)idx[b] : 0;
#pragma unroll
      for (int e = 0; e < 8; e++) xv[e] = b < B ? X[row * 8 + e] : 0.0f;
    }, h1, h2, y);
    // output layer: dy, the W3 / b3 sums and d2
    float dy[2][4];
#pragma unroll
    for (int h = 0; h < 2; h++)
#pragma unroll
      for (int i = 0; i < 4; i++) {
        const uint32_t b = s0 + 16 * h + 4 * g + i;
        const float e = b < B ? y[h][i] - T[idx[b]] : 0.0f;
        dy[h][i] = e * inv2B;
        if (r == 0) sq = sq + e * e;
        if (r == 0) gb3 = gb3 + dy[h][i];
      }
#pragma unroll
    for (int h = 0; h < 2; h++)
#pragma unroll
      for (int t = 0; t < 4; t++)
#pragma unroll
        for (int i = 0; i < 4; i++) {
          const float hv = h2[h][t][i];
          gw3[t] = gw3[t] + dy[h][i] * to_bf16(gelu_pade(hv));
          const float d2 = dy[h][i] * W.w3[t] * gelu_pade_grad(hv);
          gb2[t] = gb2[t] + d2;
          const uint16_t bits = bf16_bits(d2);
          const int s = 16 * h + 4 * g + i, n = 16 * t + r;
          S.d2_rm[s * 64 + n] = bits;
          S.d2_cm[n * kMfmaRows + s] = bits;
        }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // d1 = (d2 W2) * GELU'(h1)
#pragma unroll
    for (int h = 0; h < 2; h++) {
      const bf16x8 A0 = lds8(&S.d2_rm[(16 * h + r) * 64 + 8 * g]);
      const bf16x8 A1 = lds8(&S.d2_rm[(16 * h + r) * 64 + 32 + 8 * g]);
#pragma unroll
      for (int t = 0; t < 4; t++) {
        f32x4 c = {0.f, 0.f, 0.f, 0.f};
        c = mfma(A0, W.B2T[0][t], c);
        c = mfma(A1, W.B2T[1][t], c);
#pragma unroll
        for (int i = 0; i < 4; i++) {
          const float d1 = c[i] * gelu_pade_grad(h1[h][t][i]);
          gb1[t] = gb1[t] + d1;
          S.d1_cm[(16 * t + r) * kMfmaRows + 16 * h + 4 * g + i] = bf16_bits(d1);
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // dW2[j][i] += sum_s d2[s][j] a1[s][i]; dW1[j][k] += sum_s d1[s][j] x[s][k]
#pragma unroll
    for (int tm = 0; tm < 4; tm++) {
      const bf16x8 Ad2 = lds8(&S.d2_cm[(16 * tm + r) * kMfmaRows + 8 * g]);
#pragma unroll
      for (int tn = 0; tn < 4; tn++)
        gW2[tm][tn] = mfma(Ad2, lds8(&S.a1_cm[(16 * tn + r) * kMfmaRows + 8 * g]), gW2[tm][tn]);
      const bf16x8 Ad1 = lds8(&S.d1_cm[(16 * tm + r) * kMfmaRows + 8 * g]);
      const bf16x8 Bx = r < 8 ? lds8(&S.x_cm[r * kMfmaRows + 8 * g]) : zero8();
      gW1[tm] = mfma(Ad1, Bx, gW1[tm]);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  // the wave's sums (every slot written, zeros for a wave without steps)
  float *P = part + (size_t)wave * kMlpParams;
#pragma unroll
  for (int tm = 0; tm < 4; tm++) {
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const int j = 16 * tm + 4 * g + i;
      if (r < 8) P[j * 8 + r] = gW1[tm][i];
#pragma unroll
      for (int tn = 0; tn < 4; tn++) P[576 + j * 64 + 16 * tn + r] = gW2[tm][tn][i];
    }
  }
#pragma unroll
  for (int t = 0; t < 4; t++) {
    const float s1 = sum_groups(gb1[t]), s2 = sum_groups(gb2[t]), s3 = sum_groups(gw3[t]);
    if (g == 0) {
      P[512 + 16 * t + r] = s1;
      P[4672 + 16 * t + r] = s2;
      P[4736 + 16 * t + r] = s3;
    }
  }
  gb3 = sum_groups(gb3);  // lanes r == 0 hold the parts
  sq = sum_groups(sq);
  if (l == 0) {
    P[4800] = gb3;
    lossp[wave] = sq;
  }
}

// G[p] = sum over waves of part[w][p] in wave order; loss = sum of lossp / B.
__global__ void __launch_bounds__(256) k_mlp_grad_reduce(uint32_t nwaves, uint32_t B,
                                                          const float *__restrict__ part,
                                                          const float *__restrict__ lossp,
                                                          float *__restrict__ G,
                                                          float *__restrict__ loss) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < kMlpParams) {
    float acc = 0.f;
    for (uint32_t v = 0; v < nwaves; v++) acc = acc + part[(size_t)v * kMlpParams + p];
    G[p] = acc;
  }
  if (p == kMlpParams) {
    float acc = 0.f;
    for (uint32_t v = 0; v < nwaves; v++) acc = acc + lossp[v];
    *loss = acc / (float)B;
  }
}

}  // namespace sp
