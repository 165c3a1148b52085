// mlp.hip -- the learned priority's network on gfx950: an MLP 8 -> 64 -> 64
// -> 1 with GELU, its use inside the build (features -> int32 priority), a
// standalone forward (fp32, or bf16 on the matrix cores: mlp_mfma.hpp), and
// deterministic training kernels (MSE, Adam; fp32 per sample, or bf16 on the
// matrix cores).
//
// GELU(x) = x/2 * (1 + T(0.7978845608 * (x + 0.044715 x^3))) with T the [7/6]
// Pade approximant of tanh (Lambert's continued fraction), +-1 for
// |t| >= 4.97.  Inference is single precision, evaluated in a fixed order
// with fused multiply-add disabled (this file is compiled with
// -ffp-contract=off), and IEEE division is correctly rounded, so the
// priority bits are those of any IEEE implementation of the same formula.
// Weights: W1[64][8], b1[64], W2[64][64], b2[64], W3[64], b3 (4801 floats).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "builder.hpp"
#include "common.hpp"
#include "mlp.hpp"

#pragma clang fp contract(off)

namespace sp {

__device__ __forceinline__ float tanh_pade(float t) {
  if (t >= 4.97f) return 1.0f;
  if (t <= -4.97f) return -1.0f;
  const float t2 = t * t;
  const float num = t * (135135.0f + t2 * (17325.0f + t2 * (378.0f + t2)));
  const float den = 135135.0f + t2 * (62370.0f + t2 * (3150.0f + t2 * 28.0f));
  float r = num / den;
  r = r > 1.0f ? 1.0f : r;
  r = r < -1.0f ? -1.0f : r;
  return r;
}

__device__ __forceinline__ float gelu_pade(float x) {
  const float x3 = (x * x) * x;
  const float inner = x + 0.044715f * x3;
  const float t = 0.7978845608f * inner;
  return (0.5f * x) * (1.0f + tanh_pade(t));
}

// Exact derivative of gelu_pade (zero where T is clamped).
__device__ __forceinline__ float gelu_pade_grad(float x) {
  const float t = 0.7978845608f * (x + 0.044715f * ((x * x) * x));
  float dt = 0.0f;
  if (t < 4.97f && t > -4.97f) {
    const float t2 = t * t;
    const float num = t * (135135.0f + t2 * (17325.0f + t2 * (378.0f + t2)));
    const float den = 135135.0f + t2 * (62370.0f + t2 * (3150.0f + t2 * 28.0f));
    const float dnum = 135135.0f + t2 * (51975.0f + t2 * (1890.0f + 7.0f * t2));
    const float dden = t * (124740.0f + t2 * (12600.0f + 168.0f * t2));
    if (fabsf(num / den) <= 1.0f) dt = (dnum * den - num * dden) / (den * den);
  }
  return 0.5f * (1.0f + tanh_pade(t)) +
         0.5f * x * dt * 0.7978845608f * (1.0f + 3.0f * 0.044715f * x * x);
}

// bf16 rounding (round to nearest even), kept in a float.
__device__ __forceinline__ float to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return f;  // inf / nan unchanged
  u += 0x7fffu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xffff0000u);
}

// Input unit i of layer 2 is produced and consumed at once: h2[j] gets its
// terms in the order i = 0..63 for every j, the same sums as the row-by-row
// evaluation, with the 64 accumulators in registers.
template <bool BF16>
__device__ __forceinline__ float mlp_forward(const float *__restrict__ w, const float *x) {
  const float *W1 = w, *b1 = w + 512, *W2 = w + 576, *b2 = w + 4672, *W3 = w + 4736;
  float h2[64];
#pragma unroll
  for (int j = 0; j < 64; j++) h2[j] = b2[j];
  for (int i = 0; i < 64; i++) {
    float h = b1[i];
#pragma unroll
    for (int k = 0; k < 8; k++) h = h + W1[i * 8 + k] * x[k];
    const float a1 = BF16 ? to_bf16(gelu_pade(h)) : gelu_pade(h);
#pragma unroll
    for (int j = 0; j < 64; j++) h2[j] = h2[j] + W2[j * 64 + i] * a1;
  }
  float y = w[4800];
#pragma unroll
  for (int j = 0; j < 64; j++) {
    const float a2 = BF16 ? to_bf16(gelu_pade(h2[j])) : gelu_pade(h2[j]);
    y = y + W3[j] * a2;
  }
  return y;
}

// rint(y * scale), saturated; scale = 2^qbits (exact).
__device__ __forceinline__ int32_t priority_of(float y, float scale = 65536.0f) {
  const float z = y * scale;
  if (!(z < 2147483648.0f)) return INT32_MAX;  // also NaN
  if (z < -2147483648.0f) return INT32_MIN;
  return (int32_t)rintf(z);
}

}  // namespace sp

#include "mlp_mfma.hpp"

namespace sp {

// Weights staged in LDS by every block (4801 floats).
__device__ __forceinline__ void stage_weights(const float *__restrict__ w, float *s, bool bf16) {
  for (int i = threadIdx.x; i < kMlpParams; i += blockDim.x) s[i] = bf16 ? to_bf16(w[i]) : w[i];
  __syncthreads();
}

// Priority of every affected vertex from its current features.
__global__ void __launch_bounds__(256) k_mlp_priority(const uint32_t *__restrict__ va, uint32_t na,
                                                      const uint32_t *__restrict__ gid,
                                                      const float *__restrict__ feat,
                                                      const float *__restrict__ w,
                                                      int32_t *__restrict__ P, float scale) {
  __shared__ float sw[kMlpParams];
  stage_weights(w, sw, false);
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < na; k += stride) {
    const uint32_t u = va[k];
    const float *f = feat + (size_t)gid[u] * 8;
    float x[8];
    for (int i = 0; i < 8; i++) x[i] = f[i];
    P[u] = priority_of(mlp_forward<false>(sw, x), scale);
  }
}

template <bool BF16>
__global__ void __launch_bounds__(256) k_mlp_forward(const float *__restrict__ X, uint64_t n,
                                                     const float *__restrict__ w,
                                                     float *__restrict__ y,
                                                     int32_t *__restrict__ prio) {
  __shared__ float sw[kMlpParams];
  stage_weights(w, sw, BF16);
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
    float x[8];
    for (int i = 0; i < 8; i++) x[i] = BF16 ? to_bf16(X[k * 8 + i]) : X[k * 8 + i];
    const float v = mlp_forward<BF16>(sw, x);
    if (y) y[k] = v;
    if (prio) prio[k] = priority_of(v);
  }
}

// ---------------------------------------------------------------------------
// training: per-sample forward and backward (intermediates to scratch), then
// one thread per parameter sums over the batch in sample order, then Adam.
// ---------------------------------------------------------------------------
struct TrainScratch {
  float *xb;  // [B][8]
  float *h1, *a1, *h2, *a2, *d1, *d2;  // [B][64]
  float *dy, *err;  // [B]
};

__global__ void k_batch_index(uint64_t n, uint32_t B, uint64_t seed, uint64_t step,
                              uint32_t *__restrict__ idx, int full) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t b = blockIdx.x * blockDim.x + threadIdx.x; b < B; b += stride)
    idx[b] = full ? b : (uint32_t)(mix64(seed ^ (0x9E3779B97F4A7C15ull * (step * B + b + 1))) % n);
}

__global__ void __launch_bounds__(256) k_mlp_fwdbwd(const float *__restrict__ X,
                                                    const float *__restrict__ T,
                                                    const uint32_t *__restrict__ idx, uint32_t B,
                                                    const float *__restrict__ w, TrainScratch s) {
  const float *W1 = w, *b1 = w + 512, *W2 = w + 576, *b2 = w + 4672, *W3 = w + 4736;
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t b = blockIdx.x * blockDim.x + threadIdx.x; b < B; b += stride) {
    const uint32_t r = idx[b];
    float x[8];
    for (int i = 0; i < 8; i++) {
      x[i] = X[(size_t)r * 8 + i];
      s.xb[(size_t)b * 8 + i] = x[i];
    }
    float *h1 = s.h1 + (size_t)b * 64, *a1 = s.a1 + (size_t)b * 64;
    float *h2 = s.h2 + (size_t)b * 64, *a2 = s.a2 + (size_t)b * 64;
    float *d1 = s.d1 + (size_t)b * 64, *d2 = s.d2 + (size_t)b * 64;
    for (int j = 0; j < 64; j++) {
      float h = b1[j];
      for (int i = 0; i < 8; i++) h = h + W1[j * 8 + i] * x[i];
      h1[j] = h;
      a1[j] = gelu_pade(h);
    }
    float y = w[4800];
    for (int j = 0; j < 64; j++) {
      float h = b2[j];
      for (int i = 0; i < 64; i++) h = h + W2[j * 64 + i] * a1[i];
      h2[j] = h;
      a2[j] = gelu_pade(h);
      y = y + W3[j] * a2[j];
    }
    const float e = y - T[r];
    const float dy = 2.0f * e / (float)B;
    s.dy[b] = dy;
    s.err[b] = e;
    for (int j = 0; j < 64; j++) d2[j] = dy * W3[j] * gelu_pade_grad(h2[j]);
    for (int i = 0; i < 64; i++) {
      float acc = 0.0f;
      for (int j = 0; j < 64; j++) acc = acc + d2[j] * W2[j * 64 + i];
      d1[i] = acc * gelu_pade_grad(h1[i]);
    }
  }
}

// One thread per parameter; sums over the batch in sample order.
__global__ void __launch_bounds__(256) k_mlp_param_grad(uint32_t B, TrainScratch s,
                                                        float *__restrict__ g) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kMlpParams) return;
  float acc = 0.0f;
  if (p < 512) {  // W1[j][i]
    const uint32_t j = p / 8, i = p % 8;
    for (uint32_t b = 0; b < B; b++) acc = acc + s.d1[(size_t)b * 64 + j] * s.xb[(size_t)b * 8 + i];
  } else if (p < 576) {  // b1[j]
    const uint32_t j = p - 512;
    for (uint32_t b = 0; b < B; b++) acc = acc + s.d1[(size_t)b * 64 + j];
  } else if (p < 4672) {  // W2[j][i]
    const uint32_t q = p - 576, j = q / 64, i = q % 64;
    for (uint32_t b = 0; b < B; b++) acc = acc + s.d2[(size_t)b * 64 + j] * s.a1[(size_t)b * 64 + i];
  } else if (p < 4736) {  // b2[j]
    const uint32_t j = p - 4672;
    for (uint32_t b = 0; b < B; b++) acc = acc + s.d2[(size_t)b * 64 + j];
  } else if (p < 4800) {  // W3[i]
    const uint32_t i = p - 4736;
    for (uint32_t b = 0; b < B; b++) acc = acc + s.dy[b] * s.a2[(size_t)b * 64 + i];
  } else {  // b3
    for (uint32_t b = 0; b < B; b++) acc = acc + s.dy[b];
  }
  g[p] = acc;
}

// Mean squared error of the batch (one thread, sample order).
__global__ void k_batch_loss(uint32_t B, const float *__restrict__ err, float *__restrict__ out) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    float acc = 0.0f;
    for (uint32_t b = 0; b < B; b++) acc = acc + err[b] * err[b];
    *out = acc / (float)B;
  }
}

__global__ void k_adam(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kMlpParams) return;
  const float gp = g[p];
  const float mp = b1 * m[p] + (1.0f - b1) * gp;
  const float vp = b2 * v[p] + (1.0f - b2) * gp * gp;
  m[p] = mp;
  v[p] = vp;
  w[p] = w[p] - lr * (mp / c1) / (sqrtf(vp / c2) + eps);
}

// ---------------------------------------------------------------------------
// host wrappers
// ---------------------------------------------------------------------------
#define HIP_TRY(expr)                                   \
  do {                                                  \
    hipError_t e_ = (expr);                             \
    if (e_ != hipSuccess) return hip_error(e_, #expr);  \
  } while (0)

hipError_t launch_mlp_priority(const uint32_t *va, uint32_t na, const uint32_t *gid,
                               const float *feat, const float *w, int32_t *P, uint32_t qbits,
                               int cus, hipStream_t st) {
  if (!na) return hipSuccess;
  const unsigned g = (unsigned)std::min<uint64_t>((na + 255) / 256, (uint64_t)cus * 4);
  k_mlp_priority<<<g, 256, 0, st>>>(va, na, gid, feat, w, P, (float)(1u << qbits));
  return hipGetLastError();
}

static unsigned blocks_for(uint64_t n) {
  return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((n + 255) / 256, 4096));
}

int mlp_forward(const float *x, uint64_t n, const float *w, float *y, int32_t *prio,
                uint32_t flags, hipStream_t st) {
  const bool dev = flags & CH_MLP_ON_DEVICE, bf16 = flags & CH_MLP_BF16;
  if (!n) return CH_OK;
  DBuf dx, dw, dy, dp;
  const float *px = x;
  float *py = y;
  int32_t *pp = prio;
  HIP_TRY(dw.ensure(kMlpParams * 4));
  HIP_TRY(hipMemcpyAsync(dw.p, w, kMlpParams * 4, dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
  if (!dev) {
    HIP_TRY(dx.ensure(n * 32));
    HIP_TRY(hipMemcpyAsync(dx.p, x, n * 32, hipMemcpyHostToDevice, st));
    px = dx.as<float>();
    if (y) {
      HIP_TRY(dy.ensure(n * 4));
      py = dy.as<float>();
    }
    if (prio) {
      HIP_TRY(dp.ensure(n * 4));
      pp = dp.as<int32_t>();
    }
  }
  if (bf16) {
    const uint64_t steps = (n + kMfmaRows - 1) / kMfmaRows;
    const unsigned g = (unsigned)std::max<uint64_t>(
        1, std::min<uint64_t>((steps + kMfmaWaves - 1) / kMfmaWaves, 2048));
    k_mlp_forward_mfma<<<g, 64 * kMfmaWaves, 0, st>>>(px, n, dw.as<float>(), py, pp);
  } else {
    k_mlp_forward<false><<<blocks_for(n), 256, 0, st>>>(px, n, dw.as<float>(), py, pp);
  }
  HIP_TRY(hipGetLastError());
  if (!dev) {
    if (y) HIP_TRY(hipMemcpyAsync(y, py, n * 4, hipMemcpyDeviceToHost, st));
    if (prio) HIP_TRY(hipMemcpyAsync(prio, pp, n * 4, hipMemcpyDeviceToHost, st));
  }
  HIP_TRY(hipStreamSynchronize(st));
  DBuf *all[] = {&dx, &dw, &dy, &dp};
  for (DBuf *b : all) b->release();
  return CH_OK;
}

// Shared by mlp_grad and mlp_train: device copies of the data and scratch.
struct TrainCtx {
  DBuf X, T, W, G, M, V, idx, loss, xb, h1, a1, h2, a2, d1, d2, dy, err, part, lossp;
  TrainScratch s{};
  bool bf16 = false;
  uint32_t mblocks = 0;  // blocks of the bf16 gradient kernel
  ~TrainCtx() {
    DBuf *all[] = {&X, &T, &W, &G, &M, &V, &idx, &loss, &xb, &h1, &a1, &h2, &a2, &d1, &d2, &dy,
                   &err, &part, &lossp};
    for (DBuf *b : all) b->release();
  }
  int setup(const float *x, const float *t, uint64_t n, const float *w, uint32_t B, bool dev,
            hipStream_t st) {
    const hipMemcpyKind k = dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    HIP_TRY(X.ensure(n * 32));
    HIP_TRY(T.ensure(n * 4));
    HIP_TRY(hipMemcpyAsync(X.p, x, n * 32, k, st));
    HIP_TRY(hipMemcpyAsync(T.p, t, n * 4, k, st));
    HIP_TRY(W.ensure(kMlpParams * 4));
    HIP_TRY(hipMemcpyAsync(W.p, w, kMlpParams * 4, hipMemcpyHostToDevice, st));
    DBuf *p[] = {&G, &M, &V};
    for (DBuf *b : p) HIP_TRY(b->ensure(kMlpParams * 4));
    HIP_TRY(hipMemsetAsync(M.p, 0, kMlpParams * 4, st));
    HIP_TRY(hipMemsetAsync(V.p, 0, kMlpParams * 4, st));
    HIP_TRY(idx.ensure((size_t)B * 4));
    HIP_TRY(loss.ensure(4));
    if (bf16) {  // per-wave gradient sums instead of per-sample scratch
      const uint32_t steps = (B + kMfmaRows - 1) / kMfmaRows;
      mblocks = std::max<uint32_t>(1, std::min<uint32_t>((steps + kMfmaWaves - 1) / kMfmaWaves, 256));
      HIP_TRY(part.ensure((size_t)mblocks * kMfmaWaves * kMlpParams * 4));
      HIP_TRY(lossp.ensure((size_t)mblocks * kMfmaWaves * 4));
      return CH_OK;
    }
    HIP_TRY(xb.ensure((size_t)B * 32));
    DBuf *q[] = {&h1, &a1, &h2, &a2, &d1, &d2};
    for (DBuf *b : q) HIP_TRY(b->ensure((size_t)B * 256));
    HIP_TRY(dy.ensure((size_t)B * 4));
    HIP_TRY(err.ensure((size_t)B * 4));
    s = TrainScratch{xb.as<float>(), h1.as<float>(), a1.as<float>(), h2.as<float>(),
                     a2.as<float>(), d1.as<float>(), d2.as<float>(), dy.as<float>(),
                     err.as<float>()};
    return CH_OK;
  }
  hipError_t batch_grad(uint64_t n, uint32_t B, uint64_t seed, uint64_t step, bool full,
                        hipStream_t st) {
    k_batch_index<<<blocks_for(B), 256, 0, st>>>(n, B, seed, step, idx.as<uint32_t>(), full);
    if (bf16) {
      k_mlp_grad_mfma<<<mblocks, 64 * kMfmaWaves, 0, st>>>(X.as<float>(), T.as<float>(),
                                                            idx.as<uint32_t>(), B, W.as<float>(),
                                                            part.as<float>(), lossp.as<float>());
      k_mlp_grad_reduce<<<(kMlpParams + 256) / 256, 256, 0, st>>>(
          mblocks * kMfmaWaves, B, part.as<float>(), lossp.as<float>(), G.as<float>(),
          loss.as<float>());
      return hipGetLastError();
    }
    k_mlp_fwdbwd<<<blocks_for(B), 256, 0, st>>>(X.as<float>(), T.as<float>(), idx.as<uint32_t>(),
                                                  B, W.as<float>(), s);
    k_mlp_param_grad<<<(kMlpParams + 255) / 256, 256, 0, st>>>(B, s, G.as<float>());
    k_batch_loss<<<1, 64, 0, st>>>(B, err.as<float>(), loss.as<float>());
    return hipGetLastError();
  }
};

int mlp_grad(const float *x, const float *t, uint32_t n, const float *w, float *grad, float *loss,
             uint32_t flags, hipStream_t st) {
  if (!n) return set_error(CH_E_INVALID, "n must be positive");
  TrainCtx c;
  c.bf16 = flags & CH_MLP_BF16;
  int rc = c.setup(x, t, n, w, n, flags & CH_MLP_ON_DEVICE, st);
  if (rc) return rc;
  HIP_TRY(c.batch_grad(n, n, 0, 0, true, st));
  HIP_TRY(hipMemcpyAsync(grad, c.G.p, kMlpParams * 4, hipMemcpyDeviceToHost, st));
  if (loss) HIP_TRY(hipMemcpyAsync(loss, c.loss.p, 4, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return CH_OK;
}

int mlp_train(const float *x, const float *t, uint64_t n, float *w,
              const ch_mlp_train_params_t *p, float *losses, uint32_t flags, hipStream_t st) {
  if (!n || !p || !p->batch || p->batch > (1u << 20))
    return set_error(CH_E_INVALID, "need n > 0 and 0 < batch <= 2^20");
  TrainCtx c;
  c.bf16 = flags & CH_MLP_BF16;
  int rc = c.setup(x, t, n, w, p->batch, flags & CH_MLP_ON_DEVICE, st);
  if (rc) return rc;
  double c1 = 1.0, c2 = 1.0;
  for (uint32_t k = 0; k < p->steps; k++) {
    HIP_TRY(c.batch_grad(n, p->batch, p->seed, k, false, st));
    c1 *= p->beta1;
    c2 *= p->beta2;
    k_adam<<<(kMlpParams + 255) / 256, 256, 0, st>>>(c.W.as<float>(), c.G.as<float>(),
                                                     c.M.as<float>(), c.V.as<float>(), p->lr,
                                                     p->beta1, p->beta2, p->eps, (float)(1.0 - c1),
                                                     (float)(1.0 - c2));
    HIP_TRY(hipGetLastError());
    if (losses) HIP_TRY(hipMemcpyAsync(losses + k, c.loss.p, 4, hipMemcpyDeviceToHost, st));
  }
  HIP_TRY(hipMemcpyAsync(w, c.W.p, kMlpParams * 4, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return CH_OK;
}

}  // namespace sp
