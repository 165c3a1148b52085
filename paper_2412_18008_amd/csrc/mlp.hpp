// mlp.hpp -- the learned priority's network (mlp.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/spoch.h"

namespace sp {

constexpr int kMlpParams = CH_MLP_PARAMS;

// P[u] for every u in va from feat[gid[u]] (8 floats) and weights w (device).
hipError_t launch_mlp_priority(const uint32_t *va, uint32_t na, const uint32_t *gid,
                               const float *feat, const float *w, int32_t *P, uint32_t qbits,
                               int cus, hipStream_t st);

int mlp_forward(const float *x, uint64_t n, const float *w, float *y, int32_t *prio,
                uint32_t flags, hipStream_t st);
int mlp_grad(const float *x, const float *t, uint32_t n, const float *w, float *grad, float *loss,
             uint32_t flags, hipStream_t st);
int mlp_train(const float *x, const float *t, uint64_t n, float *w,
              const ch_mlp_train_params_t *p, float *losses, uint32_t flags, hipStream_t st);

}  // namespace sp
