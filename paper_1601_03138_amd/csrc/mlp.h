// Learned list-length predictor: sizes and device entry points (see k_mlp.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "fdx_internal.h"

namespace fdx {

constexpr int kMlpIn = 8;
constexpr int kMlpHidden = 64;
constexpr int kMlpParams = kMlpIn * kMlpHidden + kMlpHidden + kMlpHidden * kMlpHidden +
                           kMlpHidden + kMlpHidden + 1;   // 4801

hipError_t mlp_features(size_t gmax, const Groups g, const Cells c, const int64_t *sys_off,
                        const float *mu, const float *sd, float *X, DevStatus *st, hipStream_t s);
// y[i] = MLP(X[i]) for i < n (or < *n_dev when given)
hipError_t mlp_infer(size_t n, const uint32_t *n_dev, const float *X, const float *P, float *y,
                     hipStream_t s);
size_t mlp_train_blocks(size_t batch);
// gradient of mean((MLP(X[idx[k]]) - T[idx[k]])^2) over k < batch; gpart/lpart hold
// mlp_train_blocks(batch) partial rows
hipError_t mlp_grad(size_t batch, const uint32_t *idx, const float *X, const float *T,
                    const float *P, float *gpart, float *lpart, float *grad, float *loss,
                    hipStream_t s);
hipError_t mlp_adam(float *P, const float *grad, float *m, float *v, int step, float lr,
                    hipStream_t s);
hipError_t pred_caps(size_t gmax, const float *y, float margin, uint32_t cap_max, uint32_t *cap,
                     DevStatus *st, hipStream_t s);
hipError_t ovf_caps(size_t gmax, const uint32_t *nsel, const uint32_t *sel, const uint32_t *cnt_e,
                    const uint32_t *cnt_s, uint32_t *ocap, hipStream_t s);
hipError_t ovf_seg(size_t gmax, const uint32_t *nsel, const uint32_t *sel, const uint32_t *ocap,
                   const uint64_t *ooff, const uint64_t *base_total, uint64_t *seg, uint32_t *cap,
                   hipStream_t s);

}  // namespace fdx
