// Host side of the learned list-length predictor (weights, training driver, predicted walk).
#pragma once

#include <cstdint>

struct fdx_ctx;

namespace fdx {

int ext_predicted_walk(fdx_ctx *c, uint32_t G);
void predictor_release(fdx_ctx *c);

}  // namespace fdx
