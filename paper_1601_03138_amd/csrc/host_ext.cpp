// Host extensions (predictor, autotuner, queue order, graph capture).
#include "ctx.h"

namespace fdx {

int ext_predicted_walk(fdx_ctx *c, uint32_t) {
    return fail(c, FDX_EINVAL, "FDX_PREDICTOR: no predictor loaded");
}

int ext_force_variant(fdx_ctx *c) {
    if (c->n_group > 256) return 1;
    return c->ext.variant >= 0 ? c->ext.variant : 0;
}

const uint32_t *ext_queue_order(fdx_ctx *, uint32_t) { return nullptr; }

int ext_integrate_graph(fdx_ctx *c, double, int) {
    return fail(c, FDX_EINVAL, "FDX_GRAPH not available");
}

void ext_release(fdx_ctx *) {}

}  // namespace fdx
