// Host-side extensions of the force path: learned list-length predictor, force-kernel
// autotuner and HIP-graph capture of leapfrog steps.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

struct fdx_ctx;

namespace fdx {

struct HostExt {
    int variant[2] = {-1, -1};        // autotuned force-kernel variant, [FP64, FP32] (-1: default)
    void *pred = nullptr;             // predictor state (weights, normalisation)
    void *graph = nullptr;            // captured step (GraphState)
    void *exch = nullptr;             // exchange lists between domains
    void *sph = nullptr;              // SPH density state
    void *dd = nullptr;               // domain decomposition state
    int64_t graph_recoveries = 0;     // replays whose capacities overflowed and were redone
    uint32_t graph_margin_pct = 200;  // graph list segments: percent of each system's longest
    int64_t list_spills = 0;          // lists moved to the spill space by a fill walk
};

int ext_force_variant(fdx_ctx *c);
int ext_integrate_graph(fdx_ctx *c, double dt, int n_steps);
void ext_release(fdx_ctx *c);
void ext_invalidate(fdx_ctx *c);   // drop any captured graph (particles or buffers changed)
int ext_predicted_walk(fdx_ctx *c, uint32_t G);
// predicted ln list length of every group (features + network on the device, no host wait)
int ext_predicted_lengths(fdx_ctx *c, size_t gmax, const float **y);
// device buffers of ext_predicted_lengths for the current group capacity (before a capture)
int ext_predictor_reserve(fdx_ctx *c);
void exchange_release(fdx_ctx *c);
void sph_release(fdx_ctx *c);
void dd_release(fdx_ctx *c);

}  // namespace fdx
