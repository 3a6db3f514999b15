// FP64 direct summation for selected target particles (the reference for the error of the
// tree forces; equation ParticleParticleNbody, G = 1).
#include <cmath>
#include <vector>

#include "ctx.h"

using namespace fdx;

extern "C" {

int fdx_direct_forces(fdx_ctx *c, const int64_t *targets, int64_t n_targets, double eps,
                      double *out) {
    FDX_ABI_TRY
    if (!c) return FDX_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, FDX_EHIP, "hipSetDevice failed");
    if (!c->have_particles) return fail(c, FDX_ESTATE, "no particles: call fdx_set_particles first");
    if (n_targets < 0 || n_targets > (1ll << 24))
        return fail(c, FDX_EINVAL, "n_targets must be in [0, 2^24]");
    if (n_targets > 0 && (!targets || !out)) return fail(c, FDX_EINVAL, "null targets or output");
    if (!c->eps_given && !(std::isfinite(eps) && eps > 0.0))
        return fail(c, FDX_EINVAL, "eps must be finite and > 0");
    std::vector<uint32_t> t((size_t)n_targets);
    for (int64_t k = 0; k < n_targets; k++) {
        if (targets[k] < 0 || targets[k] >= c->n)
            return fail(c, FDX_EINVAL, "target index %lld out of range", (long long)targets[k]);
        t[k] = (uint32_t)targets[k];
    }
    if (n_targets == 0) return FDX_OK;
    hipStream_t s = c->stream;
    uint32_t *dt = nullptr;
    double *dout = nullptr;
    hipError_t e = hipMalloc((void **)&dt, 4 * (size_t)n_targets);
    if (e == hipSuccess) e = hipMalloc((void **)&dout, 32 * (size_t)n_targets);
    if (e == hipSuccess) e = hipMemcpyAsync(dt, t.data(), 4 * (size_t)n_targets,
                                            hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = direct_forces((uint32_t)n_targets, dt, c->x, c->y, c->z, c->m,
                          c->eps_given ? c->eps : nullptr, eps, c->sysid.p, c->sys_off.p, dout, s);
    if (e == hipSuccess) e = hipMemcpyAsync(out, dout, 32 * (size_t)n_targets,
                                            hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipStreamSynchronize(s);
    if (dt) (void)hipFree(dt);
    if (dout) (void)hipFree(dout);
    if (e != hipSuccess)
        return fail(c, e == hipErrorOutOfMemory ? FDX_ENOMEM : FDX_EHIP, "direct forces: %s",
                    hipGetErrorString(e));
    return FDX_OK;
    FDX_ABI_CATCH(c)
}

}  // extern "C"
