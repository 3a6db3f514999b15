// FP64 direct summation for selected target particles: the exact quantity the tree
// approximates (equation ParticleParticleNbody of section "An example -- gravitational N-body
// problem", G = 1), used as the reference for the error of the tree forces.
//   a_i   =  sum_{j != i} m_j (x_j - x_i) / (|x_j - x_i|^2 + eps_i^2)^{3/2}
//   phi_i = -sum_{j != i} m_j / (|x_j - x_i|^2 + eps_i^2)^{1/2}
// over the particles j of i's system.  One workgroup per target: every thread sums a strided
// share of the sources with Neumaier compensation, then one thread combines the 256 partial
// sums in thread order, so the result is deterministic.
#include "dev_util.h"
#include "fdx_internal.h"

namespace fdx {

namespace {

constexpr int kThreads = 256;

struct Comp {
    double s = 0.0, c = 0.0;
    __device__ __forceinline__ void add(double v) {
        const double t = s + v;
        c += fabs(s) >= fabs(v) ? (s - t) + v : (v - t) + s;
        s = t;
    }
};

__global__ void __launch_bounds__(kThreads)
k_direct(uint32_t nt, const uint32_t *targets, const double *x, const double *y,
         const double *z, const double *m, const double *eps, double eps_all,
         const uint32_t *sysid, const int64_t *sys_off, double *out) {
    __shared__ double part[8][kThreads];
    const uint32_t b = blockIdx.x;
    if (b >= nt) return;
    const uint32_t i = targets[b];
    const uint32_t s = sysid[i];
    const size_t j0 = (size_t)sys_off[s], j1 = (size_t)sys_off[s + 1];
    const double xi = x[i], yi = y[i], zi = z[i];
    const double ei = eps ? eps[i] : eps_all;
    const double e2 = ei * ei;
    Comp ax, ay, az, ph;
    for (size_t j = j0 + threadIdx.x; j < j1; j += kThreads) {
        if (j == i) continue;
        const double dx = x[j] - xi, dy = y[j] - yi, dz = z[j] - zi;
        const double r2 = dx * dx + dy * dy + dz * dz + e2;
        const double rinv = 1.0 / sqrt(r2);
        const double mr = m[j] * rinv;
        const double f = mr * rinv * rinv;
        ax.add(f * dx);
        ay.add(f * dy);
        az.add(f * dz);
        ph.add(-mr);
    }
    const int t = threadIdx.x;
    part[0][t] = ax.s; part[1][t] = ax.c;
    part[2][t] = ay.s; part[3][t] = ay.c;
    part[4][t] = az.s; part[5][t] = az.c;
    part[6][t] = ph.s; part[7][t] = ph.c;
    __syncthreads();
    if (t < 4) {
        Comp tot;
        for (int q = 0; q < kThreads; q++) {
            tot.add(part[2 * t][q]);
            tot.add(part[2 * t + 1][q]);
        }
        out[4 * (size_t)b + t] = tot.s + tot.c;
    }
}

}  // namespace

hipError_t direct_forces(uint32_t nt, const uint32_t *targets, const double *x, const double *y,
                         const double *z, const double *m, const double *eps, double eps_all,
                         const uint32_t *sysid, const int64_t *sys_off, double *out,
                         hipStream_t s) {
    if (nt == 0) return hipSuccess;
    hipLaunchKernelGGL(k_direct, dim3(nt), dim3(kThreads), 0, s, nt, targets, x, y, z, m, eps,
                       eps_all, sysid, sys_off, out);
    return hipGetLastError();
}

}  // namespace fdx
