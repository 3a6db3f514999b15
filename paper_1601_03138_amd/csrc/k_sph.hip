// Short-range interaction on the tree: SPH density from candidate neighbour lists.
//
// The same tree is traversed for short-range interactions with four kinds of cutoff
// (section "Interaction calculation"): fixed, j-dependent ("scatter", r < h_j), i-dependent
// ("gather", r < h_i) and symmetric (r < max(h_i, h_j)).  The walk (k_walk.hip) gives each
// group the particles of every leaf within reach; this file gives the walk its radii (the
// largest h of every cell, bottom-up, and of every group) and evaluates, per i-particle,
//   rho_i = sum_j m_j W(|r_ij|, H) over pairs with |r_ij| < H (j = i included),
//   H = r_cut (fixed), h_j (scatter), h_i (gather); symmetric: the mean of the gather and
//   scatter sums; n_i = number of such j (symmetric: |r_ij| < max(h_i, h_j)),
// with the Wendland C6 kernel of the paper's SPH application (section "Giant impact
// simulation"; Dehnen & Aly 2012), q = r / H < 1:
//   W(r, H) = 1365 / (64 pi H^3) (1 - q)^8 (1 + 8 q + 25 q^2 + 32 q^3).
// |r_ij|^2 = dx*dx + dy*dy + dz*dz is rounded as written (no contraction) and compared with
// H*H, so which pairs count is exact.  FP64 throughout; one workgroup per group, candidate
// tiles staged in LDS, per-slice partial sums combined in slice order (deterministic).
#include "dev_util.h"
#include "fdx_internal.h"

namespace fdx {

namespace {

constexpr int kThreads = 256;
constexpr double kWendlandC6 = 1365.0 / (64.0 * 3.14159265358979323846);

inline unsigned grid_for(size_t n, unsigned cap = 8192) {
    size_t b = (n + kThreads - 1) / kThreads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

// support radius of every particle in sorted order (h given) or the fixed cutoff
__global__ void k_sph_radius(size_t n, const uint32_t *perm, const double *h, double r_fixed,
                             double *sh, DevStatus *st) {
    for (size_t r = gtid(); r < n; r += gstride()) {
        const double v = h ? h[perm[r]] : r_fixed;
        if (!(v > 0.0) || !isfinite(v)) atomicOr(&st->bad_input, 1u);
        sh[r] = v;
    }
}

// largest support radius in every cell of level l (children done first)
__global__ void k_cell_hmax(int l, Cells c, const double *sh, double *hmax) {
    const uint32_t c0 = c.lvl[l], c1 = c.lvl[l + 1];
    for (size_t k = gtid(); k < c1 - c0; k += gstride()) {
        const uint32_t cid = c0 + (uint32_t)k;
        double v = 0.0;
        const uint32_t nch = c.nchild[cid];
        if (nch == 0) {
            const uint32_t b = c.begin[cid], e = b + c.count[cid];
            for (uint32_t i = b; i < e; i++) v = fmax(v, sh[i]);
        } else {
            const uint32_t f = c.first[cid];
            for (uint32_t j = f; j < f + nch; j++) v = fmax(v, hmax[j]);
        }
        hmax[cid] = v;
    }
}

// largest support radius of every group (one wave per group)
__global__ void __launch_bounds__(kThreads)
k_group_hmax(const uint32_t *ngroups, Groups g, const double *sh, double *rg) {
    const uint32_t G = min(*ngroups, g.cap);
    const int lane = lane_id();
    const size_t wave0 = gtid() / kWave, nwaves = gstride() / kWave;
    for (size_t gi = wave0; gi < G; gi += nwaves) {
        const uint32_t b = g.begin[gi], e = b + g.count[gi];
        double v = 0.0;
        for (uint32_t r = b + lane; r < e; r += kWave) v = fmax(v, sh[r]);
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) v = fmax(v, __shfl_xor(v, d, kWave));
        if (lane == 0) rg[gi] = v;
    }
}

// |r|^2 rounded as written, ((dx dx + dy dy) + dz dz), with no fused multiply-add, so the
// comparison with H^2 decides exactly as the plain definition does
__device__ __forceinline__ double dist2_as_written(double dx, double dy, double dz) {
#pragma clang fp contract(off)
    return (dx * dx + dy * dy) + dz * dz;
}

__device__ __forceinline__ double wendland(double r2, double invh, double norm) {
    const double q = __dmul_rn(sqrt(r2), invh);
    const double u = 1.0 - q, u2 = u * u, u4 = u2 * u2, u8 = u4 * u4;
    return norm * u8 * fma(q, fma(q, fma(q, 32.0, 25.0), 8.0), 1.0);
}

struct DensArgs {
    const uint32_t *ngroups;
    const uint32_t *gbegin, *gcount;
    const uint64_t *seg;
    const uint32_t *cnt_e, *list;
    const double4 *jp;
    const double *sh;
    double *rho;
    uint32_t *nngb;
};

template <int MODE>   // 0 fixed, 1 scatter, 2 gather, 3 symmetric
__global__ void __launch_bounds__(kThreads) k_density(DensArgs a) {
    __shared__ double4 tj[kThreads];
    __shared__ double th[kThreads], tinv[kThreads], tnorm[kThreads];
    __shared__ double red[kThreads];
    __shared__ uint32_t redn[kThreads];
    const uint32_t G = *a.ngroups;
    const int tid = threadIdx.x;
    for (uint32_t gi = blockIdx.x; gi < G; gi += gridDim.x) {
        const uint32_t gb = a.gbegin[gi], ni = a.gcount[gi], ne = a.cnt_e[gi];
        const uint32_t *cand = a.list + a.seg[gi];
        for (uint32_t i0 = 0; i0 < ni; i0 += kThreads) {
            const uint32_t tps = min((uint32_t)kThreads, ni - i0);
            const uint32_t nslice = kThreads / tps;
            const uint32_t slice = tid / tps, li = tid % tps;
            const bool active = slice < nslice;
            const uint32_t i = gb + i0 + li;
            const double4 pi = a.jp[active ? i : gb];
            const double hi = a.sh[active ? i : gb];
            const double hi2 = __dmul_rn(hi, hi), invhi = 1.0 / hi;
            const double normi = kWendlandC6 * invhi * invhi * invhi;
            double acc = 0.0;
            uint32_t cnt = 0;
            for (uint32_t t0 = 0; t0 < ne; t0 += kThreads) {
                const uint32_t nt = min((uint32_t)kThreads, ne - t0);
                __syncthreads();
                if ((uint32_t)tid < nt) {
                    const uint32_t j = cand[t0 + tid];
                    const double hj = a.sh[j];
                    tj[tid] = a.jp[j];
                    th[tid] = hj;
                    tinv[tid] = 1.0 / hj;
                    tnorm[tid] = kWendlandC6 / (hj * hj * hj);
                }
                __syncthreads();
                if (active) {
                    for (uint32_t jj = slice; jj < nt; jj += nslice) {
                        const double4 pj = tj[jj];
                        const double dx = __dsub_rn(pj.x, pi.x), dy = __dsub_rn(pj.y, pi.y),
                                     dz = __dsub_rn(pj.z, pi.z);
                        const double r2 = dist2_as_written(dx, dy, dz);
                        if (MODE == 0 || MODE == 2) {
                            if (r2 < hi2) { acc += pj.w * wendland(r2, invhi, normi); cnt++; }
                        } else if (MODE == 1) {
                            const double hj = th[jj];
                            if (r2 < __dmul_rn(hj, hj)) {
                                acc += pj.w * wendland(r2, tinv[jj], tnorm[jj]);
                                cnt++;
                            }
                        } else {
                            const double hj = th[jj];
                            double w = 0.0;
                            if (r2 < hi2) w += wendland(r2, invhi, normi);
                            if (r2 < __dmul_rn(hj, hj)) w += wendland(r2, tinv[jj], tnorm[jj]);
                            acc += 0.5 * pj.w * w;
                            const double H = fmax(hi, hj);
                            if (r2 < __dmul_rn(H, H)) cnt++;
                        }
                    }
                }
            }
            __syncthreads();
            red[tid] = acc;
            redn[tid] = cnt;
            __syncthreads();
            if (slice == 0) {
                double s = 0.0;
                uint32_t n = 0;
                for (uint32_t q = 0; q < nslice; q++) { s += red[q * tps + li]; n += redn[q * tps + li]; }
                a.rho[i] = s;
                a.nngb[i] = n;
            }
        }
        __syncthreads();
    }
}

// results back to the caller's order
__global__ void k_sph_unsort(size_t n, const uint32_t *inv, const double *rho_s,
                             const uint32_t *n_s, double *rho, uint32_t *nngb) {
    for (size_t u = gtid(); u < n; u += gstride()) {
        const uint32_t r = inv[u];
        rho[u] = rho_s[r];
        nngb[u] = n_s[r];
    }
}

}  // namespace

hipError_t sph_radius(size_t n, const uint32_t *perm, const double *h, double r_fixed,
                      double *sh, DevStatus *st, hipStream_t s) {
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_sph_radius, dim3(grid_for(n)), dim3(kThreads), 0, s, n, perm, h, r_fixed,
                       sh, st);
    return hipGetLastError();
}

hipError_t sph_cell_hmax(const Cells c, const double *sh, double *hmax, hipStream_t s) {
    const unsigned grid = grid_for(c.cap, 4096);
    for (int l = kLevels; l >= 0; l--)
        hipLaunchKernelGGL(k_cell_hmax, dim3(grid), dim3(kThreads), 0, s, l, c, sh, hmax);
    return hipGetLastError();
}

hipError_t sph_group_hmax(size_t gmax, const Groups g, const double *sh, double *rg,
                          DevStatus *st, hipStream_t s) {
    if (!gmax) return hipSuccess;
    hipLaunchKernelGGL(k_group_hmax, dim3(grid_for(gmax * kWave, 4096)), dim3(kThreads), 0, s,
                       &st->n_groups_c, g, sh, rg);
    return hipGetLastError();
}

hipError_t sph_density(int mode, size_t gmax, const Groups g, const uint64_t *seg,
                       const uint32_t *cnt_e, const uint32_t *list, const double4 *jp,
                       const double *sh, double *rho_s, uint32_t *n_s, DevStatus *st,
                       hipStream_t s) {
    if (!gmax) return hipSuccess;
    DensArgs a{&st->n_groups_c, g.begin, g.count, seg, cnt_e, list, jp, sh, rho_s, n_s};
    const unsigned grid = (unsigned)(gmax < 65536 ? gmax : 65536);
    switch (mode) {
        case 0: hipLaunchKernelGGL(k_density<0>, dim3(grid), dim3(kThreads), 0, s, a); break;
        case 1: hipLaunchKernelGGL(k_density<1>, dim3(grid), dim3(kThreads), 0, s, a); break;
        case 2: hipLaunchKernelGGL(k_density<2>, dim3(grid), dim3(kThreads), 0, s, a); break;
        default: hipLaunchKernelGGL(k_density<3>, dim3(grid), dim3(kThreads), 0, s, a); break;
    }
    return hipGetLastError();
}

hipError_t sph_unsort(size_t n, const uint32_t *inv, const double *rho_s, const uint32_t *n_s,
                      double *rho, uint32_t *nngb, hipStream_t s) {
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_sph_unsort, dim3(grid_for(n)), dim3(kThreads), 0, s, n, inv, rho_s, n_s,
                       rho, nngb);
    return hipGetLastError();
}

}  // namespace fdx
