// Elementwise kernels: fills, input checks, leapfrog kick/drift, return of forces to the
// caller's order, and the device-wide exclusive scan used by the tree build, the group
// numbering and the list offsets.
#include "dev_util.h"
#include "fdx_internal.h"

namespace fdx {

namespace {

constexpr int kThreads = 256;

inline unsigned grid_for(size_t n, unsigned cap = 16384) {
    size_t b = (n + kThreads - 1) / kThreads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v, size_t n) {
    for (size_t i = gtid(); i < n; i += gstride()) p[i] = v;
}
__global__ void k_fill_u64(uint64_t *p, uint64_t v, size_t n) {
    for (size_t i = gtid(); i < n; i += gstride()) p[i] = v;
}
__global__ void k_iota_u32(uint32_t *p, size_t n) {
    for (size_t i = gtid(); i < n; i += gstride()) p[i] = (uint32_t)i;
}

__global__ void k_check_input(size_t n, const double *x, const double *y, const double *z,
                              const double *m, const double *eps, DevStatus *st) {
    bool bad = false;
    for (size_t i = gtid(); i < n; i += gstride()) {
        bad |= !isfinite(x[i]) || !isfinite(y[i]) || !isfinite(z[i]);
        bad |= !(m[i] >= 0.0) || !isfinite(m[i]);
        if (eps) bad |= !(eps[i] > 0.0) || !isfinite(eps[i]);
    }
    if (bad) atomicOr(&st->bad_input, 1u);
}

// flag |= 1 if some eps[i] differs from the eps of the first particle of its system (a NaN
// differs from everything)
__global__ void k_eps_varies(size_t n, const double *eps, const uint32_t *sysid,
                             const int64_t *off, uint32_t *flag) {
    bool v = false;
    for (size_t i = gtid(); i < n; i += gstride()) v |= !(eps[i] == eps[off[sysid[i]]]);
    if (v) atomicOr(flag, 1u);
}

// sysid[i] = system of particle i (binary search in the offsets).
__global__ void k_sysid(const int64_t *off, int nsys, uint32_t *sysid, size_t n) {
    for (size_t i = gtid(); i < n; i += gstride()) {
        int lo = 0, hi = nsys - 1;             // last s with off[s] <= i
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if ((size_t)off[mid] <= i) lo = mid; else hi = mid - 1;
        }
        sysid[i] = (uint32_t)lo;
    }
}

// predict of the sample program: v += dt/2 a; x += dt v.
__global__ void k_kick_drift(size_t n, double *x, double *y, double *z, double *vx, double *vy,
                             double *vz, const double *ax, const double *ay, const double *az,
                             double dt) {
    const double h = 0.5 * dt;
    for (size_t i = gtid(); i < n; i += gstride()) {
        double u = vx[i] + h * ax[i], v = vy[i] + h * ay[i], w = vz[i] + h * az[i];
        vx[i] = u; vy[i] = v; vz[i] = w;
        x[i] += dt * u; y[i] += dt * v; z[i] += dt * w;
    }
}

// correct of the sample program: v += dt/2 a.  Skipped when the force evaluation of this
// step reported an overflow (its forces are incomplete; the host redoes force and kick).
__global__ void k_kick(size_t n, double *vx, double *vy, double *vz, const double *ax,
                       const double *ay, const double *az, double dt, const DevStatus *st) {
    if (st && status_incomplete(*st)) return;
    const double h = 0.5 * dt;
    for (size_t i = gtid(); i < n; i += gstride()) {
        vx[i] += h * ax[i]; vy[i] += h * ay[i]; vz[i] += h * az[i];
    }
}

// Forces from sorted rank back to the caller's order: a[u] = fs[inv[u]] (coalesced writes,
// one 32-byte gather per particle).
__global__ void k_unsort(size_t n, const double4 *fs, const uint32_t *inv, double *ax,
                         double *ay, double *az, double *pot) {
    for (size_t u = gtid(); u < n; u += gstride()) {
        double4 f = fs[inv[u]];
        ax[u] = f.x; ay[u] = f.y; az[u] = f.z; pot[u] = f.w;
    }
}

// ---------------------------------------------------------------------------------------
// Reduce-then-scan over a fixed grid of kScanBlocks blocks; the element count may live in
// device memory (so the whole tree build runs without host round trips).
__device__ __forceinline__ size_t scan_count(size_t n_host, const uint32_t *lo,
                                             const uint32_t *hi) {
    if (hi) return (size_t)(*hi - (lo ? *lo : 0u));
    return n_host;
}

__global__ void __launch_bounds__(kThreads)
k_scan_reduce(const uint32_t *in, size_t n_host, const uint32_t *lo, const uint32_t *hi,
              uint64_t *partial) {
    __shared__ uint64_t lds[kThreads / kWave];
    const size_t n = scan_count(n_host, lo, hi);
    const size_t chunk = (n + kScanBlocks - 1) / kScanBlocks;
    const size_t b0 = blockIdx.x * chunk, b1 = min(n, b0 + chunk);
    // four independent sums: four loads in flight per thread
    uint64_t s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    size_t i = b0 + threadIdx.x;
    for (; i + 3 * kThreads < b1; i += 4 * kThreads) {
        s0 += in[i]; s1 += in[i + kThreads]; s2 += in[i + 2 * kThreads]; s3 += in[i + 3 * kThreads];
    }
    for (; i < b1; i += kThreads) s0 += in[i];
    uint64_t s = wave_sum_u64(s0 + s1 + s2 + s3);
    if (lane_id() == 0) lds[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        for (int k = 0; k < kThreads / kWave; k++) t += lds[k];
        partial[blockIdx.x] = t;
    }
}

template <class T>
__global__ void __launch_bounds__(kScanBlocks)
k_scan_top(uint64_t *partial, T *total) {
    __shared__ uint64_t lds[kScanBlocks / kWave];
    uint64_t v = partial[threadIdx.x], tot;
    uint64_t e = block_excl_scan<kScanBlocks>(v, lds, &tot);
    partial[threadIdx.x] = e;
    if (threadIdx.x == 0) {
        partial[kScanBlocks] = tot;
        if (total) *total = (T)tot;
    }
}

template <class T>
__global__ void __launch_bounds__(kThreads)
k_scan_down(const uint32_t *in, T *out, size_t n_host, const uint32_t *lo, const uint32_t *hi,
            const uint64_t *partial) {
    __shared__ uint64_t lds[kThreads / kWave];
    const size_t n = scan_count(n_host, lo, hi);
    const size_t chunk = (n + kScanBlocks - 1) / kScanBlocks;
    const size_t b0 = blockIdx.x * chunk, b1 = min(n, b0 + chunk);
    uint64_t base = partial[blockIdx.x];
    for (size_t t0 = b0; t0 < b1; t0 += kThreads) {
        size_t i = t0 + threadIdx.x;
        uint64_t v = i < b1 ? in[i] : 0;
        uint64_t tot;
        uint64_t e = block_excl_scan<kThreads>(v, lds, &tot);
        if (i < b1) out[i] = (T)(base + e);
        base += tot;
    }
}

// The down-sweep for 32-bit outputs (the prefix fits 32 bits, so every partial sum does):
// 4 x 256 elements per iteration, each 256-element sub-tile scanned per wave with DPP, the 16
// wave totals combined through LDS -- one barrier pair per 1024 elements.  The same sums as
// k_scan_down<uint32_t> (unsigned arithmetic modulo 2^32), in far fewer barriers.
constexpr int kSub = 4;
__global__ void __launch_bounds__(kThreads)
k_scan_down32(const uint32_t *in, uint32_t *out, size_t n_host, const uint32_t *lo,
              const uint32_t *hi, const uint64_t *partial) {
    __shared__ uint32_t lds[kSub][kThreads / kWave];
    const size_t n = scan_count(n_host, lo, hi);
    const size_t chunk = (n + kScanBlocks - 1) / kScanBlocks;
    const size_t b0 = blockIdx.x * chunk, b1 = min(n, b0 + chunk);
    const int w = threadIdx.x / kWave, l = lane_id();
    uint32_t base = (uint32_t)partial[blockIdx.x];
    for (size_t t0 = b0; t0 < b1; t0 += kSub * kThreads) {
        uint32_t v[kSub], inc[kSub];
#pragma unroll
        for (int k = 0; k < kSub; k++) {
            const size_t i = t0 + (size_t)k * kThreads + threadIdx.x;
            v[k] = i < b1 ? in[i] : 0u;
        }
#pragma unroll
        for (int k = 0; k < kSub; k++) {
            inc[k] = wave_incl_scan_dpp(v[k]);
            if (l == kWave - 1) lds[k][w] = inc[k];
        }
        __syncthreads();
        // offset of (sub-tile k, wave w): every wave of the earlier sub-tiles, then the
        // earlier waves of sub-tile k
        uint32_t run = 0, off[kSub];
#pragma unroll
        for (int k = 0; k < kSub; k++) {
#pragma unroll
            for (int q = 0; q < kThreads / kWave; q++) {
                if (q == w) off[k] = run;
                run += lds[k][q];
            }
        }
#pragma unroll
        for (int k = 0; k < kSub; k++) {
            const size_t i = t0 + (size_t)k * kThreads + threadIdx.x;
            if (i < b1) out[i] = base + off[k] + inc[k] - v[k];
        }
        base += run;
        __syncthreads();
    }
}

template <class T>
hipError_t scan_impl(const uint32_t *in, T *out, size_t n_host, const uint32_t *lo,
                     const uint32_t *hi, uint64_t *partial, T *total, hipStream_t s) {
    hipLaunchKernelGGL(k_scan_reduce, dim3(kScanBlocks), dim3(kThreads), 0, s, in, n_host, lo,
                       hi, partial);
    hipLaunchKernelGGL(k_scan_top<T>, dim3(1), dim3(kScanBlocks), 0, s, partial, total);
    if constexpr (sizeof(T) == 4)
        hipLaunchKernelGGL(k_scan_down32, dim3(kScanBlocks), dim3(kThreads), 0, s, in,
                           (uint32_t *)out, n_host, lo, hi, (const uint64_t *)partial);
    else
        hipLaunchKernelGGL(k_scan_down<T>, dim3(kScanBlocks), dim3(kThreads), 0, s, in, out,
                           n_host, lo, hi, (const uint64_t *)partial);
    return hipGetLastError();
}

}  // namespace

hipError_t fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s) {
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n)), dim3(kThreads), 0, s, p, v, n);
    return hipGetLastError();
}
hipError_t fill_u64(uint64_t *p, uint64_t v, size_t n, hipStream_t s) {
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n)), dim3(kThreads), 0, s, p, v, n);
    return hipGetLastError();
}
hipError_t iota_u32(uint32_t *p, size_t n, hipStream_t s) {
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_iota_u32, dim3(grid_for(n)), dim3(kThreads), 0, s, p, n);
    return hipGetLastError();
}
hipError_t check_input(size_t n, const double *x, const double *y, const double *z,
                       const double *m, const double *eps, DevStatus *st, hipStream_t s) {
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_check_input, dim3(grid_for(n, 4096)), dim3(kThreads), 0, s, n, x, y,
                       z, m, eps, st);
    return hipGetLastError();
}
hipError_t eps_varies(size_t n, const double *eps, const uint32_t *sysid, const int64_t *off,
                      uint32_t *flag, hipStream_t s) {
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_eps_varies, dim3(grid_for(n, 4096)), dim3(kThreads), 0, s, n, eps, sysid,
                       off, flag);
    return hipGetLastError();
}
hipError_t sysid_fill(const int64_t *off, int nsys, uint32_t *sysid, size_t n, hipStream_t s) {
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_sysid, dim3(grid_for(n)), dim3(kThreads), 0, s, off, nsys, sysid, n);
    return hipGetLastError();
}
hipError_t kick_drift(size_t n, double *x, double *y, double *z, double *vx, double *vy,
                      double *vz, const double *ax, const double *ay, const double *az,
                      double dt, hipStream_t s) {
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_kick_drift, dim3(grid_for(n)), dim3(kThreads), 0, s, n, x, y, z, vx,
                       vy, vz, ax, ay, az, dt);
    return hipGetLastError();
}
hipError_t kick(size_t n, double *vx, double *vy, double *vz, const double *ax,
                const double *ay, const double *az, double dt, const DevStatus *st,
                hipStream_t s) {
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_kick, dim3(grid_for(n)), dim3(kThreads), 0, s, n, vx, vy, vz, ax, ay,
                       az, dt, st);
    return hipGetLastError();
}
hipError_t unsort_forces(size_t n, const double4 *fs, const uint32_t *inv, double *ax,
                         double *ay, double *az, double *pot, hipStream_t s) {
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_unsort, dim3(grid_for(n)), dim3(kThreads), 0, s, n, fs, inv, ax, ay,
                       az, pot);
    return hipGetLastError();
}
hipError_t scan_u32_to_u32(const uint32_t *in, uint32_t *out, size_t n_host,
                           const uint32_t *lo, const uint32_t *hi, uint64_t *partial,
                           uint32_t *total32, hipStream_t s) {
    return scan_impl<uint32_t>(in, out, n_host, lo, hi, partial, total32, s);
}
hipError_t scan_u32_to_u64(const uint32_t *in, uint64_t *out, size_t n_host,
                           const uint32_t *lo, const uint32_t *hi, uint64_t *partial,
                           uint64_t *total64, hipStream_t s) {
    return scan_impl<uint64_t>(in, out, n_host, lo, hi, partial, total64, s);
}

}  // namespace fdx
