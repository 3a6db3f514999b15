// Root cube per system and 63-bit Morton keys.
//
// The paper states only that each process constructs a Barnes-Hut octree of its particles
// (section "Interaction calculation") at O(n log n) cost (section "Tree construction").
// This library builds it from space-filling-curve keys: the root cube of a system is the
// smallest power-of-two cube anchored at the exact per-axis minimum that covers the exact
// extent; each coordinate is quantised to 21 bits and the bits are interleaved (x on bit
// 3b+2, y on 3b+1, z on 3b).  A key comes from exact min/max, one correctly rounded FP64
// subtraction (x - o), an exact scaling by the power of two 2^21 / Lr and a floor.  The
// oracle performs the same subtraction and scaling operation for operation, with
// contraction off on both sides, so keys agree bit for bit; fusing the two into an FMA,
// reassociating them or precomputing a scaled origin would break that parity.
#include "dev_util.h"
#include "fdx_internal.h"

#pragma clang fp contract(off)

namespace fdx {

namespace {

constexpr int kThreads = 256;
constexpr int kBboxChunk = 4096;

// Per-system min/max of x, y, z as order-preserving u64 (bbox_u[6 s + 2 a] = min of axis a,
// bbox_u[6 s + 2 a + 1] = max).  A block reduces a contiguous chunk; elements of a system
// other than the chunk's first (systems are contiguous, so a wave's 64 consecutive elements
// hold few of them) are reduced per wave and system and issue one set of atomics each.
__global__ void __launch_bounds__(kThreads)
k_bbox(size_t n, const double *x, const double *y, const double *z, const uint32_t *sysid,
       uint64_t *bbox_u) {
    __shared__ uint64_t red[6][kThreads / kWave];
    const size_t b0 = (size_t)blockIdx.x * kBboxChunk;
    if (b0 >= n) return;
    const size_t b1 = min(n, b0 + kBboxChunk);
    const uint32_t s0 = sysid ? sysid[b0] : 0u;
    const int lane = lane_id();
    uint64_t mn[3] = {~0ull, ~0ull, ~0ull}, mx[3] = {0, 0, 0};
    // wave-uniform trip count: every lane of a wave takes part in the ballots below
    for (size_t base = b0 + (threadIdx.x - lane); base < b1; base += kThreads) {
        const size_t i = base + lane;
        const bool valid = i < b1;
        uint64_t v[3] = {0, 0, 0};
        uint32_t s = s0;
        if (valid) {
            v[0] = dbl_to_ord(x[i]); v[1] = dbl_to_ord(y[i]); v[2] = dbl_to_ord(z[i]);
            s = sysid ? sysid[i] : s0;
            if (s == s0) {
#pragma unroll
                for (int a = 0; a < 3; a++) { mn[a] = min(mn[a], v[a]); mx[a] = max(mx[a], v[a]); }
            }
        }
        uint64_t pending = __ballot(valid && s != s0);
        while (pending) {
            const int leader = __ffsll((long long)pending) - 1;
            const uint32_t s1 = __shfl(s, leader);
            const bool mine = valid && s == s1;
            pending &= ~__ballot(mine);
            uint64_t lo[3], hi[3];
#pragma unroll
            for (int a = 0; a < 3; a++) { lo[a] = mine ? v[a] : ~0ull; hi[a] = mine ? v[a] : 0ull; }
#pragma unroll
            for (int a = 0; a < 3; a++) {
#pragma unroll
                for (int d = 32; d >= 1; d >>= 1) {
                    lo[a] = min(lo[a], (uint64_t)__shfl_xor((unsigned long long)lo[a], d, kWave));
                    hi[a] = max(hi[a], (uint64_t)__shfl_xor((unsigned long long)hi[a], d, kWave));
                }
            }
            if (lane == leader) {
#pragma unroll
                for (int a = 0; a < 3; a++) {
                    atomicMin((unsigned long long *)&bbox_u[6 * s1 + 2 * a], (unsigned long long)lo[a]);
                    atomicMax((unsigned long long *)&bbox_u[6 * s1 + 2 * a + 1], (unsigned long long)hi[a]);
                }
            }
        }
    }
#pragma unroll
    for (int a = 0; a < 3; a++) {
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
            mn[a] = min(mn[a], (uint64_t)__shfl_xor((unsigned long long)mn[a], d, kWave));
            mx[a] = max(mx[a], (uint64_t)__shfl_xor((unsigned long long)mx[a], d, kWave));
        }
    }
    const int w = threadIdx.x / kWave;
    if (lane_id() == 0) {
#pragma unroll
        for (int a = 0; a < 3; a++) { red[2 * a][w] = mn[a]; red[2 * a + 1][w] = mx[a]; }
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        const int k = threadIdx.x;
        uint64_t r = red[k][0];
        for (int j = 1; j < kThreads / kWave; j++) r = (k & 1) ? max(r, red[k][j]) : min(r, red[k][j]);
        if (k & 1) atomicMax((unsigned long long *)&bbox_u[6 * s0 + k], (unsigned long long)r);
        else atomicMin((unsigned long long *)&bbox_u[6 * s0 + k], (unsigned long long)r);
    }
}

__global__ void k_bbox_init(int nsys, uint64_t *bbox_u) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < 6 * nsys) bbox_u[k] = (k & 1) ? 0ull : ~0ull;
}

// Smallest power of two >= L (L > 0, finite), from the exponent field: L itself when its
// significand is 1.0, else the next power of two.
__device__ double pow2_ceil(double L) {
    uint64_t b = (uint64_t)__double_as_longlong(L);
    uint64_t e = (b >> 52) & 0x7FF, f = b & 0xFFFFFFFFFFFFFull;
    if (e == 0) {                          // subnormal L = f * 2^-1074: 2^ceil(log2 f) * 2^-1074
        int k = f <= 1 ? 0 : 64 - __clzll((long long)(f - 1));
        if (k >= 52) return __longlong_as_double((long long)((uint64_t)(k - 51) << 52));
        return __longlong_as_double((long long)(1ull << k));
    }
    if (f == 0) return L;
    return __longlong_as_double((long long)((e + 1) << 52));
}

// cube[4 s] = {origin x, y, z, side Lr}; an empty system gets origin 0 and side 1.
__global__ void k_root_cubes(int nsys, const uint64_t *bbox_u, double *cube) {
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < nsys; s += gridDim.x * blockDim.x) {
        const uint64_t *b = bbox_u + 6 * s;
        double lo[3], L = 0.0;
        bool empty = b[0] > b[1];
        for (int a = 0; a < 3; a++) {
            lo[a] = empty ? 0.0 : ord_to_dbl(b[2 * a]);
            double hi = empty ? 0.0 : ord_to_dbl(b[2 * a + 1]);
            double ext = hi - lo[a];
            if (ext > L) L = ext;
        }
        double Lr = L > 0.0 ? pow2_ceil(L) : 1.0;
        cube[4 * s] = lo[0]; cube[4 * s + 1] = lo[1]; cube[4 * s + 2] = lo[2]; cube[4 * s + 3] = Lr;
    }
}

__device__ __forceinline__ uint32_t grid_coord(double v, double o, double scale) {
    double t = (v - o) * scale;            // exact scale: a power of two
    double f = floor(t);
    f = f < 0.0 ? 0.0 : f;
    f = f > 2097151.0 ? 2097151.0 : f;
    return (uint32_t)f;
}

// Keys and the identity permutation; the same pass writes each particle's (x, y, z, m) record
// for the sorted gather (one read of the coordinates for both).  sysid null: one system.
__global__ void k_keys(size_t n, const double *x, const double *y, const double *z,
                       const double *m, const uint32_t *sysid, const double *cube, uint64_t *key,
                       uint32_t *perm, double4 *packed) {
    for (size_t i = gtid(); i < n; i += gstride()) {
        const double *c = cube + 4 * (size_t)(sysid ? sysid[i] : 0u);
        const double scale = 2097152.0 / c[3];
        const double xi = x[i], yi = y[i], zi = z[i];
        uint64_t qx = grid_coord(xi, c[0], scale), qy = grid_coord(yi, c[1], scale),
                 qz = grid_coord(zi, c[2], scale);
        key[i] = (spread3(qx) << 2) | (spread3(qy) << 1) | spread3(qz);
        perm[i] = (uint32_t)i;
        packed[i] = make_double4(xi, yi, zi, m[i]);
    }
}

inline unsigned grid_for(size_t n, unsigned cap = 16384) {
    size_t b = (n + kThreads - 1) / kThreads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

}  // namespace

hipError_t bbox(size_t n, const double *x, const double *y, const double *z,
                const uint32_t *sysid, int nsys, uint64_t *bbox_u, hipStream_t s) {
    // min words start at ~0 and max words at 0, so an empty system keeps min > max
    hipLaunchKernelGGL(k_bbox_init, dim3((6 * nsys + 255) / 256), dim3(256), 0, s, nsys, bbox_u);
    if (!n) return hipGetLastError();
    size_t blocks = (n + kBboxChunk - 1) / kBboxChunk;
    hipLaunchKernelGGL(k_bbox, dim3((unsigned)blocks), dim3(kThreads), 0, s, n, x, y, z,
                       nsys > 1 ? sysid : nullptr, bbox_u);
    return hipGetLastError();
}

hipError_t root_cubes(int nsys, const uint64_t *bbox_u, double *cube, hipStream_t s) {
    hipLaunchKernelGGL(k_root_cubes, dim3((nsys + 255) / 256), dim3(256), 0, s, nsys, bbox_u, cube);
    return hipGetLastError();
}

hipError_t morton_keys(size_t n, const double *x, const double *y, const double *z,
                       const double *m, const uint32_t *sysid, int nsys, const double *cube,
                       uint64_t *key, uint32_t *perm, double4 *packed, hipStream_t s) {
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_keys, dim3(grid_for(n)), dim3(kThreads), 0, s, n, x, y, z, m,
                       nsys > 1 ? sysid : nullptr, cube, key, perm, packed);
    return hipGetLastError();
}

}  // namespace fdx
