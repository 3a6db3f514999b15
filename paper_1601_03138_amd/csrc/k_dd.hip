// Domain decomposition (section "Domain decomposition"): the multisection method with the
// sampling method.  The current domains (the systems of the particle set) draw samples in
// proportion to their cost; the samples are divided into n_x slabs of equal count along x,
// each slab into n_y columns along y and each column into n_z domains along z, every cut at
// the midpoint of the two samples on either side of it; each particle then gets the domain
// whose box holds it, and the particles are grouped by destination (the exchange).
//
// Layout: samples in SoA FP64 (x, y, z per sample number); each division is a stable radix
// sort of (segment, coordinate key) over the sample numbers followed by one cut pass in
// sorted order; faces are FP64 arrays bx[nx+1], by[nx][ny+1], bz[nx*ny][nz+1].
#include <cmath>

#include "dev_util.h"
#include "fdx_internal.h"

namespace fdx {

namespace {

constexpr int kThreads = 256;

// SplitMix64 (Steele, Lea and Flood 2014): output number ctr of the generator with seed
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t ctr) {
    uint64_t z = seed + (ctr + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// order-preserving unsigned image of an FP64 value (-0 and +0 share one key)
__device__ __forceinline__ uint64_t coord_key(double v) {
    const uint64_t u = (uint64_t)__double_as_longlong(v + 0.0);
    return (u >> 63) ? ~u : (u | (1ull << 63));
}

// last index i in [0, n) with a[i] <= v (a ascending, a[0] <= v)
template <class T>
__device__ __forceinline__ uint32_t last_le(const T *a, uint32_t n, T v) {
    uint32_t lo = 0, hi = n;          // a[lo] <= v, answer in [lo, hi)
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (a[mid] <= v) lo = mid; else hi = mid;
    }
    return lo;
}

// groups come in system order, so a wave's groups belong to few systems: each wave sums its
// weights per system and issues one atomic per system it holds
__global__ void __launch_bounds__(kThreads)
k_dd_cost(uint32_t G, const uint32_t *g_sys, const uint32_t *g_count, const uint32_t *cnt_e,
          const uint32_t *cnt_s, unsigned long long *cost) {
    const uint32_t g = blockIdx.x * kThreads + threadIdx.x;
    const bool valid = g < G;
    const uint32_t sys = valid ? g_sys[g] : 0xFFFFFFFFu;
    const unsigned long long w =
        valid ? (unsigned long long)g_count[g] * ((unsigned long long)cnt_e[g] + cnt_s[g]) : 0ull;
    uint64_t pending = __ballot(valid);
    while (pending) {
        const int leader = __ffsll((long long)pending) - 1;
        const uint32_t s0 = __shfl(sys, leader);
        const bool mine = valid && sys == s0;
        pending &= ~__ballot(mine);
        unsigned long long v = mine ? w : 0ull;
        for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if (lane_id() == leader) atomicAdd(&cost[s0], v);
    }
}

// sample s of the domain p with kofs[p] <= s < kofs[p+1]: particle
// off[p] + floor(r n_p / 2^64), r = SplitMix64 output s
__global__ void __launch_bounds__(kThreads)
k_dd_sample(uint32_t K, uint32_t nsys, const int64_t *kofs, const int64_t *off, uint64_t seed,
            const double *x, const double *y, const double *z, uint32_t *idx, double *sx,
            double *sy, double *sz, uint64_t *key, uint32_t *val) {
    const uint32_t s = blockIdx.x * kThreads + threadIdx.x;
    if (s >= K) return;
    const uint32_t p = last_le<int64_t>(kofs, nsys + 1, (int64_t)s);
    const uint64_t np = (uint64_t)(off[p + 1] - off[p]);
    const uint64_t i = (uint64_t)off[p] + __umul64hi(splitmix64(seed, s), np);
    idx[s] = (uint32_t)i;
    const double vx = x[i];
    sx[s] = vx;
    sy[s] = y[i];
    sz[s] = z[i];
    key[s] = coord_key(vx);
    val[s] = s;
}

// One division: the samples sorted by (segment, coordinate, sample number), segment g at the
// sorted ranks [start[g], start[g+1]).  Run i of a segment of m samples is its ranks
// [floor(i m / n), floor((i+1) m / n)); rank j lies in run ((j + 1) n - 1) / m.
__global__ void __launch_bounds__(kThreads)
k_dd_cut(uint32_t K, uint32_t nseg, const uint32_t *start, uint32_t n, const uint32_t *val,
         const double *coord, const double *next, uint32_t *cell, uint32_t *new_start,
         double *face, uint64_t *key_next, uint32_t *val_next) {
    const uint32_t r = blockIdx.x * kThreads + threadIdx.x;
    if (r >= K) return;
    const uint32_t g = last_le<uint32_t>(start, nseg + 1, r);
    const uint64_t m = start[g + 1] - start[g], j = r - start[g];
    const uint32_t i = (uint32_t)(((j + 1) * n - 1) / m);
    const uint32_t s = val[r];
    const uint32_t c = g * n + i;
    cell[s] = c;
    double *b = face + (size_t)g * (n + 1);
    if (j == (uint64_t)i * m / n) {
        new_start[c] = r;
        if (i > 0) b[i] = (coord[val[r - 1]] + coord[s]) * 0.5;
    }
    if (j == 0) {
        b[0] = -INFINITY;
        b[n] = INFINITY;
    }
    if (r == K - 1) new_start[(size_t)nseg * n] = K;
    if (next) {
        key_next[s] = coord_key(next[s]);
        val_next[s] = s;
    }
}

// destination of every particle; it is also the grouping key (the current domains are
// contiguous and in order, so a stable grouping by destination keeps (source, position) order)
__global__ void __launch_bounds__(kThreads)
k_dd_assign(uint32_t n, const double *x, const double *y, const double *z, uint32_t nx,
            uint32_t ny, uint32_t nz, const double *bx, const double *by, const double *bz,
            uint32_t *dest, uint64_t *key, uint32_t *val) {
    const uint32_t i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    // the run [b[k], b[k+1]) holding the coordinate: last face at or below it (b[0] = -inf)
    const uint32_t a = last_le<double>(bx, nx, x[i]);
    const uint32_t c = last_le<double>(by + (size_t)a * (ny + 1), ny, y[i]);
    const uint32_t col = a * ny + c;
    const uint32_t e = last_le<double>(bz + (size_t)col * (nz + 1), nz, z[i]);
    const uint32_t d = col * nz + e;
    dest[i] = d;
    key[i] = d;
    val[i] = i;
}

// first and one-past-last grouped position of every (destination, source) run; the source of
// position r is the current domain of particle order[r]
__global__ void __launch_bounds__(kThreads)
k_dd_runs(uint32_t n, const uint64_t *dest, const uint32_t *order, const uint32_t *sysid,
          uint32_t nsrc, uint32_t *run_lo, uint32_t *run_hi) {
    const uint32_t r = blockIdx.x * kThreads + threadIdx.x;
    if (r >= n) return;
    auto pair = [&](uint32_t q) { return dest[q] * nsrc + sysid[order[q]]; };
    const uint64_t k = pair(r);
    if (r == 0 || pair(r - 1) != k) run_lo[k] = r;
    if (r == n - 1 || pair(r + 1) != k) run_hi[k] = r + 1;
}

__global__ void __launch_bounds__(kThreads)
k_dd_gather(uint32_t n, const uint32_t *order, int narr, DdArrays src, DdArrays dst) {
    const uint32_t r = blockIdx.x * kThreads + threadIdx.x;
    if (r >= n) return;
    const uint32_t i = order[r];
    for (int k = 0; k < narr; k++) dst.p[k][r] = src.p[k][i];
}

inline dim3 grid_of(size_t n) { return dim3((unsigned)((n + kThreads - 1) / kThreads)); }

}  // namespace

hipError_t dd_cost(uint32_t G, const uint32_t *g_sys, const uint32_t *g_count,
                   const uint32_t *cnt_e, const uint32_t *cnt_s, uint64_t *cost, hipStream_t s) {
    if (G == 0) return hipSuccess;
    hipLaunchKernelGGL(k_dd_cost, grid_of(G), dim3(kThreads), 0, s, G, g_sys, g_count, cnt_e,
                       cnt_s, (unsigned long long *)cost);
    return hipGetLastError();
}

hipError_t dd_sample(uint32_t K, uint32_t nsys, const int64_t *kofs, const int64_t *off,
                     uint64_t seed, const double *x, const double *y, const double *z,
                     uint32_t *idx, double *sx, double *sy, double *sz, uint64_t *key,
                     uint32_t *val, hipStream_t s) {
    if (K == 0) return hipSuccess;
    hipLaunchKernelGGL(k_dd_sample, grid_of(K), dim3(kThreads), 0, s, K, nsys, kofs, off, seed,
                       x, y, z, idx, sx, sy, sz, key, val);
    return hipGetLastError();
}

hipError_t dd_cut(uint32_t K, uint32_t nseg, const uint32_t *start, uint32_t n,
                  const uint32_t *val, const double *coord, const double *next, uint32_t *cell,
                  uint32_t *new_start, double *face, uint64_t *key_next, uint32_t *val_next,
                  hipStream_t s) {
    if (K == 0) return hipSuccess;
    hipLaunchKernelGGL(k_dd_cut, grid_of(K), dim3(kThreads), 0, s, K, nseg, start, n, val, coord,
                       next, cell, new_start, face, key_next, val_next);
    return hipGetLastError();
}

hipError_t dd_assign(uint32_t n, const double *x, const double *y, const double *z, uint32_t nx,
                     uint32_t ny, uint32_t nz, const double *bx, const double *by,
                     const double *bz, uint32_t *dest, uint64_t *key, uint32_t *val,
                     hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_dd_assign, grid_of(n), dim3(kThreads), 0, s, n, x, y, z, nx, ny, nz, bx,
                       by, bz, dest, key, val);
    return hipGetLastError();
}

hipError_t dd_runs(uint32_t n, const uint64_t *dest, const uint32_t *order,
                   const uint32_t *sysid, uint32_t nsrc, uint32_t *run_lo, uint32_t *run_hi,
                   hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_dd_runs, grid_of(n), dim3(kThreads), 0, s, n, dest, order, sysid, nsrc,
                       run_lo, run_hi);
    return hipGetLastError();
}

hipError_t dd_gather(uint32_t n, const uint32_t *order, int narr, const DdArrays &src,
                     const DdArrays &dst, hipStream_t s) {
    if (n == 0 || narr == 0) return hipSuccess;
    hipLaunchKernelGGL(k_dd_gather, grid_of(n), dim3(kThreads), 0, s, n, order, narr, src, dst);
    return hipGetLastError();
}

}  // namespace fdx
