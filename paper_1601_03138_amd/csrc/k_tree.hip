// Octree topology, multipole moments and i-particle groups on sorted keys.
//
// Cells are runs of sorted particles that share the top 3l key bits (level l).  Reading of
// the paper's silent tree construction: one root (level 0) per system; a cell holding more
// than n_leaf particles below level 21 is split into its non-empty octants, in octant
// order; cells are numbered breadth first.  The build runs level by level entirely on the
// device (level sizes stay in device memory), so it needs no host round trip.
//
// Moments (superparticles up to the quadrupole, section "Design concept of FDPS"): mass,
// centre of mass and the traceless quadrupole Q_ab = sum m (3 d_a d_b - d^2 delta_ab) about
// the centre of mass, accumulated bottom-up (leaves from particles, parents from children by
// the parallel-axis shift).
//
// Groups (modified tree algorithm, section "Tree traverse and interaction calculation"):
// maximal cells of at most n_group particles; an over-full leaf is cut into runs of n_group.
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

// (x, y, z, m) of every particle as one 32-byte record in the caller's order (coalesced), so
// the sorted gather below reads one sector per particle instead of four.
__global__ void k_pack(size_t n, const double *x, const double *y, const double *z,
                       const double *m, double4 *packed) {
    for (size_t i = gtid(); i < n; i += gstride()) packed[i] = make_double4(x[i], y[i], z[i], m[i]);
}

__global__ void k_gather_sorted(size_t n, const uint32_t *perm, const double4 *packed,
                                const double *eps, double eps_all, double4 *jp, double *seps,
                                uint32_t *inv) {
    for (size_t r = gtid(); r < n; r += gstride()) {
        const uint32_t i = perm[r];
        jp[r] = packed[i];
        seps[r] = eps ? eps[i] : eps_all;
        inv[i] = (uint32_t)r;
    }
}

// roots: cell s = system s, level 0
__global__ void k_tree_init(int nsys, const int64_t *off, Cells c, DevStatus *st) {
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < nsys; s += gridDim.x * blockDim.x) {
        c.level[s] = 0;
        c.prefix[s] = 0;
        c.begin[s] = (uint32_t)off[s];
        c.count[s] = (uint32_t)(off[s + 1] - off[s]);
        c.parent[s] = kNone;
        c.first[s] = kNone;
        c.nchild[s] = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        c.lvl[0] = 0;
        c.lvl[1] = (uint32_t)nsys;
        for (int l = 2; l <= kLevels + 1; l++) c.lvl[l] = (uint32_t)nsys;
        st->cell_overflow = 0;
    }
}

// first index in [b, e) whose octant digit (bits sh..sh+2) is >= o; digits ascend on [b, e)
__device__ __forceinline__ uint32_t lower_digit(const uint64_t *k, uint32_t b, uint32_t e,
                                                int sh, uint32_t o) {
    while (b < e) {
        uint32_t mid = b + ((e - b) >> 1);
        if ((uint32_t)((k[mid] >> sh) & 7u) < o) b = mid + 1; else e = mid;
    }
    return b;
}

__device__ __forceinline__ void octant_bounds(const uint64_t *skey, uint32_t b, uint32_t e,
                                              int sh, uint32_t *bd) {
    bd[0] = b;
    bd[8] = e;
    // 7 boundaries by nested binary search: octants 4, then 2/6, then odd
    bd[4] = lower_digit(skey, b, e, sh, 4);
    bd[2] = lower_digit(skey, b, bd[4], sh, 2);
    bd[6] = lower_digit(skey, bd[4], e, sh, 6);
    bd[1] = lower_digit(skey, b, bd[2], sh, 1);
    bd[3] = lower_digit(skey, bd[2], bd[4], sh, 3);
    bd[5] = lower_digit(skey, bd[4], bd[6], sh, 5);
    bd[7] = lower_digit(skey, bd[6], e, sh, 7);
}

// number of children of every cell of level l
__global__ void k_tree_split(int l, int n_leaf, const uint64_t *skey, Cells c, uint32_t *tmp_n) {
    const uint32_t c0 = c.lvl[l], c1 = c.lvl[l + 1];
    const int sh = 3 * (kLevels - 1 - l);
    for (size_t k = gtid(); k < c1 - c0; k += gstride()) {
        const uint32_t cid = c0 + (uint32_t)k;
        uint32_t nch = 0;
        const uint32_t cnt = c.count[cid];
        if (l < kLevels && cnt > (uint32_t)n_leaf) {
            uint32_t bd[9];
            octant_bounds(skey, c.begin[cid], c.begin[cid] + cnt, sh, bd);
#pragma unroll
            for (int o = 0; o < 8; o++) nch += bd[o + 1] > bd[o] ? 1u : 0u;
        }
        tmp_n[k] = nch;
    }
}

// write the children of level l (first child index from the scan of tmp_n); *total = number
// of cells of level l+1
__global__ void k_tree_emit(int l, const uint64_t *skey, Cells c, const uint32_t *tmp_n,
                            const uint32_t *tmp_off, const uint32_t *total, DevStatus *st) {
    const uint32_t c0 = c.lvl[l], c1 = c.lvl[l + 1];
    const uint32_t next = c1 + *total;
    const bool ovf = next > c.cap || st->cell_overflow;
    if (gtid() == 0) {
        if (ovf) st->cell_overflow = 1;
        c.lvl[l + 2] = ovf ? c1 : next;
        for (int k = l + 3; k <= kLevels + 1; k++) c.lvl[k] = ovf ? c1 : next;
    }
    const int sh = 3 * (kLevels - 1 - l);
    for (size_t k = gtid(); k < c1 - c0; k += gstride()) {
        const uint32_t cid = c0 + (uint32_t)k;
        const uint32_t nch = ovf ? 0u : tmp_n[k];
        c.nchild[cid] = nch;
        if (nch == 0) { c.first[cid] = kNone; continue; }
        const uint32_t first = c1 + tmp_off[k];
        c.first[cid] = first;
        uint32_t bd[9];
        const uint32_t b = c.begin[cid];
        octant_bounds(skey, b, b + c.count[cid], sh, bd);
        const uint64_t pre = c.prefix[cid] << 3;
        uint32_t j = first;
#pragma unroll
        for (int o = 0; o < 8; o++) {
            if (bd[o + 1] > bd[o]) {
                c.level[j] = (uint32_t)(l + 1);
                c.prefix[j] = pre | (uint64_t)o;
                c.begin[j] = bd[o];
                c.count[j] = bd[o + 1] - bd[o];
                c.parent[j] = cid;
                c.first[j] = kNone;
                c.nchild[j] = 0;
                j++;
            }
        }
    }
}

// walk views: half-grid centre + level/nchild, and the leaf/internal link
__global__ void k_tree_nodes(Cells c) {
    const uint32_t nc = c.lvl[kLevels + 1];
    for (size_t k = gtid(); k < nc; k += gstride()) {
        const uint32_t l = c.level[k];
        const uint64_t corner = c.prefix[k] << (3 * (kLevels - l));
        const uint32_t half = 1u << (kLevels - l);
        uint4 nd;
        nd.x = 2u * compact3(corner >> 2) + half;
        nd.y = 2u * compact3(corner >> 1) + half;
        nd.z = 2u * compact3(corner) + half;
        nd.w = l | (c.nchild[k] << 8);
        c.node[k] = nd;
        c.link[k] = c.nchild[k] ? make_uint2(c.first[k], c.count[k])
                                : make_uint2(c.begin[k], c.count[k]);
    }
}

// moments of the cells of one level (children already done)
__global__ void k_moments(int l, Cells c, const double4 *jp) {
    const uint32_t c0 = c.lvl[l], c1 = c.lvl[l + 1];
    for (size_t k = gtid(); k < c1 - c0; k += gstride()) {
        const uint32_t cid = c0 + (uint32_t)k;
        double M = 0, X = 0, Y = 0, Z = 0;
        double q[6] = {0, 0, 0, 0, 0, 0};
        const uint32_t nch = c.nchild[cid];
        if (nch == 0) {
            const uint32_t b = c.begin[cid], e = b + c.count[cid];
            double sx = 0, sy = 0, sz = 0;
            for (uint32_t i = b; i < e; i++) {
                double4 p = jp[i];
                M += p.w; sx += p.w * p.x; sy += p.w * p.y; sz += p.w * p.z;
            }
            if (M > 0) { X = sx / M; Y = sy / M; Z = sz / M; }
            for (uint32_t i = b; i < e; i++) {
                double4 p = jp[i];
                double dx = p.x - X, dy = p.y - Y, dz = p.z - Z;
                double d2 = dx * dx + dy * dy + dz * dz;
                q[0] += p.w * (3.0 * dx * dx - d2);
                q[1] += p.w * (3.0 * dy * dy - d2);
                q[2] += p.w * (3.0 * dz * dz - d2);
                q[3] += p.w * (3.0 * dx * dy);
                q[4] += p.w * (3.0 * dx * dz);
                q[5] += p.w * (3.0 * dy * dz);
            }
        } else {
            const uint32_t f = c.first[cid];
            double sx = 0, sy = 0, sz = 0;
            for (uint32_t j = f; j < f + nch; j++) {
                const double *o = c.mom + 10 * (size_t)j;
                M += o[0]; sx += o[0] * o[1]; sy += o[0] * o[2]; sz += o[0] * o[3];
            }
            if (M > 0) { X = sx / M; Y = sy / M; Z = sz / M; }
            for (uint32_t j = f; j < f + nch; j++) {
                const double *o = c.mom + 10 * (size_t)j;
                double dx = o[1] - X, dy = o[2] - Y, dz = o[3] - Z;
                double d2 = dx * dx + dy * dy + dz * dz;
                q[0] += o[4] + o[0] * (3.0 * dx * dx - d2);
                q[1] += o[5] + o[0] * (3.0 * dy * dy - d2);
                q[2] += o[6] + o[0] * (3.0 * dz * dz - d2);
                q[3] += o[7] + o[0] * (3.0 * dx * dy);
                q[4] += o[8] + o[0] * (3.0 * dx * dz);
                q[5] += o[9] + o[0] * (3.0 * dy * dz);
            }
        }
        double *o = c.mom + 10 * (size_t)cid;
        o[0] = M; o[1] = X; o[2] = Y; o[3] = Z;
#pragma unroll
        for (int a = 0; a < 6; a++) o[4 + a] = q[a];
    }
}

// Mark the first particle of every group: flag[r] = 1, gcell_at[r] = its cell.
__global__ void k_group_flags(Cells c, int n_group, uint32_t *flag, uint32_t *gcell_at) {
    const uint32_t nc = c.lvl[kLevels + 1];
    for (size_t k = gtid(); k < nc; k += gstride()) {
        const uint32_t cnt = c.count[k];
        if (cnt == 0) continue;
        const uint32_t par = c.parent[k];
        const bool maximal = par == kNone || c.count[par] > (uint32_t)n_group;
        if (!maximal) continue;
        const uint32_t b = c.begin[k];
        if (cnt <= (uint32_t)n_group) {
            flag[b] = 1; gcell_at[b] = (uint32_t)k;
        } else if (c.nchild[k] == 0) {          // over-full leaf: runs of n_group
            for (uint32_t o = 0; o < cnt; o += (uint32_t)n_group) {
                flag[b + o] = 1; gcell_at[b + o] = (uint32_t)k;
            }
        }
    }
}

__global__ void k_group_emit(size_t n, int n_group, Cells c, const uint32_t *flag,
                             const uint32_t *gcell_at, const uint32_t *gpos, Groups g) {
    for (size_t r = gtid(); r < n; r += gstride()) {
        if (!flag[r]) continue;
        const uint32_t gi = gpos[r], cell = gcell_at[r];
        if (gi >= g.cap) continue;             // host sees n_groups > cap and retries larger
        const uint32_t cb = c.begin[cell], cn = c.count[cell];
        uint32_t cnt = cn <= (uint32_t)n_group ? cn : min((uint32_t)n_group, cb + cn - (uint32_t)r);
        g.cell[gi] = cell;
        g.begin[gi] = (uint32_t)r;
        g.count[gi] = cnt;
    }
}

// One wave per group: integer box of the members' grid cells, centre of the group's cell,
// and the group's system.
__global__ void __launch_bounds__(kThreads)
k_group_geom(const uint32_t *ngroups, int nsys, const int64_t *off, Cells c,
             const uint64_t *skey, const double *cube, Groups g, DevStatus *st) {
    const uint32_t G = min(*ngroups, g.cap);
    if (gtid() == 0) {
        st->n_groups_c = G;
        if (*ngroups > g.cap) st->group_overflow = 1;
    }
    const int lane = lane_id();
    const size_t wave0 = gtid() / kWave, nwaves = gstride() / kWave;
    for (size_t gi = wave0; gi < G; gi += nwaves) {
        const uint32_t b = g.begin[gi], e = b + g.count[gi];
        uint32_t lo[3] = {kNone, kNone, kNone}, hi[3] = {0, 0, 0};
        for (uint32_t r = b + lane; r < e; r += kWave) {
            const uint64_t k = skey[r];
            const uint32_t q[3] = {compact3(k >> 2), compact3(k >> 1), compact3(k)};
#pragma unroll
            for (int a = 0; a < 3; a++) { lo[a] = min(lo[a], q[a]); hi[a] = max(hi[a], q[a]); }
        }
#pragma unroll
        for (int a = 0; a < 3; a++) { lo[a] = wave_min_u32(lo[a]); hi[a] = wave_max_u32(hi[a]); }
        if (lane == 0) {
            int slo = 0, shi = nsys - 1;               // last s with off[s] <= b
            while (slo < shi) {
                int mid = (slo + shi + 1) >> 1;
                if ((uint64_t)off[mid] <= b) slo = mid; else shi = mid - 1;
            }
            const uint32_t cell = g.cell[gi];
            const uint32_t l = c.level[cell];
            const uint64_t corner = c.prefix[cell] << (3 * (kLevels - l));
            const uint32_t cq[3] = {compact3(corner >> 2), compact3(corner >> 1), compact3(corner)};
            const double *cb = cube + 4 * slo;
            const double h = cb[3] / 4194304.0;        // half-grid unit: Lr / 2^22
            g.sys[gi] = (uint32_t)slo;
#pragma unroll
            for (int a = 0; a < 3; a++) {
                g.box[6 * gi + a] = lo[a];
                g.box[6 * gi + 3 + a] = hi[a];
                const double hg = (double)(2u * cq[a] + (1u << (kLevels - l)));
                g.centre[3 * gi + a] = __dadd_rn(cb[a], __dmul_rn(hg, h));
            }
        }
    }
}

}  // namespace

hipError_t pack_particles(size_t n, const double *x, const double *y, const double *z,
                          const double *m, double4 *packed, hipStream_t s) {
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_pack, dim3(grid_for(n)), dim3(kThreads), 0, s, n, x, y, z, m, packed);
    return hipGetLastError();
}

hipError_t gather_sorted(size_t n, const uint32_t *perm, const double4 *packed,
                         const double *eps, double eps_all, double4 *jp, double *seps,
                         uint32_t *inv, hipStream_t s) {
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_gather_sorted, dim3(grid_for(n)), dim3(kThreads), 0, s, n, perm, packed,
                       eps, eps_all, jp, seps, inv);
    return hipGetLastError();
}

hipError_t tree_build(size_t n, int nsys, const int64_t *sys_off, const uint64_t *skey,
                      int n_leaf, Cells c, uint32_t *tmp_n, uint32_t *tmp_off,
                      uint64_t *partial, DevStatus *st, hipStream_t s) {
    hipLaunchKernelGGL(k_tree_init, dim3((nsys + 255) / 256), dim3(256), 0, s, nsys, sys_off, c, st);
    // Level sizes are bounded by n (cells of one level are disjoint and non-empty, roots
    // aside), so the grids are sized from n and the kernels stride over the true size.
    const unsigned grid = grid_for(n + (size_t)nsys, 4096);
    uint32_t *total = tmp_off + (n + (size_t)nsys);  // one word past the offsets
    for (int l = 0; l < kLevels; l++) {
        hipLaunchKernelGGL(k_tree_split, dim3(grid), dim3(kThreads), 0, s, l, n_leaf, skey, c, tmp_n);
        hipError_t e = scan_u32_to_u32(tmp_n, tmp_off, 0, c.lvl + l, c.lvl + l + 1, partial,
                                       total, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_tree_emit, dim3(grid), dim3(kThreads), 0, s, l, skey, c, tmp_n,
                           tmp_off, total, st);
    }
    hipLaunchKernelGGL(k_tree_nodes, dim3(grid_for(c.cap, 8192)), dim3(kThreads), 0, s, c);
    return hipGetLastError();
}

hipError_t tree_moments(Cells c, const double4 *jp, hipStream_t s) {
    const unsigned grid = grid_for(c.cap, 4096);
    for (int l = kLevels; l >= 0; l--)
        hipLaunchKernelGGL(k_moments, dim3(grid), dim3(kThreads), 0, s, l, c, jp);
    return hipGetLastError();
}

hipError_t make_groups(size_t n, int nsys, const int64_t *sys_off, Cells c,
                       const uint64_t *skey, const double *cube, int n_group, Groups g,
                       uint32_t *flag, uint32_t *gcell_at, uint32_t *gpos, uint64_t *partial,
                       DevStatus *st, hipStream_t s) {
    hipError_t e = fill_u32(flag, 0u, n, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_group_flags, dim3(grid_for(c.cap, 8192)), dim3(kThreads), 0, s, c,
                       n_group, flag, gcell_at);
    e = scan_u32_to_u32(flag, gpos, n, nullptr, nullptr, partial, &st->n_groups, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_group_emit, dim3(grid_for(n)), dim3(kThreads), 0, s, n, n_group, c, flag,
                       gcell_at, gpos, g);
    hipLaunchKernelGGL(k_group_geom, dim3(grid_for(n / 16 + 64, 4096)), dim3(kThreads), 0, s,
                       &st->n_groups, nsys, sys_off, c, skey, cube, g, st);
    return hipGetLastError();
}

}  // namespace fdx
