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

// system holding sorted position r: the last s with off[s] <= r (skips empty systems)
__device__ __forceinline__ int system_of(const int64_t *off, int nsys, size_t r) {
    int lo = 0, hi = nsys - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((uint64_t)off[mid] <= r) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Sorted records, softenings and the inverse permutation.  The records are read from the
// (x, y, z, m) array the key kernel wrote in the caller's order (one 32-byte sector per
// particle instead of four scattered reads).  The sort keeps every system's
// particles in the same range [off[s], off[s + 1]) as the caller's layout, so when every
// system's particles share one softening (per_system) rank r takes it from the first particle
// of its system -- a cached read per system instead of a random read per particle.
__global__ void k_gather_sorted(size_t n, const uint32_t *perm, const double4 *packed,
                                const double *eps, double eps_all, int per_system,
                                const int64_t *off, int nsys, double4 *jp, double *seps,
                                uint32_t *inv) {
    for (size_t r = gtid(); r < n; r += gstride()) {
        const uint32_t i = perm[r];
        jp[r] = packed[i];
        seps[r] = per_system ? eps[off[system_of(off, nsys, r)]] : (eps ? eps[i] : eps_all);
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

// ---------------------------------------------------------------------------------------
// Topology from the sorted keys in O(N) work and a fixed number of launches.
//
// Two sorted keys of one system lie in the same level-L cell iff they share their first L
// octal digits; shared(a, b) = number of leading digits a and b have in common.  With
// lo(r) = shared(k[r-1], k[r]) + 1 (1 at the start of a system), a cell of level L >= 1 can
// start at sorted position r only if L >= lo(r).  It exists iff its parent (the level L-1
// cell holding r) has more than n_leaf particles and L <= 21.  The level-m cell holding r has
// more than n_leaf particles iff some window of n_leaf + 1 consecutive keys of the system
// that contains r shares m digits, so with c(a) = shared(k[a], k[a + n_leaf]) (-1 past the
// end of the system) and D(r) = max c(a) over a in [r - n_leaf, r] (within the system), the
// cells starting at r are exactly the levels L in [lo(r), hi(r)], hi(r) = min(D(r) + 1, 21).
// A cell (L, r) is split iff c(r) >= L and L < 21; its first child is then (L + 1, r).
// Breadth-first numbering (level by level, by position within a level) comes from one
// exclusive scan over per-wave-tile cell counts laid out level-major.
// ---------------------------------------------------------------------------------------

constexpr int kTileRounds = 16;                    // rounds of 64 positions per wave tile
constexpr int kTileW = kTileRounds * kWave;        // 1024 positions per wave tile

__device__ __forceinline__ int shared_levels(uint64_t a, uint64_t b) {
    const uint64_t x = a ^ b;                       // keys use the low 63 bits
    return x ? (__clzll((long long)x) - 1) / 3 : kLevels;
}

// per position: lo(r) and c(r)
__global__ void k_cells_prefix(size_t n, int nsys, const int64_t *off, const uint64_t *skey,
                               int n_leaf, uint8_t *lo8, int8_t *c8) {
    for (size_t r = gtid(); r < n; r += gstride()) {
        const int sys = system_of(off, nsys, r);
        const size_t s0 = (size_t)off[sys], s1 = (size_t)off[sys + 1];
        const uint64_t k = skey[r];
        lo8[r] = (uint8_t)(r == s0 ? 1 : shared_levels(skey[r - 1], k) + 1);
        c8[r] = (int8_t)(r + (size_t)n_leaf < s1 ? shared_levels(k, skey[r + n_leaf]) : -1);
    }
}

// per position hi(r); per wave tile and level, the number of cells starting in the tile:
// wcount[(L - 1) * ntiles + tile]
__global__ void __launch_bounds__(kThreads)
k_cells_count(size_t n, int nsys, const int64_t *off, int n_leaf, const uint8_t *lo8,
              const int8_t *c8, uint8_t *hi8, uint32_t ntiles, uint32_t *wcount) {
    const size_t tile = gtid() / kWave;
    if (tile >= ntiles) return;
    const int lane = lane_id();
    uint32_t cnt = 0;                              // lane L-1 counts level L
    for (int q = 0; q < kTileRounds; q++) {
        const size_t r = tile * kTileW + (size_t)q * kWave + lane;
        int lo = kLevels + 1, hi = 0;
        if (r < n) {
            const int sys = system_of(off, nsys, r);
            const size_t s0 = (size_t)off[sys];
            const size_t a0 = r >= s0 + (size_t)n_leaf ? r - (size_t)n_leaf : s0;
            int d = -1;
            for (size_t a = a0; a <= r; a++) d = max(d, (int)c8[a]);
            hi = min(d + 1, kLevels);
            lo = lo8[r];
            hi8[r] = (uint8_t)hi;
        }
        // levels present in this round: a ballot per level, counts kept by lane L-1
        const int lmin = (int)wave_min_u32((uint32_t)lo);
        const int lmax = (int)wave_max_u32((uint32_t)hi);
        for (int L = lmin; L <= lmax; L++) {
            const uint32_t c = (uint32_t)__popcll(__ballot(lo <= L && L <= hi));
            if (lane == L - 1) cnt += c;
        }
    }
    if (lane < kLevels) wcount[(size_t)lane * ntiles + tile] = cnt;
}

// level starts from the scanned counts; if the cells of every level do not fit the capacity,
// keep the levels that do (the deepest kept level's cells become leaves) and flag it
__global__ void k_cells_levels(int nsys, uint32_t ntiles, const uint32_t *woff,
                               const uint32_t *total, Cells c, DevStatus *st) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    uint32_t lv[kLevels + 2];
    lv[0] = 0;
    lv[1] = (uint32_t)nsys;
    for (int L = 1; L <= kLevels; L++) {
        const uint32_t nxt = L < kLevels ? woff[(size_t)L * ntiles] : *total;
        lv[L + 1] = (uint32_t)nsys + nxt;
    }
    int top = kLevels;
    while (top > 0 && lv[top + 1] > c.cap) top--;
    const bool ovf = top < kLevels && lv[kLevels + 1] > c.cap;
    for (int L = 0; L <= kLevels + 1; L++) c.lvl[L] = L <= top + 1 ? lv[L] : lv[top + 1];
    st->cell_overflow = ovf ? 1u : 0u;
    st->top_level = (uint32_t)top;
}

// write the cells of levels 1..top starting in each wave tile: level, prefix, begin, and
// first-child links (a split cell's first child starts at the same position one level down)
__global__ void __launch_bounds__(kThreads)
k_cells_emit(size_t n, int nsys, const int64_t *off, const uint64_t *skey, const uint8_t *lo8,
             const uint8_t *hi8, uint32_t ntiles, const uint32_t *woff, Cells c,
             const DevStatus *st) {
    const size_t tile = gtid() / kWave;
    if (tile >= ntiles) return;
    const int lane = lane_id();
    const uint64_t lt = lanemask_lt();
    const int top = (int)st->top_level;
    uint8_t lo[kTileRounds], hi[kTileRounds];
    uint32_t prev[kTileRounds];
    int lmin = kLevels + 1, lmax = 0;
#pragma unroll
    for (int q = 0; q < kTileRounds; q++) {
        const size_t r = tile * kTileW + (size_t)q * kWave + lane;
        lo[q] = r < n ? lo8[r] : (uint8_t)(kLevels + 1);
        hi[q] = r < n ? hi8[r] : (uint8_t)0;
        prev[q] = kNone;
        lmin = min(lmin, (int)lo[q]);
        lmax = max(lmax, (int)hi[q]);
    }
    lmin = (int)wave_min_u32((uint32_t)lmin);
    lmax = min((int)wave_max_u32((uint32_t)lmax), top);
    for (int L = lmin; L <= lmax; L++) {
        uint32_t run = (uint32_t)nsys + woff[(size_t)(L - 1) * ntiles + tile];
        const int sh = 3 * (kLevels - L);
#pragma unroll
        for (int q = 0; q < kTileRounds; q++) {
            const bool has = lo[q] <= L && L <= hi[q];
            const uint64_t b = __ballot(has);
            if (has) {
                const size_t r = tile * kTileW + (size_t)q * kWave + lane;
                const uint32_t idx = run + (uint32_t)__popcll(b & lt);
                c.level[idx] = (uint32_t)L;
                c.prefix[idx] = skey[r] >> sh;
                c.begin[idx] = (uint32_t)r;
                c.first[idx] = kNone;
                if (L > lo[q]) {
                    c.first[prev[q]] = idx;               // parent (L-1, r) was split
                } else if (L == 1) {
                    const int sys = system_of(off, nsys, r);
                    if ((size_t)off[sys] == r) c.first[sys] = idx;   // root split
                }
                prev[q] = idx;
            }
            run += (uint32_t)__popcll(b);
        }
    }
}

// per cell: particle count (end of the run of keys sharing the cell's L digits, found by a
// galloping search bounded by the system's end), children (the at most 8 cells of level
// L + 1 from the first child on that start before the end) and their parent link, and the
// walk views (half-grid centre + level/nchild, leaf or internal link)
__global__ void k_cells_finish(int nsys, const int64_t *off, const uint64_t *skey, Cells c) {
    const uint32_t nc = c.lvl[kLevels + 1];
    for (size_t k = gtid(); k < nc; k += gstride()) {
        const uint32_t cid = (uint32_t)k;
        const uint32_t L = c.level[cid];
        const uint32_t b = c.begin[cid];
        uint32_t cnt;
        if (cid < (uint32_t)nsys) {
            cnt = c.count[cid];
        } else {
            const int sys = system_of(off, nsys, b);
            const uint32_t s1 = (uint32_t)off[sys + 1];
            const uint64_t kb = skey[b];
            // last position known inside (in) and first known outside or at the end (out)
            uint32_t in = b, out = s1;
            for (uint64_t step = 1; (uint64_t)in + step < s1; step <<= 1) {
                const uint32_t pr = in + (uint32_t)step;
                if (shared_levels(skey[pr], kb) < (int)L) { out = pr; break; }
                in = pr;
            }
            while (out - in > 1) {
                const uint32_t mid = in + (out - in) / 2;
                if (shared_levels(skey[mid], kb) >= (int)L) in = mid; else out = mid;
            }
            cnt = out - b;
            c.count[cid] = cnt;
        }
        const uint32_t first = c.first[cid];
        uint32_t nch = 0;
        if (first != kNone && L + 2 <= (uint32_t)kLevels + 1) {
            const uint32_t e = b + cnt, lim = min(first + 8u, c.lvl[L + 2]);
            for (uint32_t j = first; j < lim && c.begin[j] < e; j++) {
                c.parent[j] = cid;
                nch++;
            }
        }
        c.nchild[cid] = nch;
        const uint64_t corner = c.prefix[cid] << (3 * (kLevels - L));
        const uint32_t half = 1u << (kLevels - L);
        uint4 nd;
        nd.x = 2u * compact3(corner >> 2) + half;
        nd.y = 2u * compact3(corner >> 1) + half;
        nd.z = 2u * compact3(corner) + half;
        nd.w = L | (nch << 8);
        c.node[cid] = nd;
        c.link[cid] = nch ? make_uint2(first, cnt) : make_uint2(b, cnt);
    }
}

// Moments of one cell: a leaf from its particles, an internal cell from its children (in
// child order).  One pass over the cell's particles (leaf) or children (internal cell), about a reference
// point inside the cell -- the first particle, or the first child's centre of mass -- so the
// offsets are bounded by the cell's size:
//   M = sum m,  s = sum m r,  T = sum m r r^T (+ the children's own Q),  r = x - ref;
//   X = ref + s / M,  A = T - M d d^T with d = s / M,  Q = 3 A - tr(A) I (traceless, about X).
// A massless cell gets X = 0 and Q = 0.
__device__ void cell_moments(const Cells &c, const double4 *jp, uint32_t cid) {
    double M = 0, sx = 0, sy = 0, sz = 0;
    double txx = 0, tyy = 0, tzz = 0, txy = 0, txz = 0, tyz = 0;
    double q[6] = {0, 0, 0, 0, 0, 0};
    double rx = 0, ry = 0, rz = 0;
    const uint32_t nch = c.nchild[cid];
    auto add = [&](double m, double x, double y, double z) {
        const double dx = x - rx, dy = y - ry, dz = z - rz;
        const double mx = m * dx, my = m * dy, mz = m * dz;
        M += m; sx += mx; sy += my; sz += mz;
        txx += mx * dx; tyy += my * dy; tzz += mz * dz;
        txy += mx * dy; txz += mx * dz; tyz += my * dz;
    };
    if (nch == 0) {
        const uint32_t b = c.begin[cid], e = b + c.count[cid];
        if (e > b) {
            const double4 p0 = jp[b];
            rx = p0.x; ry = p0.y; rz = p0.z;
        }
        // chunks of 8 with every load of a chunk issued before its sums (leaves hold at most
        // n_leaf particles, except at the deepest level)
        for (uint32_t i0 = b; i0 < e; i0 += 8) {
            double4 p[8];
#pragma unroll
            for (int k = 0; k < 8; k++) p[k] = jp[i0 + k < e ? i0 + k : b];   // in range
#pragma unroll
            for (int k = 0; k < 8; k++)
                if (i0 + k < e) add(p[k].w, p[k].x, p[k].y, p[k].z);
        }
    } else {
        const uint32_t f = c.first[cid];
        const double2 *m0 = reinterpret_cast<const double2 *>(c.mom + 10 * (size_t)f);
        const double2 x01 = m0[0], x23 = m0[1];
        rx = x01.y; ry = x23.x; rz = x23.y;
        // at most 8 children: their records are loaded together, then summed in order
        double2 a[8], bb[8];
#pragma unroll
        for (uint32_t k = 0; k < 8; k++) {
            const uint32_t j = k < nch ? f + k : f;                          // in range
            const double2 *o = reinterpret_cast<const double2 *>(c.mom + 10 * (size_t)j);
            a[k] = o[0];
            bb[k] = o[1];
        }
#pragma unroll
        for (uint32_t k = 0; k < 8; k++)
            if (k < nch) add(a[k].x, a[k].y, bb[k].x, bb[k].y);
#pragma unroll
        for (uint32_t k = 0; k < 8; k++) {
            if (k < nch) {
                const double2 *o = reinterpret_cast<const double2 *>(c.mom + 10 * (size_t)(f + k));
                const double2 cq = o[2], dq = o[3], eq = o[4];
                q[0] += cq.x; q[1] += cq.y; q[2] += dq.x; q[3] += dq.y; q[4] += eq.x;
                q[5] += eq.y;
            }
        }
    }
    double X = 0, Y = 0, Z = 0;
    if (M > 0) {
        const double dx = sx / M, dy = sy / M, dz = sz / M;
        X = rx + dx; Y = ry + dy; Z = rz + dz;
        const double axx = txx - sx * dx, ayy = tyy - sy * dy, azz = tzz - sz * dz;
        const double axy = txy - sx * dy, axz = txz - sx * dz, ayz = tyz - sy * dz;
        const double tr = axx + ayy + azz;
        q[0] += 3.0 * axx - tr; q[1] += 3.0 * ayy - tr; q[2] += 3.0 * azz - tr;
        q[3] += 3.0 * axy; q[4] += 3.0 * axz; q[5] += 3.0 * ayz;
    }
    double2 *o = reinterpret_cast<double2 *>(c.mom + 10 * (size_t)cid);
    o[0] = make_double2(M, X);
    o[1] = make_double2(Y, Z);
    o[2] = make_double2(q[0], q[1]);
    o[3] = make_double2(q[2], q[3]);
    o[4] = make_double2(q[4], q[5]);
}

// moments of the cells of one level (children already done)
__global__ void k_moments(int l, Cells c, const double4 *jp) {
    const uint32_t c0 = c.lvl[l], c1 = c.lvl[l + 1];
    for (size_t k = gtid(); k < c1 - c0; k += gstride()) cell_moments(c, jp, c0 + (uint32_t)k);
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

// level of every particle's leaf (leaves partition the particles)
__global__ void k_leaf_level(Cells c, uint8_t *plev) {
    const uint32_t nc = min(c.lvl[kLevels + 1], c.cap);
    for (size_t k = gtid(); k < nc; k += gstride()) {
        if (c.nchild[k] != 0) continue;
        const uint32_t b = c.begin[k], e = b + c.count[k];
        const uint8_t l = (uint8_t)c.level[k];
        for (uint32_t r = b; r < e; r++) plev[r] = l;
    }
}

// groups flagged wide, appended in any order (each is evaluated on its own); the counter
// starts from zero
__global__ void k_wide_list(const uint32_t *ngroups_c, Groups g, uint32_t *list, DevStatus *st) {
    const uint32_t G = *ngroups_c;
    for (size_t gi = gtid(); gi < G; gi += gstride())
        if (g.wide[gi]) list[atomicAdd(&st->wide_groups, 1u)] = (uint32_t)gi;
}

// Per group: the integer box of its members' keys, its deepest member leaf level, its smallest
// softening, its system, the centre of its cell and the wide flag.  Four groups per wave, one
// per 16-lane row: the members are read 16 at a time, the reductions are four DPP lane moves
// within the row (the row's last lane ends up with the row's result), and the rows' last lanes
// write the four groups in parallel.  Median groups hold a few tens of particles, so one group
// per wave left most lanes idle and spent six reduction steps and a one-lane epilogue on each.
__global__ void __launch_bounds__(kThreads)
k_group_geom(const uint32_t *ngroups, int nsys, const int64_t *off, Cells c,
             const uint64_t *skey, const double *cube, const double *seps, const uint8_t *plev,
             Groups g, DevStatus *st) {
    const uint32_t G = min(*ngroups, g.cap);
    if (gtid() == 0) {
        st->n_groups_c = G;
        if (*ngroups > g.cap) st->group_overflow = 1;
    }
    const int lane = lane_id();
    const int row = lane >> 4, rl = lane & 15;
    const size_t wave0 = gtid() / kWave, nwaves = gstride() / kWave;
    // wave-uniform trip count: every lane reaches the row reductions below
    for (size_t g0 = 4 * wave0; g0 < G; g0 += 4 * nwaves) {
        const size_t gi = g0 + (size_t)row;
        const bool valid = gi < G;
        const uint32_t b = valid ? g.begin[gi] : 0u;
        const uint32_t e = valid ? b + g.count[gi] : 0u;
        uint32_t lo[3] = {kNone, kNone, kNone}, hi[3] = {0, 0, 0};
        uint32_t deep = 0;
        double emin = INFINITY;
        for (uint32_t r = b + (uint32_t)rl; r < e; r += 16) {
            const uint64_t k = skey[r];
            const uint32_t q[3] = {compact3(k >> 2), compact3(k >> 1), compact3(k)};
#pragma unroll
            for (int a = 0; a < 3; a++) { lo[a] = min(lo[a], q[a]); hi[a] = max(hi[a], q[a]); }
            deep = max(deep, (uint32_t)plev[r]);
            emin = fmin(emin, seps[r]);
        }
#pragma unroll
        for (int a = 0; a < 3; a++) { lo[a] = row_min_u32(lo[a]); hi[a] = row_max_u32(hi[a]); }
        deep = row_max_u32(deep);
        emin = row_min_nonneg_f64(emin);
        if (valid && rl == 15) {
            const int slo = system_of(off, nsys, b);      // last s with off[s] <= b
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
            // wide: 9 u min(S / eps_min, 2^d) > 1e-4 with u = 2^-24
            const double side = ldexp(cb[3], -(int)l);
            const double span = ldexp(1.0, (int)deep - (int)l);
            const double m = fmin(side / emin, span);
            g.wide[gi] = (9.0 * 5.9604644775390625e-8) * m > 1e-4 ? 1u : 0u;
        }
    }
}

}  // namespace

hipError_t gather_sorted(size_t n, const uint32_t *perm, const double4 *packed,
                         const double *eps, double eps_all, bool per_system, const int64_t *off,
                         int nsys, double4 *jp, double *seps, uint32_t *inv, hipStream_t s) {
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_gather_sorted, dim3(grid_for(n)), dim3(kThreads), 0, s, n, perm, packed,
                       eps, eps_all, (per_system && eps) ? 1 : 0, off, nsys, jp, seps, inv);
    return hipGetLastError();
}

size_t tree_scratch_u32(size_t n) {
    const size_t ntiles = (n + kTileW - 1) / kTileW;
    return 2 * (size_t)kLevels * (ntiles ? ntiles : 1) + 2;
}

hipError_t tree_build(size_t n, int nsys, const int64_t *sys_off, const uint64_t *skey,
                      int n_leaf, Cells c, uint8_t *bytes, uint32_t *scratch,
                      uint64_t *partial, DevStatus *st, hipStream_t s) {
    hipLaunchKernelGGL(k_tree_init, dim3((nsys + 255) / 256), dim3(256), 0, s, nsys, sys_off, c, st);
    const size_t ntiles = (n + kTileW - 1) / kTileW;
    uint8_t *lo8 = bytes, *hi8 = bytes + n;
    int8_t *c8 = (int8_t *)(bytes + 2 * n);
    uint32_t *wcount = scratch, *woff = scratch + (size_t)kLevels * ntiles;
    uint32_t *total = woff + (size_t)kLevels * ntiles;
    if (n) {
        hipLaunchKernelGGL(k_cells_prefix, dim3(grid_for(n)), dim3(kThreads), 0, s, n, nsys,
                           sys_off, skey, n_leaf, lo8, c8);
        const unsigned tb = (unsigned)((ntiles * kWave + kThreads - 1) / kThreads);
        hipLaunchKernelGGL(k_cells_count, dim3(tb), dim3(kThreads), 0, s, n, nsys, sys_off,
                           n_leaf, lo8, c8, hi8, (uint32_t)ntiles, wcount);
        hipError_t e = scan_u32_to_u32(wcount, woff, (size_t)kLevels * ntiles, nullptr, nullptr,
                                       partial, total, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_cells_levels, dim3(1), dim3(64), 0, s, nsys, (uint32_t)ntiles, woff,
                           total, c, st);
        hipLaunchKernelGGL(k_cells_emit, dim3(tb), dim3(kThreads), 0, s, n, nsys, sys_off, skey,
                           lo8, hi8, (uint32_t)ntiles, woff, c, st);
    }
    hipLaunchKernelGGL(k_cells_finish, dim3(grid_for(c.cap, 8192)), dim3(kThreads), 0, s, nsys,
                       sys_off, skey, c);
    return hipGetLastError();
}

hipError_t tree_moments(Cells c, const double4 *jp, hipStream_t s) {
    const unsigned grid = grid_for(c.cap, 4096);
    for (int l = kLevels; l >= 0; l--)
        hipLaunchKernelGGL(k_moments, dim3(grid), dim3(kThreads), 0, s, l, c, jp);
    return hipGetLastError();
}

hipError_t make_groups(size_t n, int nsys, const int64_t *sys_off, Cells c,
                       const uint64_t *skey, const double *cube, const double *seps,
                       int n_group, Groups g, uint32_t *flag, uint32_t *gcell_at, uint32_t *gpos,
                       uint8_t *plev, uint64_t *partial, DevStatus *st, hipStream_t s) {
    hipError_t e = fill_u32(flag, 0u, n, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_group_flags, dim3(grid_for(c.cap, 8192)), dim3(kThreads), 0, s, c,
                       n_group, flag, gcell_at);
    e = scan_u32_to_u32(flag, gpos, n, nullptr, nullptr, partial, &st->n_groups, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_group_emit, dim3(grid_for(n)), dim3(kThreads), 0, s, n, n_group, c, flag,
                       gcell_at, gpos, g);
    hipLaunchKernelGGL(k_leaf_level, dim3(grid_for(c.cap, 8192)), dim3(kThreads), 0, s, c, plev);
    hipLaunchKernelGGL(k_group_geom, dim3(grid_for(n / 16 + 64, 4096)), dim3(kThreads), 0, s,
                       &st->n_groups, nsys, sys_off, c, skey, cube, seps, plev, g, st);
    return hipGetLastError();
}

hipError_t wide_group_list(size_t gmax, const Groups g, uint32_t *list, DevStatus *st,
                           hipStream_t s) {
    hipError_t e = fill_u32(&st->wide_groups, 0u, 1, s);
    if (e == hipSuccess) e = fill_u32(&st->queue_head, 0u, 1, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_wide_list, dim3(grid_for(gmax + 1, 4096)), dim3(kThreads), 0, s,
                       &st->n_groups_c, g, list, st);
    return hipGetLastError();
}

}  // namespace fdx
