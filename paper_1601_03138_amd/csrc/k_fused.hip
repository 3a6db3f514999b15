// Walk and force in one persistent launch: the paper's "multiwalk" for accelerators (section
// "Design concept of FDPS": many groups' interaction lists evaluated by one accelerator call)
// taken to the point where the lists are never stored.
//
// Every wave works on its own: it pops a group from its XCD's queue, walks the tree for it
// exactly as the walk kernel does (a per-wave LDS stack, up to 64 cells tested per iteration,
// the same opening test, so the same entries in the same order), and keeps the entries the
// walk emits in small per-wave LDS buffers -- superparticles as cell ids, particles as ranges
// of sorted ranks (an opened leaf is one contiguous range).  Whenever 64 entries of a kind are
// pending they are evaluated as one tile: each lane gathers one entry's j-data into the wave's
// LDS tile (FP32 relative to the group's centre, or FP64), then the lanes, split into
// floor(64 / ceil(n_i / IPL)) slices of i-particles with IPL i-particles per lane (IPL = 1, 2
// or 4, whichever keeps the most lanes busy for this group), sum the tile's interactions; tile
// sums are added into FP64 accumulators.  At the end of the walk the partial tiles are
// evaluated, the slices are combined in slice order and the group's rows are written.  No
// workgroup barrier is used: the four waves of a workgroup are independent, and the walk's
// latency hides behind the arithmetic of the other waves on the SIMD.
//
// The queue: the groups in tree order are cut into eight runs, one per XCD, at equal
// cumulative cost (bounds[0..8]); cost = members x predicted list length when the learned
// predictor is used (no walk precedes this kernel, so list lengths are not known), else the
// members alone.  A wave pops its own XCD's run and then takes slots from the others'.
// Results do not depend on the queue: each group is evaluated by one wave in a fixed order.
#include "dev_util.h"
#include "fdx_internal.h"
#include "interact.h"
#include "opening.h"

namespace fdx {

namespace {

constexpr int kFT = 256;                 // threads per workgroup: four independent waves
constexpr int kFW = kFT / kWave;
constexpr int kStack = 512;              // per-wave walk stack (entries)
constexpr int kSlack = 160;              // stack entries kept free for sequential descent
constexpr int kTile = 64;                // entries per evaluated tile (one per lane)

template <class T>
struct WaveMem {
    using V = typename V4<T>::t;
    uint32_t stk[kStack];
    uint32_t spj[2 * kTile];             // pending superparticle cell ids
    uint32_t rpre[2 * kTile];            // exclusive prefix of the pending ranges' counts
    uint2 rng[2 * kTile];                // pending particle ranges {first rank, count}
    union {
        V t[3 * kTile];                  // tile: particles 1 record, superparticles 3
        double red[4 * kTile];           // slice partials at the end of a group
    } u;
};

// the tile's interactions with the first IPL of the lane's i-particle slots
template <class T, bool QUAD, int IPL>
__device__ __forceinline__ void eval_tile(const WaveMem<T> &wm, bool spj_tile, uint32_t nt,
                                          uint32_t nslice, uint32_t slice, bool active,
                                          const T *xi, const T *yi, const T *zi, const T *e2,
                                          double *ax, double *ay, double *az, double *ph) {
    using V = typename V4<T>::t;
    if (!active) return;
    T tx[IPL], ty[IPL], tz[IPL], tp[IPL];
#pragma unroll
    for (int k = 0; k < IPL; k++) tx[k] = ty[k] = tz[k] = tp[k] = 0;
    // a contiguous run of kmain entries per slice, then the leftover entries one per slice
    const uint32_t kmain = nt / nslice;
    const uint32_t j1 = kmain * nslice + slice;
    if (!spj_tile) {
        const V *run = wm.u.t + slice * kmain;
#pragma unroll 4
        for (uint32_t q = 0; q < kmain; q++) {
            const V J = run[q];
#pragma unroll
            for (int k = 0; k < IPL; k++)
                pp<T>(J, xi[k], yi[k], zi[k], e2[k], tx[k], ty[k], tz[k], tp[k]);
        }
        if (j1 < nt) {
            const V J = wm.u.t[j1];
#pragma unroll
            for (int k = 0; k < IPL; k++)
                pp<T>(J, xi[k], yi[k], zi[k], e2[k], tx[k], ty[k], tz[k], tp[k]);
        }
    } else {
        const V *run = wm.u.t + 3 * slice * kmain;
#pragma unroll 1
        for (uint32_t q = 0; q < kmain; q++) {
            const V A = run[3 * q];
            V B, C;
            if (QUAD) { B = run[3 * q + 1]; C = run[3 * q + 2]; } else { B = A; C = A; }
#pragma unroll
            for (int k = 0; k < IPL; k++)
                pc<T, QUAD>(A, B, C, xi[k], yi[k], zi[k], e2[k], tx[k], ty[k], tz[k], tp[k]);
        }
        if (j1 < nt) {
            const V A = wm.u.t[3 * j1];
            V B, C;
            if (QUAD) { B = wm.u.t[3 * j1 + 1]; C = wm.u.t[3 * j1 + 2]; } else { B = A; C = A; }
#pragma unroll
            for (int k = 0; k < IPL; k++)
                pc<T, QUAD>(A, B, C, xi[k], yi[k], zi[k], e2[k], tx[k], ty[k], tz[k], tp[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < IPL; k++) {
        ax[k] += (double)tx[k]; ay[k] += (double)ty[k]; az[k] += (double)tz[k];
        ph[k] += (double)tp[k];
    }
}

// IPL of this group (1, 2 or 4; wave-uniform) with slots for IPLMAX
template <class T, bool QUAD, int IPLMAX>
__device__ __forceinline__ void eval_tile_ipl(uint32_t ipl, const WaveMem<T> &wm, bool spj_tile,
                                              uint32_t nt, uint32_t nslice, uint32_t slice,
                                              bool active, const T *xi, const T *yi,
                                              const T *zi, const T *e2, double *ax, double *ay,
                                              double *az, double *ph) {
    if (ipl == 1)
        eval_tile<T, QUAD, 1>(wm, spj_tile, nt, nslice, slice, active, xi, yi, zi, e2, ax, ay, az,
                              ph);
    else if (ipl == 2 || IPLMAX < 4)
        eval_tile<T, QUAD, 2>(wm, spj_tile, nt, nslice, slice, active, xi, yi, zi, e2, ax, ay, az,
                              ph);
    else
        eval_tile<T, QUAD, (IPLMAX >= 4 ? 4 : 2)>(wm, spj_tile, nt, nslice, slice, active, xi, yi,
                                                  zi, e2, ax, ay, az, ph);
}

// One group: walk, tiles as the walk emits them, final tiles, rows.  One copy of this body per
// kernel; only the tile evaluation is specialised for the group's IPL.
template <class T, bool QUAD, int IPLMAX>
__device__ __forceinline__ void fused_group(const FusedArgs &a, uint32_t gi, uint32_t ni,
                                            uint32_t ipl, WaveMem<T> &wm) {
    constexpr int IPL = IPLMAX;          // register slots per lane
    using V = typename V4<T>::t;
    const int lane = lane_id();
    const uint64_t lt = lanemask_lt();
    const Groups &g = a.g;
    const uint32_t gb = (uint32_t)__builtin_amdgcn_readfirstlane((int)g.begin[gi]);
    const bool fp32 = sizeof(T) == 4;
    // the group's values are the same in every lane: held in scalar registers
    const double cx = fp32 ? uniform_f64(g.centre[3 * (size_t)gi]) : 0.0;
    const double cy = fp32 ? uniform_f64(g.centre[3 * (size_t)gi + 1]) : 0.0;
    const double cz = fp32 ? uniform_f64(g.centre[3 * (size_t)gi + 2]) : 0.0;

    uint32_t tps = (ni + ipl - 1) / ipl;
    tps = tps < 1 ? 1 : (tps > (uint32_t)kWave ? (uint32_t)kWave : tps);
    const uint32_t nslice = kWave / tps;
    const uint32_t slice = (uint32_t)lane / tps, li = (uint32_t)lane % tps;
    const bool active = slice < nslice;

    T xi[IPL], yi[IPL], zi[IPL], e2[IPL];
    double ax[IPL], ay[IPL], az[IPL], ph[IPL];
#pragma unroll
    for (int k = 0; k < IPL; k++) {
        const uint32_t i = li + k * tps;
        const uint32_t r = gb + (i < ni ? i : 0);
        const double4 p = a.jp[r];
        xi[k] = (T)(p.x - cx); yi[k] = (T)(p.y - cy); zi[k] = (T)(p.z - cz);
        const double e = a.seps[r];
        e2[k] = (T)(e * e);
        ax[k] = ay[k] = az[k] = ph[k] = 0.0;
    }

    // list capture (checks): EPJ from the front of the group's segment, SPJ from its back
    uint64_t lbase = 0;
    uint32_t lcap = 0;
    if (a.list) {
        lbase = (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)a.seg[gi]) |
                ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(a.seg[gi] >> 32)) << 32);
        lcap = (uint32_t)__builtin_amdgcn_readfirstlane((int)a.cap[gi]);
    }

    const uint32_t *bx = g.box + 6 * (size_t)gi;
    const int bminx = 2 * (int)uniform_u32(bx[0]), bminy = 2 * (int)uniform_u32(bx[1]);
    const int bminz = 2 * (int)uniform_u32(bx[2]);
    const int bmaxx = 2 * (int)uniform_u32(bx[3]) + 2, bmaxy = 2 * (int)uniform_u32(bx[4]) + 2;
    const int bmaxz = 2 * (int)uniform_u32(bx[5]) + 2;

    // wave-uniform bookkeeping
    uint32_t ns_p = 0, ne_p = 0, nr = 0;         // pending superparticles, particles, ranges
    uint32_t ns_tot = 0, ne_tot = 0;             // entries evaluated so far
    uint32_t sp = 1;
    bool err = false;

    // the tile evaluators
    auto spj_tile = [&](uint32_t nt) {
        if ((uint32_t)lane < nt) {
            const uint32_t id = wm.spj[lane];
            const double *o = a.mom + 10 * (size_t)id;
            V A;
            A.x = (T)(o[1] - cx); A.y = (T)(o[2] - cy); A.z = (T)(o[3] - cz); A.w = (T)o[0];
            wm.u.t[3 * lane] = A;
            if (QUAD) {
                V B, C;
                B.x = (T)o[4]; B.y = (T)o[5]; B.z = (T)o[6]; B.w = (T)o[7];
                C.x = (T)o[8]; C.y = (T)o[9]; C.z = 0; C.w = 0;
                wm.u.t[3 * lane + 1] = B;
                wm.u.t[3 * lane + 2] = C;
            }
            if (a.list && ns_tot + lane < lcap) a.list[lbase + lcap - 1 - (ns_tot + lane)] = id;
        }
        wave_barrier();
        eval_tile_ipl<T, QUAD, IPLMAX>(ipl, wm, true, nt, nslice, slice, active, xi, yi, zi, e2,
                                       ax, ay, az, ph);
        wave_barrier();
        ns_tot += nt;
    };
    auto epj_tile = [&](uint32_t nt) {
        if ((uint32_t)lane < nt) {
            // the range holding pending position `lane`: the last r with rpre[r] <= lane
            uint32_t lo = 0, hi = nr - 1;
            while (lo < hi) {
                const uint32_t mid = (lo + hi + 1) >> 1;
                if (wm.rpre[mid] <= (uint32_t)lane) lo = mid; else hi = mid - 1;
            }
            const uint32_t idx = wm.rng[lo].x + ((uint32_t)lane - wm.rpre[lo]);
            const double4 p = a.jp[idx];
            V v;
            v.x = (T)(p.x - cx); v.y = (T)(p.y - cy); v.z = (T)(p.z - cz); v.w = (T)p.w;
            wm.u.t[lane] = v;
            if (a.list && ne_tot + lane < lcap) a.list[lbase + ne_tot + lane] = idx;
        }
        wave_barrier();
        eval_tile_ipl<T, QUAD, IPLMAX>(ipl, wm, false, nt, nslice, slice, active, xi, yi, zi, e2,
                                       ax, ay, az, ph);
        wave_barrier();
        ne_tot += nt;
    };

    if (lane == 0) wm.stk[0] = g.sys[gi];            // roots are cells 0..nsys-1
    wave_barrier();
    while (sp > 0) {
        int room = kStack - kSlack - (int)sp;
        uint32_t p = min(64u, sp);
        if (room < 7 * (int)p) p = room >= 7 ? (uint32_t)(room / 7) : 1u;
        const bool act = (uint32_t)lane < p;
        uint32_t cid = 0;
        if (act) cid = wm.stk[sp - p + lane];
        if (__ballot(act && cid >= a.ccap)) { err = true; break; }   // never: stack intact
        wave_barrier();
        sp -= p;
        const uint4 nd = a.node[cid];
        const uint2 lk = a.link[cid];
        const uint32_t nch = nd.w >> 8;
        const bool accept =
            act && cell_accepted(nd, bminx, bminy, bminz, bmaxx, bmaxy, bmaxz, a.theta2);
        const bool open = act && !accept;
        const bool leaf = open && nch == 0 && lk.y > 0;
        const bool inner = open && nch != 0;
        // superparticles: appended to the pending ids (fewer than 64 were pending)
        const uint64_t bs = __ballot(accept);
        if (accept) wm.spj[ns_p + (uint32_t)__popcll(bs & lt)] = cid;
        ns_p += (uint32_t)__popcll(bs);
        // opened leaves: appended as ranges; children of opened cells: pushed
        const uint32_t lc = leaf ? lk.y : 0u;
        const uint32_t cc = inner ? nch : 0u;
        uint32_t lex, ltot, cex, ctot;
        if (__ballot(lc >= (1u << 16)) == 0) {
            const uint32_t pk = lc | (cc << 22);
            const uint32_t inc = wave_incl_scan_dpp(pk);
            const uint32_t tot = (uint32_t)__builtin_amdgcn_readlane((int)inc, kWave - 1);
            const uint32_t ex = inc - pk;
            lex = ex & 0x3FFFFFu; cex = ex >> 22;
            ltot = tot & 0x3FFFFFu; ctot = tot >> 22;
        } else {
            const uint32_t li2 = wave_incl_scan_dpp(lc), ci = wave_incl_scan_dpp(cc);
            ltot = (uint32_t)__builtin_amdgcn_readlane((int)li2, kWave - 1);
            ctot = (uint32_t)__builtin_amdgcn_readlane((int)ci, kWave - 1);
            lex = li2 - lc; cex = ci - cc;
        }
        const uint64_t bl = __ballot(leaf);
        if (leaf) {
            const uint32_t k = nr + (uint32_t)__popcll(bl & lt);
            wm.rng[k] = make_uint2(lk.x, lk.y);
            wm.rpre[k] = ne_p + lex;
        }
        nr += (uint32_t)__popcll(bl);
        ne_p += ltot;
        if (sp + ctot > (uint32_t)kStack) { err = true; break; }
        if (inner) {
            uint32_t *d = wm.stk + sp + cex;
#pragma unroll
            for (uint32_t k = 0; k < 8; k++)
                if (k < cc) d[k] = lk.x + k;
        }
        sp += ctot;
        wave_barrier();
        // full tiles
        while (ns_p >= (uint32_t)kTile) {
            spj_tile(kTile);
            // the pending ids past the tile move to the front (reads >= 64, writes < 64)
            const uint32_t rest = ns_p - kTile;
            if ((uint32_t)lane < rest) wm.spj[lane] = wm.spj[kTile + lane];
            ns_p = rest;
            wave_barrier();
        }
        while (ne_p >= (uint32_t)kTile) {
            epj_tile(kTile);
            // drop the ranges the tile used up, trim the one it cut, shift the rest down
            uint2 rv[2];
            uint32_t pv[2];
            bool keep[2];
#pragma unroll
            for (int h = 0; h < 2; h++) {
                const uint32_t r = (uint32_t)lane + h * kWave;
                keep[h] = false;
                if (r < nr) {
                    rv[h] = wm.rng[r];
                    pv[h] = wm.rpre[r];
                    keep[h] = pv[h] + rv[h].y > (uint32_t)kTile;
                    if (pv[h] < (uint32_t)kTile) {
                        const uint32_t used = kTile - pv[h];
                        rv[h].x += used; rv[h].y -= used; pv[h] = 0;
                    } else {
                        pv[h] -= kTile;
                    }
                }
            }
            const uint32_t dropped = (uint32_t)__popcll(__ballot(((uint32_t)lane < nr) && !keep[0])) +
                                     (uint32_t)__popcll(__ballot(((uint32_t)lane + kWave < nr) && !keep[1]));
            wave_barrier();
#pragma unroll
            for (int h = 0; h < 2; h++) {
                if (keep[h]) {
                    const uint32_t r = (uint32_t)lane + h * kWave - dropped;
                    wm.rng[r] = rv[h];
                    wm.rpre[r] = pv[h];
                }
            }
            nr -= dropped;
            ne_p -= kTile;
            wave_barrier();
        }
    }
    wave_barrier();
    if (!err) {
        if (ns_p) spj_tile(ns_p);
        if (ne_p) epj_tile(ne_p);
    }
    // combine the slices in slice order, remove the self term of the potential, write rows
#pragma unroll
    for (int k = 0; k < IPL; k++) {
        if ((uint32_t)k >= ipl) break;
        wave_barrier();
        wm.u.red[lane] = ax[k];
        wm.u.red[kWave + lane] = ay[k];
        wm.u.red[2 * kWave + lane] = az[k];
        wm.u.red[3 * kWave + lane] = ph[k];
        wave_barrier();
        const uint32_t i = li + k * tps;
        if (slice == 0 && i < ni) {
            double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
            for (uint32_t q = 0; q < nslice; q++) {
                const uint32_t l = q * tps + li;
                s0 += wm.u.red[l]; s1 += wm.u.red[kWave + l];
                s2 += wm.u.red[2 * kWave + l]; s3 += wm.u.red[3 * kWave + l];
            }
            const uint32_t r = gb + i;
            const T mi = (T)a.jp[r].w;
            const T self = mi * rsqrt_t(e2[k]);
            a.fs[r] = make_double4(s0, s1, s2, s3 + (double)self);
        }
    }
    wave_barrier();
    if (lane == 0) {
        a.cnt_e[gi] = ne_tot;
        a.cnt_s[gi] = ns_tot;
    }
    if (err && lane == 0) atomicOr(&a.st->walk_error, 1u);
    if (a.list && (uint64_t)ne_tot + ns_tot > lcap && lane == 0)
        atomicAdd(&a.st->list_overflow, 1u);
}

// lanes kept busy per i-particle slot, n_i x slices / (64 x IPL), times 64 x 4 (an integer,
// so the choice below is exact)
__device__ __forceinline__ uint32_t ipl_fill(uint32_t ni, uint32_t ipl) {
    uint32_t tps = (ni + ipl - 1) / ipl;
    if (tps < 1) tps = 1;
    if (tps > (uint32_t)kWave) return 0u;
    return ni * (kWave / tps) * (4u / ipl);
}

// IPL in {1, 2, 4 (if allowed)} with the most lanes busy; ties go to the smaller
__device__ __forceinline__ uint32_t best_ipl(uint32_t ni, int iplmax) {
    const uint32_t f1 = ipl_fill(ni, 1), f2 = ipl_fill(ni, 2);
    const uint32_t f4 = iplmax >= 4 ? ipl_fill(ni, 4) : 0u;
    if (f1 >= f2 && f1 >= f4) return 1u;
    return f2 >= f4 ? 2u : 4u;
}

// FP32 with up to two i-particles per lane: register budget held to 96, five waves per SIMD
// (the LDS of five workgroups fits a CU); measured 2-4 % faster than four waves per SIMD
template <class T, bool QUAD, int IPLMAX>
__global__ void __launch_bounds__(kFT, (sizeof(T) == 4 && IPLMAX == 2) ? 5 : 1)
k_fused(FusedArgs a) {
    __shared__ WaveMem<T> wmem[kFW];
    WaveMem<T> &wm = wmem[threadIdx.x / kWave];
    const int lane = lane_id();
    const uint32_t x = (uint32_t)__builtin_amdgcn_readfirstlane((int)(blockIdx.x % 8u));
    // every value that steers the control flow is made wave-uniform explicitly and the only
    // lane-divergent regions are single atomics and stores, so the loop stays a scalar loop
    // that all 64 lanes run together (a divergent-looking loop here was compiled into one that
    // dropped lanes after the first group)
    for (;;) {
        uint32_t slot = kNone;
        if (a.order) {
            uint32_t k = 0;
            if (lane == 0) k = atomicAdd(&a.st->queue_head, 1u);
            k = (uint32_t)__builtin_amdgcn_readfirstlane((int)k);
            if (k < (uint32_t)__builtin_amdgcn_readfirstlane((int)*a.count)) slot = k;
        } else {
            for (uint32_t t = 0; t < 8u; t++) {
                const uint32_t q = (x + t) & 7u;
                const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)a.bounds[q]);
                const uint32_t hi =
                    (uint32_t)__builtin_amdgcn_readfirstlane((int)a.bounds[q + 1]);
                if (lo >= hi) continue;
                uint32_t k = 0;
                if (lane == 0) k = atomicAdd(&a.st->xcd_head[q], 1u);
                k = (uint32_t)__builtin_amdgcn_readfirstlane((int)k);
                if (k < hi - lo) {
                    slot = lo + k;
                    break;
                }
            }
        }
        if (slot == kNone) break;
        const uint32_t gi =
            (uint32_t)__builtin_amdgcn_readfirstlane((int)(a.order ? a.order[slot] : slot));
        if (a.skip_wide && __builtin_amdgcn_readfirstlane((int)a.g.wide[gi]) != 0) continue;
        const uint32_t ni = (uint32_t)__builtin_amdgcn_readfirstlane((int)a.g.count[gi]);
        const uint32_t ipl =
            (uint32_t)__builtin_amdgcn_readfirstlane((int)best_ipl(ni, IPLMAX));
        fused_group<T, QUAD, IPLMAX>(a, gi, ni, ipl, wm);
    }
}

// cost of every group for the queue runs: members x (|EPJ| + ws |SPJ|) from the walk's exact
// counts, or members x predicted list length (y = predicted ln length), or members
__global__ void k_queue_cost(const uint32_t *ngroups_c, const uint32_t *gcount, const float *y,
                             const uint32_t *cnt_e, const uint32_t *cnt_s, float ws,
                             uint32_t *cost) {
    const uint32_t G = *ngroups_c;
    for (size_t gi = gtid(); gi < G; gi += gstride()) {
        float c = (float)gcount[gi];
        if (cnt_e) c *= (float)cnt_e[gi] + ws * (float)cnt_s[gi];
        else if (y) c *= ceilf(__expf(fminf(y[gi], 20.0f)));
        cost[gi] = (uint32_t)fminf(fmaxf(c, 1.0f), 4.0e9f);
    }
}

// bounds[x] = first group whose exclusive cost prefix reaches x/8 of the total (x = 1..7);
// bounds[0] = 0, bounds[8] = G
__global__ void k_fused_bounds(const uint32_t *ngroups_c, const uint64_t *pre,
                               const uint64_t *total, uint32_t *bounds) {
    const uint32_t G = *ngroups_c;
    const int x = threadIdx.x;
    if (x > 8) return;
    if (x == 0) { bounds[0] = 0; return; }
    if (x == 8) { bounds[8] = G; return; }
    const uint64_t target = (*total / 8) * (uint64_t)x + (*total % 8) * (uint64_t)x / 8;
    uint32_t lo = 0, hi = G;                     // first g with pre[g] >= target
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (pre[mid] >= target) hi = mid; else lo = mid + 1;
    }
    bounds[x] = lo;
}

template <class T, bool QUAD, int IPLMAX>
hipError_t launch_fused(const FusedArgs &a, size_t gmax, hipStream_t s) {
    int dev = 0, ncu = 256, per_cu = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, reinterpret_cast<const void *>(k_fused<T, QUAD, IPLMAX>), kFT, 0);
    if (per_cu < 1) per_cu = 1;
    size_t grid = (size_t)ncu * per_cu;
    const size_t need = (gmax + kFW - 1) / kFW;
    if (need && grid > need) grid = need;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL((k_fused<T, QUAD, IPLMAX>), dim3((unsigned)grid), dim3(kFT), 0, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t queue_bounds(size_t gmax, const uint32_t *gcount, const float *y,
                        const uint32_t *cnt_e, const uint32_t *cnt_s, float ws, uint32_t *cost,
                        uint64_t *pre, uint32_t *bounds, uint64_t *partial, DevStatus *st,
                        hipStream_t s) {
    size_t b = (gmax + 255) / 256;
    b = b < 1 ? 1 : (b > 4096 ? 4096 : b);
    hipLaunchKernelGGL(k_queue_cost, dim3((unsigned)b), dim3(256), 0, s, &st->n_groups_c, gcount,
                       y, cnt_e, cnt_s, ws, cost);
    hipError_t e = scan_u32_to_u64(cost, pre, 0, nullptr, &st->n_groups_c, partial, pre + gmax, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fused_bounds, dim3(1), dim3(64), 0, s, &st->n_groups_c, pre, pre + gmax,
                       bounds);
    return hipGetLastError();
}

hipError_t fused(size_t gmax, const FusedArgs &a, bool fp32, bool quad, int n_group,
                 hipStream_t s) {
    // up to two i-particles per lane for groups of at most 128 (fewer registers, more waves
    // per SIMD), up to four beyond
    const bool wide = n_group > 2 * kWave;
    if (fp32) {
        if (quad) return wide ? launch_fused<float, true, 4>(a, gmax, s)
                              : launch_fused<float, true, 2>(a, gmax, s);
        return wide ? launch_fused<float, false, 4>(a, gmax, s)
                    : launch_fused<float, false, 2>(a, gmax, s);
    }
    if (quad) return wide ? launch_fused<double, true, 4>(a, gmax, s)
                          : launch_fused<double, true, 2>(a, gmax, s);
    return wide ? launch_fused<double, false, 4>(a, gmax, s)
                : launch_fused<double, false, 2>(a, gmax, s);
}

}  // namespace fdx
