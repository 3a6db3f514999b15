// Group walk: one shared interaction list per i-particle group (the modified tree algorithm
// of Barnes 1990 that the paper's interaction-list model assumes, section "Tree traverse
// and interaction calculation").
//
// One wavefront walks one group.  Cells to visit sit on a per-wave LDS stack; every
// iteration pops up to 64 of them, one per lane, and tests them together.  Opening test
// (reading of "a fixed opening angle theta"): a cell of side S whose centre lies at distance
// D from the group's box is taken as a superparticle (SPJ) iff S^2 < theta^2 D^2.  All
// lengths are integers in half-grid units (S = 2^(22-l), D^2 < 2^50), so D^2 is exact in
// FP64 and the decision is one rounding of theta^2 * D^2: bit-reproducible.  An opened leaf
// contributes its particles (EPJ); an opened internal cell pushes its children.
//
// Lists live in one array: group g owns [seg[g], seg[g] + cap[g]); EPJ entries are written
// from the front and SPJ entries from the back, so the same kernel fills exact-size segments
// (count pass first) and predicted-capacity segments (single pass, overflow detected).  With
// spill on, a wave whose list outgrew its segment knows the exact length at the end of its
// walk: it reserves that much of the space after all segments (st->list_total onwards, up to
// list_cap), points the group's segment there and walks the group again; only when that
// space is exhausted is the group left empty and queued for the host.
#include "dev_util.h"
#include "fdx_internal.h"
#include "opening.h"
#include "walk_order.h"

namespace fdx {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / kWave;
constexpr int kSlack = 160;     // stack entries kept free for sequential descent

// Short-range walks (the same tree traversed with a cutoff instead of an opening angle): a
// cell is dropped iff the distance between the box and the cell's cube exceeds the search
// radius, in half-grid units D^2 > R^2 with R = r * 2^22 / Lr (an exact scaling of the
// physical radius r, one rounding in R * R); kept cells are opened and kept leaves give
// their particles as candidates.
__device__ __forceinline__ bool cell_far(const uint4 nd, int bminx, int bminy, int bminz,
                                         int bmaxx, int bmaxy, int bmaxz, double R2) {
    const int half = 1 << (kLevels - (int)(nd.w & 0xFFu));
    const int cx = (int)nd.x, cy = (int)nd.y, cz = (int)nd.z;
    const int dx = max(0, max(bminx - (cx + half), (cx - half) - bmaxx));
    const int dy = max(0, max(bminy - (cy + half), (cy - half) - bmaxy));
    const int dz = max(0, max(bminz - (cz + half), (cz - half) - bmaxz));
    const double D2 = (double)dx * (double)dx + (double)dy * (double)dy +
                      (double)dz * (double)dz;
    return D2 > R2;
}

// KIND 0: gravity (opening angle; accepted cells are superparticles).  Short range, search
// radius r: 1 the group's radius (fixed cutoff or the group's largest h), 2 the cell's largest
// h (scatter), 3 the larger of the two (symmetric).  4: tree part of TreePM, cells beyond the
// cutoff (sa.r_fixed) dropped, the opening angle for the rest.
template <bool FILL, int KIND>
__global__ void __launch_bounds__(kThreads)
k_walk(const uint32_t *ngroups, Groups g, const uint4 *node, const uint2 *link, uint32_t ccap,
       double theta2,
       uint64_t *seg, uint32_t *cap, uint64_t list_cap, uint32_t *list,
       uint32_t *cnt_e, uint32_t *cnt_s, uint32_t *ovf_list, const uint32_t *sel,
       const uint32_t *nsel, DevStatus *st, ShortArgs sa, int spill) {
    __shared__ uint32_t stack_all[kWaves][kWalkStack];
    const int w = threadIdx.x / kWave, lane = lane_id();
    const uint64_t lt = lanemask_lt();
    uint32_t *stk = stack_all[w];
    const uint32_t G = sel ? *nsel : min(*ngroups, g.cap);
    for (size_t q = (size_t)blockIdx.x * kWaves + w; q < G; q += (size_t)gridDim.x * kWaves) {
        const size_t gi = sel ? sel[q] : q;
        const uint32_t *bx = g.box + 6 * gi;
        const int bminx = 2 * (int)bx[0], bminy = 2 * (int)bx[1], bminz = 2 * (int)bx[2];
        const int bmaxx = 2 * (int)bx[3] + 2, bmaxy = 2 * (int)bx[4] + 2, bmaxz = 2 * (int)bx[5] + 2;
        uint64_t base = FILL ? seg[gi] : 0;
        bool seg_ok = !FILL || base + cap[gi] <= list_cap;
        uint32_t capg = FILL && seg_ok ? cap[gi] : 0;
        uint32_t ne = 0, ns = 0, sp = 1;
        bool err = false;
        double scale = 0.0, rg = 0.0, Rg2 = 0.0;
        if (KIND != 0) {
            scale = 4194304.0 / sa.cube[4 * (size_t)g.sys[gi] + 3];    // exact: Lr = 2^k
            rg = sa.rg ? sa.rg[gi] : sa.r_fixed;
            const double R = __dmul_rn(rg, scale);
            Rg2 = __dmul_rn(R, R);
        }
        for (int pass = 0;; pass++) {
        ne = 0; ns = 0; sp = 1; err = false;
        if (lane == 0) stk[0] = g.sys[gi];          // roots are cells 0..nsys-1
        wave_barrier();
        while (sp > 0) {
            int room = kWalkStack - kSlack - (int)sp;
            uint32_t p = min(64u, sp);
            if (room < 7 * (int)p) p = room >= 7 ? (uint32_t)(room / 7) : 1u;
            const bool act = (uint32_t)lane < p;
            uint32_t cid = 0;
            if (act) cid = stk[sp - p + lane];
            if (__ballot(act && cid >= ccap)) { err = true; break; }     // never: stack intact
            wave_barrier();
            sp -= p;
            // every lane loads (idle lanes read cell 0) and the outcome is selected without
            // branches, so both loads are issued together and nothing is loaded later
            const uint4 nd = node[cid];
            const uint2 lk = link[cid];
            const uint32_t nch = nd.w >> 8;
            // accept: emitted as a superparticle (gravity); drop: out of range (short range,
            // cutoff); otherwise opened
            bool accept = false, drop = false;
            if (KIND == 0) {
                accept = act && cell_accepted(nd, bminx, bminy, bminz, bmaxx, bmaxy, bmaxz, theta2);
            } else if (KIND == 4) {
                drop = act && cell_far(nd, bminx, bminy, bminz, bmaxx, bmaxy, bmaxz, Rg2);
                accept = act && !drop &&
                         cell_accepted(nd, bminx, bminy, bminz, bmaxx, bmaxy, bmaxz, theta2);
            } else {
                double R2 = Rg2;
                if (KIND != 1) {
                    const double hm = sa.hmax[cid];
                    const double r = (KIND == 2 || hm > rg) ? hm : rg;
                    const double R = __dmul_rn(r, scale);
                    R2 = __dmul_rn(R, R);
                }
                drop = act && cell_far(nd, bminx, bminy, bminz, bmaxx, bmaxy, bmaxz, R2);
            }
            const bool open = act && !accept && !drop;
            const bool leaf = open && nch == 0 && lk.y > 0;
            const bool inner = open && nch != 0;
            // superparticles, from the back of the segment
            if (KIND == 0 || KIND == 4) {
                const uint64_t bs = __ballot(accept);
                if (FILL && accept) {
                    const uint32_t j = ns + (uint32_t)__popcll(bs & lt);
                    if (j < capg) list[base + capg - 1 - j] = cid;
                }
                ns += (uint32_t)__popcll(bs);
            }
            // particles of opened leaves (front of the segment) and children of opened
            // internal cells (stack): offsets from one prefix sum of both counts packed in a
            // word (children, at most 8 per lane, in bits 22-31), unless a leaf holds 2^16
            // particles or more (coincident keys at the deepest level)
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
                const uint32_t li = wave_incl_scan_dpp(lc), ci = wave_incl_scan_dpp(cc);
                ltot = (uint32_t)__builtin_amdgcn_readlane((int)li, kWave - 1);
                ctot = (uint32_t)__builtin_amdgcn_readlane((int)ci, kWave - 1);
                lex = li - lc; cex = ci - cc;
            }
            // the stores of a lane run in unrolled chunks of 8 with immediate offsets (the
            // capacity bound hoisted out of the chunk), so a wave spends a few instructions
            // per slot instead of a masked loop iteration; no store is predicated (a slot past
            // the lane's count rewrites its last slot with the same value), which keeps the
            // exec mask and the scalar unit out of the chunk
            if (FILL && leaf) {
                const uint32_t e0 = ne + lex;
                const uint32_t nw = e0 < capg ? min(lc, capg - e0) : 0u;
                uint32_t *dst = list + base + e0;
                // unconditional stores: slots past nw rewrite slot nw - 1 with its own value
                for (uint32_t k0 = 0; k0 < nw; k0 += 8) {
#pragma unroll
                    for (uint32_t k = 0; k < 8; k++) {
                        const uint32_t j = min(k0 + k, nw - 1);
                        dst[j] = lk.x + j;
                    }
                }
            }
            ne += ltot;
            // children of opened internal cells onto the stack (at most 8 per cell)
            if (sp + ctot > (uint32_t)kWalkStack) { err = true; break; }
            if (inner) {
                // unconditional stores, as for the list entries
                uint32_t *d = stk + sp + cex;
#pragma unroll
                for (uint32_t k = 0; k < 8; k++) {
                    const uint32_t j = min(k, cc - 1);
                    d[j] = lk.x + j;
                }
            }
            sp += ctot;
            wave_barrier();
        }
        wave_barrier();
        if (FILL && spill && pass == 0 && !err && ((uint64_t)ne + ns > capg || !seg_ok)) {
            const uint32_t need = ne + ns;
            unsigned long long off = 0;
            if (lane == 0)
                off = atomicAdd((unsigned long long *)&st->spill_used, (unsigned long long)need);
            const uint32_t olo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)off);
            const uint32_t ohi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(off >> 32));
            const uint64_t nb = st->list_total + (((uint64_t)ohi << 32) | olo);
            if (nb + need <= list_cap) {
                base = nb;
                capg = need;
                seg_ok = true;
                if (lane == 0) {
                    seg[gi] = nb;
                    cap[gi] = need;
                    atomicAdd(&st->spilled, 1u);
                }
                continue;                               // walk the group again into its new space
            }
        }
        break;
        }
        if (lane == 0) {
            if (err) atomicOr(&st->walk_error, 1u);
            if (FILL && ((uint64_t)ne + ns > capg || !seg_ok)) {
                // the list did not fit: leave the group empty and queue it for an exact re-walk
                cnt_e[gi] = 0;
                cnt_s[gi] = 0;
                uint32_t k = atomicAdd(&st->list_overflow, 1u);
                if (ovf_list && k < g.cap) ovf_list[k] = (uint32_t)gi;
            } else {
                cnt_e[gi] = ne;
                cnt_s[gi] = ns;
            }
        }
    }
}

// ---------------------------------------------------------------------------------------
// Gravity walk by runs of kRun consecutive groups (tree order, so neighbours in space) that
// share the upper tree.  The run's box B contains every member's box, so for a cell c:
//   * if c passes the opening test against B, it passes against every member's box (the
//     distance to a member's box is at least the distance to B, and the rounded product is
//     monotone in it);
//   * if c fails the test even at B's far corners (per axis the larger distance from the
//     cell centre to B's faces bounds the distance to any member's box), every member opens c;
//   * otherwise c is a frontier cell: each member tests it in its own walk.
// A first walk of B descends only through cells every member opens and emits the entries
// every member's list holds (accepted cells, particles of opened leaves) into each member's
// segment; each member then walks on from the frontier.  Every member's list is the same set
// as the one its own walk from the root gives (all of an emitted cell's ancestors are opened
// by every member); only the order of the entries differs.  Runs that straddle two systems,
// or whose frontier outgrows kFront, are walked group by group from the root.  With a
// selection (groups re-walked after an overflow) a selected group repeats its run's first
// walk, so its entries come in the same order as in a walk of all groups.
constexpr int kRun = 4;                 // groups per run
static_assert(kWaves == (int)kWalkOrderWaves, "walk_order.h assumes the walk's waves per block");
constexpr int kFront = 224;             // frontier cells kept per wave

// the opening test at the box's far corners: false means every box inside [bmin, bmax] opens
// the cell (per axis max(c - bmin, bmax - c) bounds the distance to any box inside; the
// squares are exact integers and the product is rounded once, as in cell_accepted)
__device__ __forceinline__ bool far_accepted(const uint4 nd, int bminx, int bminy, int bminz,
                                             int bmaxx, int bmaxy, int bmaxz, double theta2) {
    const int lv = (int)(nd.w & 0xFFu);
    const int cx = (int)nd.x, cy = (int)nd.y, cz = (int)nd.z;
    const int ex = max(cx - bminx, bmaxx - cx);
    const int ey = max(cy - bminy, bmaxy - cy);
    const int ez = max(cz - bminz, bmaxz - cz);
    const double E2 = (double)ex * (double)ex + (double)ey * (double)ey +
                      (double)ez * (double)ez;
    const double S2 = __longlong_as_double((long long)(1023 + 2 * (22 - lv)) << 52);
    return S2 < __dmul_rn(theta2, E2);
}

// The stack loop of one walk (the loop of k_walk, gravity only).  SUPER: the run's first walk
// (frontier cells to `front`, entries to the first nt of kRun targets); else a member's own
// walk (one target).  Returns 0, 1 when the stack is exhausted, 2 when the frontier is full.
template <bool FILL, bool SUPER>
__device__ __forceinline__ int run_stack(uint32_t *stk, uint32_t sp, uint32_t *front,
                                         uint32_t &nf, const uint4 *node, const uint2 *link,
                                         uint32_t ccap, double theta2, const int (&b)[6],
                                         uint32_t *list, const uint64_t (&base)[kRun],
                                         const uint32_t (&capg)[kRun], int nt, uint32_t &ne,
                                         uint32_t &ns) {
    constexpr int NT = SUPER ? kRun : 1;
    const int lane = lane_id();
    const uint64_t lt = lanemask_lt();
    while (sp > 0) {
        const int room = kWalkStack - kSlack - (int)sp;
        uint32_t p = min(64u, sp);
        if (room < 7 * (int)p) p = room >= 7 ? (uint32_t)(room / 7) : 1u;
        const bool act = (uint32_t)lane < p;
        uint32_t cid = 0;
        if (act) cid = stk[sp - p + lane];
        if (__ballot(act && cid >= ccap)) return 1;                  // never: stack intact
        wave_barrier();
        sp -= p;
        const uint4 nd = node[cid];
        const uint2 lk = link[cid];
        const uint32_t nch = nd.w >> 8;
        const bool accept = act && cell_accepted(nd, b[0], b[1], b[2], b[3], b[4], b[5], theta2);
        bool open = act && !accept;
        if (SUPER) {
            const bool all = open && !far_accepted(nd, b[0], b[1], b[2], b[3], b[4], b[5], theta2);
            const bool fr = open && !all;
            open = all;
            const uint64_t bf = __ballot(fr);
            const uint32_t ftot = (uint32_t)__popcll(bf);
            if (nf + ftot > (uint32_t)kFront) return 2;
            if (fr) front[nf + (uint32_t)__popcll(bf & lt)] = cid;
            nf += ftot;
        }
        const bool leaf = open && nch == 0 && lk.y > 0;
        const bool inner = open && nch != 0;
        // superparticles, from the back of each target's segment
        const uint64_t bs = __ballot(accept);
        if (FILL && accept) {
            const uint32_t j = ns + (uint32_t)__popcll(bs & lt);
#pragma unroll
            for (int k = 0; k < NT; k++)
                if (k < nt && j < capg[k]) list[base[k] + capg[k] - 1 - j] = cid;
        }
        ns += (uint32_t)__popcll(bs);
        // leaf particles and children: one prefix sum of both counts packed in a word unless
        // a leaf holds 2^16 particles or more (as in k_walk)
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
            const uint32_t li = wave_incl_scan_dpp(lc), ci = wave_incl_scan_dpp(cc);
            ltot = (uint32_t)__builtin_amdgcn_readlane((int)li, kWave - 1);
            ctot = (uint32_t)__builtin_amdgcn_readlane((int)ci, kWave - 1);
            lex = li - lc; cex = ci - cc;
        }
        if (FILL && leaf) {
            const uint32_t e0 = ne + lex;
#pragma unroll
            for (int k = 0; k < NT; k++) {
                if (k >= nt) continue;
                const uint32_t nw = e0 < capg[k] ? min(lc, capg[k] - e0) : 0u;
                uint32_t *dst = list + base[k] + e0;
                // unconditional stores: slots past nw rewrite slot nw - 1 with its own value
                for (uint32_t k0 = 0; k0 < nw; k0 += 8) {
#pragma unroll
                    for (uint32_t u = 0; u < 8; u++) {
                        const uint32_t j = min(k0 + u, nw - 1);
                        dst[j] = lk.x + j;
                    }
                }
            }
        }
        ne += ltot;
        if (sp + ctot > (uint32_t)kWalkStack) return 1;
        if (inner) {
            uint32_t *d = stk + sp + cex;
#pragma unroll
            for (uint32_t u = 0; u < 8; u++) {
                const uint32_t j = min(u, cc - 1);
                d[j] = lk.x + j;
            }
        }
        sp += ctot;
        wave_barrier();
    }
    return 0;
}

// a group's box in half-grid units
__device__ __forceinline__ void group_box(const Groups &g, uint32_t gi, int (&b)[6]) {
    const uint32_t *bx = g.box + 6 * (size_t)gi;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        b[a] = 2 * (int)bx[a];
        b[3 + a] = 2 * (int)bx[3 + a] + 2;
    }
}

// One wave per run (or per selected group).  Arguments as k_walk's (gravity).  Held to 8
// waves per SIMD (the limit that the LDS of 8 workgroups per CU also sets); the bound makes
// the compiler keep some scalar values in vector lanes, and without it the kernel ran at 7
// waves per SIMD and was slower.
//
// Order of the runs without a selection: XCD-aware chunks of `chunk` runs (walk_order.h);
// with a selection the waves stride over it.
template <bool FILL>
__global__ void __launch_bounds__(kThreads, 8)
k_walk_runs(const uint32_t *ngroups, Groups g, const uint4 *node, const uint2 *link,
            uint32_t ccap, double theta2, uint64_t *seg, uint32_t *cap, uint64_t list_cap,
            uint32_t *list, uint32_t *cnt_e, uint32_t *cnt_s, uint32_t *ovf_list,
            const uint32_t *sel, const uint32_t *nsel, DevStatus *st, int spill,
            uint32_t chunk) {
    __shared__ uint32_t stack_all[kWaves][kWalkStack];
    __shared__ uint32_t front_all[kWaves][kFront];
    const int w = threadIdx.x / kWave, lane = lane_id();
    uint32_t *stk = stack_all[w];
    uint32_t *front = front_all[w];
    const uint32_t G = min(*ngroups, g.cap);
    const uint32_t items = sel ? *nsel : (G + kRun - 1) / kRun;
    // this wave's slot within each W: a permutation of 0..W-1
    const uint32_t slot = walk_order_slot(blockIdx.x, (uint32_t)w, gridDim.x, sel ? 0u : chunk);
    // the two arguments the stack loops read: apart from the argument tuples, so that the
    // loops reload none of the scalar registers spilled under the occupancy bound (each such
    // reload was 16 readlanes in the opening test and in the particle-entry stores)
    const double th2 = own_sgpr_pair(theta2);
    uint32_t *const lst = own_sgpr_pair(list);
    for (size_t q = slot; q < items; q += (size_t)gridDim.x * kWaves) {
        // targets [t0, t1) of run [r0, r1)
        const uint32_t t0 = uniform_u32(sel ? sel[q] : (uint32_t)q * kRun);
        if (t0 >= G) continue;
        const uint32_t t1 = sel ? t0 + 1 : min(t0 + kRun, G);
        const uint32_t r0 = t0 / kRun * kRun, r1 = min(r0 + kRun, G);
        const int nt = (int)(t1 - t0);
        const uint32_t root = g.sys[r0];                  // roots are cells 0..nsys-1
        bool shared = r1 - r0 > 1 && g.sys[r1 - 1] == root;
        int rb[6];
        group_box(g, r0, rb);
        for (uint32_t k = r0 + 1; k < r1; k++) {
            int b[6];
            group_box(g, k, b);
#pragma unroll
            for (int a = 0; a < 3; a++) {
                rb[a] = min(rb[a], b[a]);
                rb[3 + a] = max(rb[3 + a], b[3 + a]);
            }
        }
        // the members' segments for the run's first walk (constant indices only, so the
        // arrays stay in registers)
        uint64_t base[kRun];
        uint32_t capg[kRun];
#pragma unroll
        for (int k = 0; k < kRun; k++) {
            base[k] = 0; capg[k] = 0;
            if (FILL && k < nt) {
                base[k] = seg[t0 + k];
                capg[k] = base[k] + cap[t0 + k] <= list_cap ? cap[t0 + k] : 0u;
            }
        }
        bool err = false;
        uint32_t ne0 = 0, ns0 = 0, nf = 0;
        if (shared) {
            if (lane == 0) stk[0] = root;
            wave_barrier();
            const int r = run_stack<FILL, true>(stk, 1, front, nf, node, link, ccap, th2, rb,
                                                lst, base, capg, nt, ne0, ns0);
            if (r == 1) err = true;
            if (r != 0) shared = false;                // each member walks from the root
        }
        if (!shared) { ne0 = 0; ns0 = 0; nf = 0; }
        for (int k = 0; k < nt; k++) {
            const uint32_t gi = t0 + (uint32_t)k;
            int gb[6];
            group_box(g, gi, gb);
            uint64_t bk[kRun] = {0, 0, 0, 0};
            uint32_t ck[kRun] = {0, 0, 0, 0};
            bool ok = true;
            if (FILL) {                                // as read for the first walk
                bk[0] = seg[gi];
                ok = bk[0] + cap[gi] <= list_cap;
                ck[0] = ok ? cap[gi] : 0u;
            }
            uint32_t ne = 0, ns = 0;
            bool gerr = false;
            for (int pass = 0;; pass++) {
                ne = ne0; ns = ns0;
                if (pass > 0 && shared) {
                    // the run's first walk again, into this group's new space only
                    uint32_t nf2 = 0;
                    ne = 0; ns = 0;
                    if (lane == 0) stk[0] = root;
                    wave_barrier();
                    if (run_stack<FILL, true>(stk, 1, front, nf2, node, link, ccap, th2, rb,
                                              lst, bk, ck, 1, ne, ns) != 0)
                        gerr = true;                   // never: the first walk completed
                }
                uint32_t sp;
                if (shared) {
                    for (uint32_t i = (uint32_t)lane; i < nf; i += kWave) stk[i] = front[i];
                    sp = nf;
                } else {
                    if (lane == 0) stk[0] = g.sys[gi];
                    sp = 1;
                }
                wave_barrier();
                uint32_t nf_unused = 0;
                if (!gerr && run_stack<FILL, false>(stk, sp, nullptr, nf_unused, node, link, ccap,
                                                    th2, gb, lst, bk, ck, 1, ne, ns) != 0)
                    gerr = true;
                wave_barrier();
                if (FILL && spill && pass == 0 && !gerr && ((uint64_t)ne + ns > ck[0] || !ok)) {
                    const uint32_t need = ne + ns;
                    unsigned long long off = 0;
                    if (lane == 0)
                        off = atomicAdd((unsigned long long *)&st->spill_used,
                                        (unsigned long long)need);
                    const uint64_t nb = st->list_total + uniform_u64((uint64_t)off);
                    if (nb + need <= list_cap) {
                        bk[0] = nb;
                        ck[0] = need;
                        ok = true;
                        if (lane == 0) {
                            seg[gi] = nb;
                            cap[gi] = need;
                            atomicAdd(&st->spilled, 1u);
                        }
                        continue;                      // walk the group again into its new space
                    }
                }
                break;
            }
            if (lane == 0) {
                if (err || gerr) atomicOr(&st->walk_error, 1u);
                if (FILL && ((uint64_t)ne + ns > ck[0] || !ok)) {
                    cnt_e[gi] = 0;
                    cnt_s[gi] = 0;
                    uint32_t o = atomicAdd(&st->list_overflow, 1u);
                    if (ovf_list && o < g.cap) ovf_list[o] = gi;
                } else {
                    cnt_e[gi] = ne;
                    cnt_s[gi] = ns;
                }
            }
        }
    }
}

// cap[g] = |EPJ| + |SPJ| (exact segment sizes)
__global__ void k_list_caps(const uint32_t *ngroups, uint32_t gmax, const uint32_t *cnt_e,
                            const uint32_t *cnt_s, uint32_t *cap) {
    const uint32_t G = min(*ngroups, gmax);
    for (size_t gi = gtid(); gi < G; gi += gstride()) cap[gi] = cnt_e[gi] + cnt_s[gi];
}

// cap[g] = sys_cap[system of g]: per-system segment sizes (a system's particle count bounds
// |EPJ| + |SPJ| of its groups, since a list's entries -- opened leaves' particles, accepted
// cells -- cover disjoint sets of the system's particles)
__global__ void k_sys_caps(const uint32_t *ngroups, uint32_t gmax, const uint32_t *gsys,
                           const uint32_t *sys_cap, uint32_t *cap) {
    const uint32_t G = min(*ngroups, gmax);
    for (size_t gi = gtid(); gi < G; gi += gstride()) cap[gi] = sys_cap[gsys[gi]];
}

// lmax[s] = longest list of system s, gcount[s] = its groups (both cleared by the caller)
__global__ void k_sys_lmax(const uint32_t *ngroups, uint32_t gmax, const uint32_t *gsys,
                           const uint32_t *cnt_e, const uint32_t *cnt_s, uint32_t *lmax,
                           uint32_t *gcount) {
    const uint32_t G = min(*ngroups, gmax);
    for (size_t gi = gtid(); gi < G; gi += gstride()) {
        const uint32_t s = gsys[gi];
        atomicMax(&lmax[s], cnt_e[gi] + cnt_s[gi]);
        atomicAdd(&gcount[s], 1u);
    }
}

// every group's entries out of its segment into contiguous per-kind arrays (one workgroup per
// group): EPJ from the front of the segment, SPJ from its back
__global__ void __launch_bounds__(kThreads)
k_compact_lists(size_t G, const uint64_t *seg, const uint32_t *cap, const uint32_t *cnt_e,
                const uint32_t *cnt_s, const uint64_t *oe, const uint64_t *os,
                const uint32_t *list, uint32_t *epj, uint32_t *spj) {
    for (size_t g = blockIdx.x; g < G; g += gridDim.x) {
        const uint64_t b = seg[g], e0 = oe[g], s0 = os[g];
        const uint32_t ne = cnt_e[g], ns = cnt_s[g];
        const uint64_t sb = b + cap[g] - ns;
        for (uint32_t k = threadIdx.x; k < ne; k += kThreads) epj[e0 + k] = list[b + k];
        for (uint32_t k = threadIdx.x; k < ns; k += kThreads) spj[s0 + k] = list[sb + k];
    }
}

__global__ void __launch_bounds__(kThreads)
k_list_stats(const uint32_t *ngroups, uint32_t gmax, const uint32_t *gcount,
             const uint32_t *cnt_e, const uint32_t *cnt_s, DevStatus *st) {
    const uint32_t G = min(*ngroups, gmax);
    uint64_t e = 0, s = 0, pp = 0, pc = 0;
    for (size_t gi = gtid(); gi < G; gi += gstride()) {
        const uint64_t ni = gcount[gi];
        e += cnt_e[gi]; s += cnt_s[gi];
        pp += ni * cnt_e[gi]; pc += ni * cnt_s[gi];
    }
    // wave sums, then the block's waves through LDS: one set of atomics per block (a few
    // dozen blocks), not per wave
    __shared__ uint64_t part[kWaves][4];
    e = wave_sum_u64(e); s = wave_sum_u64(s); pp = wave_sum_u64(pp); pc = wave_sum_u64(pc);
    const int w = threadIdx.x / kWave;
    if (lane_id() == 0) { part[w][0] = e; part[w][1] = s; part[w][2] = pp; part[w][3] = pc; }
    __syncthreads();
    if (threadIdx.x < 4) {
        uint64_t v = 0;
#pragma unroll
        for (int k = 0; k < kWaves; k++) v += part[k][threadIdx.x];
        unsigned long long *dst[4] = {(unsigned long long *)&st->n_epj,
                                      (unsigned long long *)&st->n_spj,
                                      (unsigned long long *)&st->inter_pp,
                                      (unsigned long long *)&st->inter_pc};
        if (v) atomicAdd(dst[threadIdx.x], (unsigned long long)v);
    }
}

// Exchange lists between domains (section "Exchange of particles and superparticles",
// long-range mode).  The list of the ordered pair (sender s, receiver r != s) is the walk of
// s's tree against the exact bounding box of r's particles in s's integer grid,
// q = floor((x - o) * 2^21 / Lr), clamped to [-2^24, 2^24] so half-grid distances stay exact
// in FP64 (a clamped box is closer, so more cells open and the list stays sufficient).  Boxes
// are stored as int32 in the u32 box array; the walk reads them back as signed values.
//
// Each pair's walk is split over the sender's frontier at level kFrontier (its cells of that
// level and its leaves above it; at most 8^kFrontier cells, covering every particle once).
// Every cell is decided from itself and the box alone, so the full walk equals, for each
// frontier cell c: nothing if an ancestor of c is accepted, except that the frontier cell
// sharing the first particle of the highest accepted ancestor a emits a; otherwise the walk
// of c's subtree.  A sub-walk is one "group" of the walk kernel whose start cell is c (or a,
// which the kernel then accepts at once).
__global__ void k_fill_one(uint32_t *p) { *p = 0u; }

constexpr int kFrontier = 2;
constexpr int kFrontierMax = 64;                    // 8^kFrontier

__device__ __forceinline__ int grid_signed(double x, double o, double Lr) {
    const double sc = 2097152.0 / Lr;                  // a power of two: exact
    double f = floor(__dmul_rn(__dsub_rn(x, o), sc));
    f = fmin(fmax(f, -16777216.0), 16777216.0);
    return (int)f;
}

// frontier cells of every system (depth-first, child order): front[kFrontierMax s + f]
__global__ void k_exchange_frontier(int nsys, Cells c, uint32_t *front, uint32_t *fcount) {
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < nsys; s += gridDim.x * blockDim.x) {
        uint32_t stk[1 + 7 * kFrontier], sp = 0, nf = 0;
        stk[sp++] = (uint32_t)s;
        while (sp) {
            const uint32_t cid = stk[--sp];
            const uint32_t nch = c.nchild[cid];
            if (c.level[cid] >= (uint32_t)kFrontier || nch == 0) {
                front[kFrontierMax * (size_t)s + nf++] = cid;
            } else {
                const uint32_t f = c.first[cid];
                for (uint32_t k = nch; k-- > 0;) stk[sp++] = f + k;
            }
        }
        fcount[s] = nf;
    }
}

// one sub-walk per (pair k, frontier slot f): box, start cell and segment size (0 = idle);
// the active sub-walks are appended to sel.  With by_bound the segment is sized by the start
// cell's particle count (a sub-walk's entries cover disjoint sets of its particles), else
// the count walk sizes it afterwards.
__global__ void k_exchange_split(int nsys, Cells c, const uint32_t *front, const uint32_t *fcount,
                                 const uint64_t *bbox_u, const double *cube, double theta2,
                                 uint32_t *box, uint32_t *start, uint32_t *cap, uint32_t *sel,
                                 uint32_t *nsel) {
    const size_t P = (size_t)nsys * (size_t)(nsys - 1);
    for (size_t g = gtid(); g < P * kFrontierMax; g += gstride()) {
        const size_t k = g / kFrontierMax;
        const uint32_t f = (uint32_t)(g % kFrontierMax);
        const uint32_t s = (uint32_t)(k / (nsys - 1)), j = (uint32_t)(k % (nsys - 1));
        const uint32_t r = j < s ? j : j + 1;
        cap[g] = 0;
        if (f >= fcount[s]) continue;
        const double *cb = cube + 4 * (size_t)s;
        int q[6];
#pragma unroll
        for (int a = 0; a < 3; a++) {
            q[a] = grid_signed(ord_to_dbl(bbox_u[6 * (size_t)r + 2 * a]), cb[a], cb[3]);
            q[3 + a] = grid_signed(ord_to_dbl(bbox_u[6 * (size_t)r + 2 * a + 1]), cb[a], cb[3]);
            box[6 * g + a] = (uint32_t)q[a];
            box[6 * g + 3 + a] = (uint32_t)q[3 + a];
        }
        const uint32_t cell = front[kFrontierMax * (size_t)s + f];
        // the ancestors of the frontier cell, root first
        uint32_t anc[kFrontier];
        int na = 0;
        for (uint32_t a = c.parent[cell]; a != kNone && na < kFrontier; a = c.parent[a]) anc[na++] = a;
        uint32_t st = cell, sz = c.count[cell];
        for (int i = na - 1; i >= 0; i--) {
            if (cell_accepted(c.node[anc[i]], 2 * q[0], 2 * q[1], 2 * q[2], 2 * q[3] + 2,
                              2 * q[4] + 2, 2 * q[5] + 2, theta2)) {
                st = anc[i];
                sz = c.begin[cell] == c.begin[st] ? 1u : 0u;
                break;
            }
        }
        start[g] = st;
        cap[g] = sz;
        if (sz) sel[atomicAdd(nsel, 1u)] = (uint32_t)g;
    }
}

__global__ void k_exchange_caps(size_t G, const uint32_t *sel, const uint32_t *nsel,
                                const uint32_t *ne, const uint32_t *ns, uint32_t *cap) {
    const uint32_t n = *nsel;
    for (size_t i = gtid(); i < n; i += gstride()) {
        const uint32_t g = sel[i];
        if (g < G) cap[g] = ne[g] + ns[g];
    }
}

inline unsigned grid_waves(size_t gmax) {
    size_t b = (gmax + kWaves - 1) / kWaves;
    if (b < 1) b = 1;
    if (b > 16384) b = 16384;
    return (unsigned)b;
}

}  // namespace

size_t exchange_subwalks(int nsys) {
    return (size_t)nsys * (size_t)(nsys - 1) * kFrontierMax;
}

hipError_t exchange_split(int nsys, const Cells c, const uint64_t *bbox_u, const double *cube,
                          double theta2, uint32_t *front, uint32_t *fcount, uint32_t *box,
                          uint32_t *start, uint32_t *cap, uint32_t *sel, uint32_t *nsel,
                          hipStream_t s) {
    const size_t G = exchange_subwalks(nsys);
    if (!G) return hipSuccess;
    hipLaunchKernelGGL(k_exchange_frontier, dim3((nsys + 63) / 64), dim3(64), 0, s, nsys, c, front,
                       fcount);
    hipLaunchKernelGGL(k_fill_one, dim3(1), dim3(1), 0, s, nsel);
    size_t b = (G + kThreads - 1) / kThreads;
    b = b > 8192 ? 8192 : b;
    hipLaunchKernelGGL(k_exchange_split, dim3((unsigned)b), dim3(kThreads), 0, s, nsys, c, front,
                       fcount, bbox_u, cube, theta2, box, start, cap, sel, nsel);
    return hipGetLastError();
}

hipError_t exchange_caps(size_t G, const uint32_t *sel, const uint32_t *nsel, const uint32_t *ne,
                         const uint32_t *ns, uint32_t *cap, hipStream_t s) {
    if (!G) return hipSuccess;
    size_t b = (G + kThreads - 1) / kThreads;
    b = b > 4096 ? 4096 : b;
    hipLaunchKernelGGL(k_exchange_caps, dim3((unsigned)b), dim3(kThreads), 0, s, G, sel, nsel, ne,
                       ns, cap);
    return hipGetLastError();
}

template <int KIND>
static void launch_walk(bool fill, size_t gmax, const Groups &g, const Cells &c, double theta2,
                        uint64_t *seg, uint32_t *cap, uint64_t list_cap,
                        uint32_t *list, uint32_t *cnt_e, uint32_t *cnt_s, uint32_t *ovf_list,
                        const uint32_t *sel, const uint32_t *nsel, DevStatus *st,
                        const ShortArgs &sa, hipStream_t s, bool spill = false) {
    if (fill)
        hipLaunchKernelGGL((k_walk<true, KIND>), dim3(grid_waves(gmax)), dim3(kThreads), 0, s,
                           &st->n_groups, g, c.node, c.link, c.cap, theta2, seg, cap, list_cap,
                           list, cnt_e, cnt_s, ovf_list, sel, nsel, st, sa, spill ? 1 : 0);
    else
        hipLaunchKernelGGL((k_walk<false, KIND>), dim3(grid_waves(gmax)), dim3(kThreads), 0, s,
                           &st->n_groups, g, c.node, c.link, c.cap, theta2, seg, cap, list_cap,
                           list, cnt_e, cnt_s, ovf_list, sel, nsel, st, sa, 0);
}

hipError_t walk(bool fill, size_t gmax, const Groups g, const Cells c, double theta2,
                uint64_t *seg, uint32_t *cap, uint64_t list_cap, uint32_t *list,
                uint32_t *cnt_e, uint32_t *cnt_s, uint32_t *ovf_list, const uint32_t *sel,
                const uint32_t *nsel, DevStatus *st, hipStream_t s, bool spill) {
    launch_walk<0>(fill, gmax, g, c, theta2, seg, cap, list_cap, list, cnt_e, cnt_s, ovf_list,
                   sel, nsel, st, ShortArgs{}, s, spill);
    return hipGetLastError();
}

hipError_t walk_runs(bool fill, size_t gmax, const Groups g, const Cells c, double theta2,
                     uint64_t *seg, uint32_t *cap, uint64_t list_cap, uint32_t *list,
                     uint32_t *cnt_e, uint32_t *cnt_s, uint32_t *ovf_list, const uint32_t *sel,
                     const uint32_t *nsel, DevStatus *st, hipStream_t s, bool spill) {
    const size_t items = sel ? gmax : (gmax + kRun - 1) / kRun;
    size_t grid = grid_waves(items);
    uint32_t chunk = 0;
    if (!sel) walk_order_launch(items, grid, &grid, &chunk);
    if (fill)
        hipLaunchKernelGGL(k_walk_runs<true>, dim3((unsigned)grid), dim3(kThreads), 0, s,
                           &st->n_groups, g, c.node, c.link, c.cap, theta2, seg, cap, list_cap,
                           list, cnt_e, cnt_s, ovf_list, sel, nsel, st, spill ? 1 : 0, chunk);
    else
        hipLaunchKernelGGL(k_walk_runs<false>, dim3((unsigned)grid), dim3(kThreads), 0, s,
                           &st->n_groups, g, c.node, c.link, c.cap, theta2, seg, cap, list_cap,
                           list, cnt_e, cnt_s, ovf_list, sel, nsel, st, 0, chunk);
    return hipGetLastError();
}

hipError_t walk_short(bool fill, int kind, size_t gmax, const Groups g, const Cells c,
                      const ShortArgs sa, double theta2, const uint64_t *seg_c,
                      const uint32_t *cap_c, uint64_t list_cap, uint32_t *list, uint32_t *cnt_e,
                      uint32_t *cnt_s, uint32_t *ovf_list, DevStatus *st, hipStream_t s) {
    // short walks never relocate a list, so the segment arrays are only read
    uint64_t *seg = const_cast<uint64_t *>(seg_c);
    uint32_t *cap = const_cast<uint32_t *>(cap_c);
    switch (kind) {
        case 1: launch_walk<1>(fill, gmax, g, c, 0.0, seg, cap, list_cap, list, cnt_e, cnt_s,
                               ovf_list, nullptr, nullptr, st, sa, s); break;
        case 2: launch_walk<2>(fill, gmax, g, c, 0.0, seg, cap, list_cap, list, cnt_e, cnt_s,
                               ovf_list, nullptr, nullptr, st, sa, s); break;
        case 3: launch_walk<3>(fill, gmax, g, c, 0.0, seg, cap, list_cap, list, cnt_e, cnt_s,
                               ovf_list, nullptr, nullptr, st, sa, s); break;
        default: launch_walk<4>(fill, gmax, g, c, theta2, seg, cap, list_cap, list, cnt_e, cnt_s,
                                ovf_list, nullptr, nullptr, st, sa, s); break;
    }
    return hipGetLastError();
}

hipError_t list_caps(size_t gmax, const uint32_t *cnt_e, const uint32_t *cnt_s, uint32_t *cap,
                     DevStatus *st, hipStream_t s) {
    size_t b = (gmax + kThreads - 1) / kThreads;
    b = b < 1 ? 1 : (b > 8192 ? 8192 : b);
    hipLaunchKernelGGL(k_list_caps, dim3((unsigned)b), dim3(kThreads), 0, s, &st->n_groups_c,
                       (uint32_t)gmax, cnt_e, cnt_s, cap);
    return hipGetLastError();
}

hipError_t sys_caps(size_t gmax, const uint32_t *gsys, const uint32_t *sys_cap, uint32_t *cap,
                    DevStatus *st, hipStream_t s) {
    size_t b = (gmax + kThreads - 1) / kThreads;
    b = b < 1 ? 1 : (b > 8192 ? 8192 : b);
    hipLaunchKernelGGL(k_sys_caps, dim3((unsigned)b), dim3(kThreads), 0, s, &st->n_groups_c,
                       (uint32_t)gmax, gsys, sys_cap, cap);
    return hipGetLastError();
}

hipError_t sys_lmax(size_t gmax, const uint32_t *gsys, const uint32_t *cnt_e,
                    const uint32_t *cnt_s, uint32_t *lmax, uint32_t *gcount, DevStatus *st,
                    hipStream_t s) {
    size_t b = (gmax + kThreads - 1) / kThreads;
    b = b < 1 ? 1 : (b > 8192 ? 8192 : b);
    hipLaunchKernelGGL(k_sys_lmax, dim3((unsigned)b), dim3(kThreads), 0, s, &st->n_groups_c,
                       (uint32_t)gmax, gsys, cnt_e, cnt_s, lmax, gcount);
    return hipGetLastError();
}

hipError_t compact_lists(size_t G, const uint64_t *seg, const uint32_t *cap,
                         const uint32_t *cnt_e, const uint32_t *cnt_s, const uint64_t *oe,
                         const uint64_t *os, const uint32_t *list, uint32_t *epj, uint32_t *spj,
                         hipStream_t s) {
    if (!G) return hipSuccess;
    hipLaunchKernelGGL(k_compact_lists, dim3((unsigned)(G < 65536 ? G : 65536)), dim3(kThreads),
                       0, s, G, seg, cap, cnt_e, cnt_s, oe, os, list, epj, spj);
    return hipGetLastError();
}

hipError_t list_stats(size_t gmax, const Groups g, const uint32_t *cnt_e, const uint32_t *cnt_s,
                      DevStatus *st, hipStream_t s) {
    size_t b = (gmax + kThreads - 1) / kThreads;
    b = b < 1 ? 1 : (b > 64 ? 64 : b);
    hipLaunchKernelGGL(k_list_stats, dim3((unsigned)b), dim3(kThreads), 0, s, &st->n_groups_c,
                       (uint32_t)gmax, g.count, cnt_e, cnt_s, st);
    return hipGetLastError();
}

}  // namespace fdx
