// Internal declarations of the gfx950 Barnes-Hut library: device helpers and the host-side
// launchers of every kernel.  Not part of the C ABI (include/fdx.h is).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace fdx {

constexpr int kLevels = 21;              // key bits per axis; deepest cell level
constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr int kMaxGroup = 512;           // largest n_group the force kernels take
constexpr int kWalkStack = 1024;         // per-wave LDS stack of the group walk (entries)

// Device-side status and counters of one evaluation, read back once per force call.
struct DevStatus {
    uint32_t cell_overflow;   // the tree needed more cells than were allocated
    uint32_t bad_input;       // a non-finite coordinate, negative mass or eps <= 0 was seen
    uint32_t walk_error;      // a walk stack would have overflowed (group left incomplete)
    uint32_t list_overflow;   // groups whose list did not fit its segment or the list buffer
    uint32_t n_groups;
    uint32_t depth;
    uint32_t queue_head;      // persistent force kernel: next queue slot to pop
    uint32_t n_groups_c;      // min(n_groups, group capacity): what the kernels iterate over
    uint64_t list_total;      // entries needed by all lists
    uint64_t n_epj, n_spj;
    uint64_t inter_pp, inter_pc;
    uint32_t group_overflow;  // more groups than the group arrays hold
    uint32_t top_level;       // deepest tree level whose cells fit the cell capacity
    uint32_t wide_groups;     // FP32 evaluation: groups too wide for group-relative FP32
    uint32_t eps_varies;      // fdx_set_particles, device eps: some eps differs from the eps of
                              // its system's first particle
    uint32_t xcd_head[8];     // persistent force kernel: next slot of each XCD's queue
    uint64_t spill_used;      // fill walk: entries taken after list_total by relocated lists
    uint32_t spilled;         // fill walk: groups whose list was relocated there
    uint32_t pad2_;
};

// any device-reported condition that makes this evaluation's forces incomplete
__host__ __device__ inline bool status_incomplete(const DevStatus &s) {
    return s.cell_overflow | s.group_overflow | s.list_overflow | s.walk_error;
}

// Tree cell arrays (breadth-first order) and walk-friendly views.
struct Cells {
    uint32_t *level, *begin, *count, *first, *nchild, *parent;
    uint64_t *prefix;
    uint4 *node;      // {2*corner_x + 2^(21-l), ... y, ... z, level | nchild << 8} (half-grid)
    uint2 *link;      // leaf: {begin, count}; internal: {first_child, count}
    double *mom;      // 10 per cell: M, X, Y, Z, Qxx, Qyy, Qzz, Qxy, Qxz, Qyz
    uint32_t *lvl;    // lvl[l] = first cell of level l, l = 0..22
    uint32_t cap;
};

struct Groups {
    uint32_t *cell, *begin, *count, *sys;
    uint32_t *box;    // 6 per group: qmin x y z, qmax x y z (grid units)
    double *centre;   // 3 per group: geometric centre of the group's cell
    uint32_t *wide;   // 1 where group-relative FP32 would be too coarse (evaluated in FP64)
    uint32_t cap;
};

// ---------------------------------------------------------------------------------------
// launchers (every one enqueues on `s` and returns the launch status)

// misc
hipError_t fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s);
hipError_t fill_u64(uint64_t *p, uint64_t v, size_t n, hipStream_t s);
hipError_t iota_u32(uint32_t *p, size_t n, hipStream_t s);
hipError_t check_input(size_t n, const double *x, const double *y, const double *z,
                       const double *m, const double *eps, DevStatus *st, hipStream_t s);
hipError_t sysid_fill(const int64_t *sys_off, int nsys, uint32_t *sysid, size_t n,
                      hipStream_t s);
hipError_t kick_drift(size_t n, double *x, double *y, double *z, double *vx, double *vy,
                      double *vz, const double *ax, const double *ay, const double *az,
                      double dt, hipStream_t s);
hipError_t kick(size_t n, double *vx, double *vy, double *vz, const double *ax,
                const double *ay, const double *az, double dt, const DevStatus *st,
                hipStream_t s);
hipError_t unsort_forces(size_t n, const double4 *fs, const uint32_t *inv, double *ax,
                         double *ay, double *az, double *pot, hipStream_t s);

// scan: exclusive prefix sums of u32 counts.  The element count is n_host, or, if lo/hi are
// given, (*hi - *lo) read on the device.  partial must hold kScanBlocks + 1 entries.
constexpr int kScanBlocks = 512;
hipError_t scan_u32_to_u32(const uint32_t *in, uint32_t *out, size_t n_host,
                           const uint32_t *lo, const uint32_t *hi, uint64_t *partial,
                           uint32_t *total32, hipStream_t s);
hipError_t scan_u32_to_u64(const uint32_t *in, uint64_t *out, size_t n_host,
                           const uint32_t *lo, const uint32_t *hi, uint64_t *partial,
                           uint64_t *total64, hipStream_t s);

// keys
hipError_t bbox(size_t n, const double *x, const double *y, const double *z,
                const uint32_t *sysid, int nsys, uint64_t *bbox_u, hipStream_t s);
hipError_t root_cubes(int nsys, const uint64_t *bbox_u, double *cube, hipStream_t s);
// keys, the identity permutation and each particle's (x, y, z, m) record for the sorted gather
hipError_t morton_keys(size_t n, const double *x, const double *y, const double *z,
                       const double *m, const uint32_t *sysid, int nsys, const double *cube,
                       uint64_t *key, uint32_t *perm, double4 *packed, hipStream_t s);

// radix sort of (key, perm) pairs by key, then (stable) by system id of the original index.
size_t radix_scratch_u32(size_t n);
// key_bits = significant low bits of the keys (passes of 8 bits over them).  carry: optional
// 2n 16-bit scratch; with 2..65536 systems their ids then travel with the elements instead of
// being gathered through the index in the system-id passes (the val array must start as the
// identity, and sysid be indexed by the original index).
hipError_t radix_sort(size_t n, uint64_t *key, uint64_t *key_alt, uint32_t *val,
                      uint32_t *val_alt, const uint32_t *sysid, int nsys, int key_bits,
                      uint32_t *scratch, uint64_t *partial, bool *result_in_alt, hipStream_t s,
                      uint16_t *carry = nullptr);

// sorted particle data
// flag |= 1 if some eps[i] differs from the eps of its system's first particle
hipError_t eps_varies(size_t n, const double *eps, const uint32_t *sysid, const int64_t *off,
                      uint32_t *flag, hipStream_t s);
// per_system: every system's particles share one eps (taken from its first particle)
hipError_t gather_sorted(size_t n, const uint32_t *perm, const double4 *packed,
                         const double *eps, double eps_all, bool per_system, const int64_t *off,
                         int nsys, double4 *jp, double *seps, uint32_t *inv, hipStream_t s);

// tree
// scratch words tree_build needs besides 3 n bytes
size_t tree_scratch_u32(size_t n);
hipError_t tree_build(size_t n, int nsys, const int64_t *sys_off, const uint64_t *skey,
                      int n_leaf, Cells c, uint8_t *bytes, uint32_t *scratch,
                      uint64_t *partial, DevStatus *st, hipStream_t s);
hipError_t tree_moments(Cells c, const double4 *jp, hipStream_t s);
// groups, their boxes and centres, and the wide flag: with d = depth of the group's deepest
// leaf below its cell, S the cell side and eps_min the smallest softening among its members,
// a group is wide iff 9 u min(S / eps_min, 2^d) > 1e-4 (u = 2^-24), i.e. FP32 rounding of
// coordinates taken relative to the group's centre could move a close pair's force by more
// than 1e-4 of itself.  plev (n bytes) receives the level of every particle's leaf.
hipError_t make_groups(size_t n, int nsys, const int64_t *sys_off, Cells c,
                       const uint64_t *skey, const double *cube, const double *seps,
                       int n_group, Groups g, uint32_t *flag, uint32_t *gcell_at, uint32_t *gpos,
                       uint8_t *plev, uint64_t *partial, DevStatus *st, hipStream_t s);
// list of the wide groups (any order; count in st->wide_groups) and a reset of the persistent
// queue head for the pass that evaluates them
hipError_t wide_group_list(size_t gmax, const Groups g, uint32_t *list, DevStatus *st,
                           hipStream_t s);

// walk: count (fill = false) or fill (fill = true) the interaction lists.
// seg[g]/cap[g] = start and capacity of group g's segment in `list`; EPJ entries grow from
// the front, SPJ entries from the back.  cnt_e/cnt_s receive the exact counts.
// A group whose entries do not fit its segment (or whose segment passes list_cap) writes
// nothing, gets zero counts and is appended to ovf_list (st->list_overflow counts them).
// sel (optional, with nsel): walk only the listed groups (predictor re-walk).
// exchange lists: every ordered domain pair's walk split into sub-walks over the sender's
// frontier (exchange_subwalks(nsys) slots, pair-major); exchange_split writes each slot's
// receiver box, start cell and segment bound (0 = idle) and appends the active slots to sel
// (*nsel of them); exchange_caps sets the segment sizes of the active slots from a count walk
hipError_t exchange_split(int nsys, const Cells c, const uint64_t *bbox_u, const double *cube,
                          double theta2, uint32_t *front, uint32_t *fcount, uint32_t *box,
                          uint32_t *start, uint32_t *cap, uint32_t *sel, uint32_t *nsel,
                          hipStream_t s);
hipError_t exchange_caps(size_t G, const uint32_t *sel, const uint32_t *nsel, const uint32_t *ne,
                         const uint32_t *ns, uint32_t *cap, hipStream_t s);
size_t exchange_subwalks(int nsys);
constexpr int kExchangeFrontierMax = 64;
// short-range walks: search radius per group (rg, or r_fixed for every group when rg is
// null), largest support radius per cell (hmax), root cube per system (cube)
struct ShortArgs {
    const double *rg = nullptr;
    const double *hmax = nullptr;
    const double *cube = nullptr;
    double r_fixed = 0.0;
};
// spill (fill only): a group whose list outgrew its segment moves to the space after all
// segments (st->list_total + st->spill_used, up to list_cap; seg / cap rewritten) and is walked
// again; st->spilled counts such groups.  Without room it is left empty and queued in ovf_list.
hipError_t walk(bool fill, size_t gmax, const Groups g, const Cells c, double theta2,
                uint64_t *seg, uint32_t *cap, uint64_t list_cap, uint32_t *list,
                uint32_t *cnt_e, uint32_t *cnt_s, uint32_t *ovf_list, const uint32_t *sel,
                const uint32_t *nsel, DevStatus *st, hipStream_t s, bool spill = false);
// the same lists (as sets; the order differs) from walks that share the upper tree between
// runs of consecutive groups; for the tree's own groups (g.sys holds each group's system)
hipError_t walk_runs(bool fill, size_t gmax, const Groups g, const Cells c, double theta2,
                     uint64_t *seg, uint32_t *cap, uint64_t list_cap, uint32_t *list,
                     uint32_t *cnt_e, uint32_t *cnt_s, uint32_t *ovf_list, const uint32_t *sel,
                     const uint32_t *nsel, DevStatus *st, hipStream_t s, bool spill = false);
// short-range walk (kind 1: group radius, 2: cell radius, 3: the larger; no superparticles)
// or the TreePM cutoff walk (kind 4: cells beyond sa.r_fixed dropped, opening angle theta
// for the rest)
hipError_t walk_short(bool fill, int kind, size_t gmax, const Groups g, const Cells c,
                      const ShortArgs sa, double theta2, const uint64_t *seg, const uint32_t *cap,
                      uint64_t list_cap, uint32_t *list, uint32_t *cnt_e, uint32_t *cnt_s,
                      uint32_t *ovf_list, DevStatus *st, hipStream_t s);
// SPH density on short-range lists (k_sph.hip): support radii in sorted order (h given, else
// r_fixed; a non-positive or non-finite radius sets bad_input), largest radius per cell
// (bottom-up) and per group, density and neighbour count per sorted particle (mode 0 fixed,
// 1 scatter, 2 gather, 3 symmetric), and their return to the caller's order
hipError_t sph_radius(size_t n, const uint32_t *perm, const double *h, double r_fixed,
                      double *sh, DevStatus *st, hipStream_t s);
hipError_t sph_cell_hmax(const Cells c, const double *sh, double *hmax, hipStream_t s);
hipError_t sph_group_hmax(size_t gmax, const Groups g, const double *sh, double *rg,
                          DevStatus *st, hipStream_t s);
hipError_t sph_density(int mode, size_t gmax, const Groups g, const uint64_t *seg,
                       const uint32_t *cnt_e, const uint32_t *list, const double4 *jp,
                       const double *sh, double *rho_s, uint32_t *n_s, DevStatus *st,
                       hipStream_t s);
hipError_t sph_unsort(size_t n, const uint32_t *inv, const double *rho_s, const uint32_t *n_s,
                      double *rho, uint32_t *nngb, hipStream_t s);
// domain decomposition (k_dd.hip): cost of each current domain from the last walk (sum of
// members x list length over its groups, added to cost), samples of the current domains,
// one division pass over samples sorted by (segment, coordinate), destination (the grouping
// key) of every particle, the (destination, source) runs of the grouped order, and the
// gather of up to 8 FP64 arrays into the new order
struct DdArrays {
    double *p[8];
};
hipError_t dd_cost(uint32_t G, const uint32_t *g_sys, const uint32_t *g_count,
                   const uint32_t *cnt_e, const uint32_t *cnt_s, uint64_t *cost, hipStream_t s);
hipError_t dd_sample(uint32_t K, uint32_t nsys, const int64_t *kofs, const int64_t *off,
                     uint64_t seed, const double *x, const double *y, const double *z,
                     uint32_t *idx, double *sx, double *sy, double *sz, uint64_t *key,
                     uint32_t *val, hipStream_t s);
hipError_t dd_cut(uint32_t K, uint32_t nseg, const uint32_t *start, uint32_t n,
                  const uint32_t *val, const double *coord, const double *next, uint32_t *cell,
                  uint32_t *new_start, double *face, uint64_t *key_next, uint32_t *val_next,
                  hipStream_t s);
hipError_t dd_assign(uint32_t n, const double *x, const double *y, const double *z, uint32_t nx,
                     uint32_t ny, uint32_t nz, const double *bx, const double *by,
                     const double *bz, uint32_t *dest, uint64_t *key, uint32_t *val,
                     hipStream_t s);
hipError_t dd_runs(uint32_t n, const uint64_t *dest, const uint32_t *order,
                   const uint32_t *sysid, uint32_t nsrc, uint32_t *run_lo, uint32_t *run_hi,
                   hipStream_t s);
hipError_t dd_gather(uint32_t n, const uint32_t *order, int narr, const DdArrays &src,
                     const DdArrays &dst, hipStream_t s);

// FP64 direct summation for nt target particles (caller's order indices) over their
// systems; out = 4 per target (ax, ay, az, phi)
hipError_t direct_forces(uint32_t nt, const uint32_t *targets, const double *x, const double *y,
                         const double *z, const double *m, const double *eps, double eps_all,
                         const uint32_t *sysid, const int64_t *sys_off, double *out,
                         hipStream_t s);

// walk + force in one persistent launch (k_fused.hip): each wave pops a group, walks it and
// evaluates the entries in tiles of 64 as the walk emits them; no list is stored unless `list`
// is given (then every group's entries are also written to its segment [seg, seg + cap):
// particles from the front, superparticles from the back).  Groups come from eight per-XCD runs
// [bounds[x], bounds[x+1]) in tree order, or, with order, from order[k] for k < *count.
struct FusedArgs {
    Groups g;
    const uint4 *node;
    const uint2 *link;
    uint32_t ccap;
    const double4 *jp;
    const double *seps;
    const double *mom;
    double theta2;
    const uint32_t *bounds;
    const uint32_t *order;
    const uint32_t *count;
    uint32_t *cnt_e, *cnt_s;
    const uint64_t *seg;
    const uint32_t *cap;
    uint32_t *list;
    double4 *fs;
    DevStatus *st;
    int skip_wide;           // FP32 pass: groups flagged wide are left to an FP64 pass
};
constexpr int kFusedMaxGroup = 256;      // largest n_group the fused kernel takes
// bounds[0..8] of the eight per-XCD runs of groups (tree order) at equal cumulative cost:
// members x (|EPJ| + ws |SPJ|) with the walk's counts (cnt_e, cnt_s), else members x exp(y)
// with predicted ln lengths y, else members; cost: G words, pre: G + 1 words of scratch
hipError_t queue_bounds(size_t gmax, const uint32_t *gcount, const float *y,
                        const uint32_t *cnt_e, const uint32_t *cnt_s, float ws, uint32_t *cost,
                        uint64_t *pre, uint32_t *bounds, uint64_t *partial, DevStatus *st,
                        hipStream_t s);
hipError_t fused(size_t gmax, const FusedArgs &a, bool fp32, bool quad, int n_group,
                 hipStream_t s);

hipError_t list_caps(size_t gmax, const uint32_t *cnt_e, const uint32_t *cnt_s, uint32_t *cap,
                     DevStatus *st, hipStream_t s);
// lists out of their segments: epj[oe[g] ...] and spj[os[g] ...] (offsets exclusive sums)
hipError_t compact_lists(size_t G, const uint64_t *seg, const uint32_t *cap,
                         const uint32_t *cnt_e, const uint32_t *cnt_s, const uint64_t *oe,
                         const uint64_t *os, const uint32_t *list, uint32_t *epj, uint32_t *spj,
                         hipStream_t s);
// cap[g] = sys_cap[system of g]
hipError_t sys_caps(size_t gmax, const uint32_t *gsys, const uint32_t *sys_cap, uint32_t *cap,
                    DevStatus *st, hipStream_t s);
// lmax[s] = max over the groups of system s of |EPJ| + |SPJ|, gcount[s] = groups of system
// s (both zeroed by the caller); gmax must not exceed the group arrays' current size
hipError_t sys_lmax(size_t gmax, const uint32_t *gsys, const uint32_t *cnt_e,
                    const uint32_t *cnt_s, uint32_t *lmax, uint32_t *gcount, DevStatus *st,
                    hipStream_t s);
hipError_t list_stats(size_t gmax, const Groups g, const uint32_t *cnt_e,
                      const uint32_t *cnt_s, DevStatus *st, hipStream_t s);

// force
struct ForceArgs {
    const Groups *g;
    const double4 *jp;      // sorted x, y, z, m
    const double *seps;     // sorted eps
    const double *mom;
    const uint64_t *seg;
    const uint32_t *cap, *cnt_e, *cnt_s;
    const uint32_t *list;   // interaction list segments
    const uint32_t *order;  // queue order (null: group order)
    const uint32_t *bounds = nullptr;  // persistent launch: the eight per-XCD runs (null: equal
                                       // group counts)
    double4 *fs;            // sorted output {ax, ay, az, phi}
    DevStatus *st;
    bool quad, fp32, persistent;
    int variant;            // kernel shape chosen by the autotuner
    double r_cut = 0.0;     // > 0: tree part of TreePM (monopole, S2 cutoff), no potential
    const uint32_t *count = nullptr;   // persistent launch: device group count (default: all)
};
// G = number of groups (direct launch: one workgroup per group; persistent launch: G bounds
// the grid and the kernel reads the true count from the device status).
hipError_t force(size_t G, const ForceArgs &a, hipStream_t s);
int force_variants();
const char *force_variant_name(int v);
int force_variant_capacity(int v);   // largest group one workgroup of variant v takes
// scratch (private) bytes per lane of variant v's kernel for this precision, moment order and
// launch: > 0 when its registers spill to memory (-1 if the runtime cannot tell)
int force_variant_scratch(bool fp32, bool quad, bool persistent, int v);

}  // namespace fdx
