// C ABI (include/fdx.h) and host orchestration of the gfx950 Barnes-Hut hot path.
//
// One force evaluation is one pass over: root cubes and keys -> radix sort -> sorted
// particle gather -> level-by-level octree -> bottom-up moments -> groups -> walk (count,
// scan, fill) -> force kernel -> return of forces to the caller's order.  Everything runs on
// the bound stream; the host waits once per evaluation, after the counting walk, to size
// the list buffer (and to read the device status: bad input, tree overflow).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "ctx.h"

using namespace fdx;

namespace fdx {

int fail(fdx_ctx *c, int code, const char *fmt, ...) {
    if (!c) return code;
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(c->err, sizeof c->err, fmt, ap);
    va_end(ap);
    return code;
}

}  // namespace fdx

namespace fdx {

bool finite_all(const double *p, int64_t n) {
    for (int64_t i = 0; i < n; i++)
        if (!std::isfinite(p[i])) return false;
    return true;
}

int ensure_tree_buffers(fdx_ctx *c, uint32_t cell_cap, uint32_t group_cap) {
    const size_t n = (size_t)c->n, S = (size_t)c->nsys;
    if (cell_cap > c->cell_cap || !c->c_level.p) {
        c->gen++;
        HIPCHK(c, c->c_level.ensure(cell_cap));
        HIPCHK(c, c->c_begin.ensure(cell_cap));
        HIPCHK(c, c->c_count.ensure(cell_cap));
        HIPCHK(c, c->c_first.ensure(cell_cap));
        HIPCHK(c, c->c_nchild.ensure(cell_cap));
        HIPCHK(c, c->c_parent.ensure(cell_cap));
        HIPCHK(c, c->c_prefix.ensure(cell_cap));
        HIPCHK(c, c->c_node.ensure(cell_cap));
        HIPCHK(c, c->c_link.ensure(cell_cap));
        HIPCHK(c, c->c_mom.ensure(10 * (size_t)cell_cap));
        c->cell_cap = cell_cap;
    }
    HIPCHK(c, c->c_lvl.ensure(kLevels + 2));
    HIPCHK(c, c->f_bounds.ensure(9));
    HIPCHK(c, c->tmp_n.ensure(n + S + 1));                 // >= 3 n bytes
    HIPCHK(c, c->tmp_off.ensure(std::max(n + S + 2, tree_scratch_u32(n))));
    if (group_cap > c->group_cap || !c->g_cell.p) {
        c->gen++;
        HIPCHK(c, c->g_cell.ensure(group_cap));
        HIPCHK(c, c->g_begin.ensure(group_cap));
        HIPCHK(c, c->g_count.ensure(group_cap));
        HIPCHK(c, c->g_sys.ensure(group_cap));
        HIPCHK(c, c->g_box.ensure(6 * (size_t)group_cap));
        HIPCHK(c, c->g_centre.ensure(3 * (size_t)group_cap));
        HIPCHK(c, c->g_wide.ensure(group_cap));
        HIPCHK(c, c->wide_list.ensure(group_cap));
        HIPCHK(c, c->cnt_e.ensure(group_cap));
        HIPCHK(c, c->cnt_s.ensure(group_cap));
        HIPCHK(c, c->lcap.ensure(group_cap));
        HIPCHK(c, c->seg.ensure((size_t)group_cap + 1));
        HIPCHK(c, c->ovf_list.ensure(group_cap));
        HIPCHK(c, c->rs_scratch.ensure(radix_scratch_u32(std::max<size_t>(n, group_cap))));
        HIPCHK(c, c->f_cost.ensure(group_cap));
        HIPCHK(c, c->f_pre.ensure((size_t)group_cap + 1));
        c->group_cap = group_cap;
    }
    return FDX_OK;
}

Cells cells_view(fdx_ctx *c) {
    Cells v;
    v.level = c->c_level.p; v.begin = c->c_begin.p; v.count = c->c_count.p;
    v.first = c->c_first.p; v.nchild = c->c_nchild.p; v.parent = c->c_parent.p;
    v.prefix = c->c_prefix.p; v.node = c->c_node.p; v.link = c->c_link.p; v.mom = c->c_mom.p;
    v.lvl = c->c_lvl.p; v.cap = c->cell_cap;
    return v;
}

Groups groups_view(fdx_ctx *c) {
    Groups g;
    g.cell = c->g_cell.p; g.begin = c->g_begin.p; g.count = c->g_count.p; g.sys = c->g_sys.p;
    g.box = c->g_box.p; g.centre = c->g_centre.p; g.wide = c->g_wide.p; g.cap = c->group_cap;
    return g;
}

void mark(fdx_ctx *c, int k) {
    if (c->flags & FDX_TIMING) (void)hipEventRecord(c->ev[k], c->stream);
}

int read_status(fdx_ctx *c) {
    HIPCHK(c, hipMemcpyAsync(&c->hst->st, c->st, sizeof(DevStatus), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipMemcpyAsync(c->hst->lvl, c->c_lvl.p, sizeof(uint32_t) * (kLevels + 2),
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return FDX_OK;
}

// Keys, sort and sorted gather (no host wait).  Resets the device status first.
int enqueue_keys_sort(fdx_ctx *c) {
    const size_t n = (size_t)c->n;
    const int S = c->nsys;
    hipStream_t s = c->stream;
    HIPCHK(c, fill_u32((uint32_t *)c->st, 0u, sizeof(DevStatus) / 4, s));
    if (c->borrowed || !c->eps_given)
        HIPCHK(c, check_input(n, c->x, c->y, c->z, c->m, c->eps_given ? c->eps : nullptr, c->st, s));
    mark(c, 0);
    HIPCHK(c, bbox(n, c->x, c->y, c->z, c->sysid.p, S, c->bbox_u.p, s));
    HIPCHK(c, root_cubes(S, c->bbox_u.p, c->cube.p, s));
    HIPCHK(c, morton_keys(n, c->x, c->y, c->z, c->m, c->sysid.p, S, c->cube.p, c->key.p,
                          c->perm.p, c->packed.p, s));
    mark(c, 1);
    bool alt = false;
    HIPCHK(c, radix_sort(n, c->key.p, c->key_alt.p, c->perm.p, c->perm_alt.p, c->sysid.p, S, 64,
                         c->rs_scratch.p, c->partial.p, &alt, s,
                         S > 1 && S <= 65536 && c->sys_carry.cap >= 2 * n ? c->sys_carry.p
                                                                           : nullptr));
    c->skey = alt ? c->key_alt.p : c->key.p;
    c->sperm = alt ? c->perm_alt.p : c->perm.p;
    HIPCHK(c, gather_sorted(n, c->sperm, c->packed.p, c->eps_given ? c->eps : nullptr,
                            c->eps_all, c->eps_given && c->eps_per_system, c->sys_off.p, S,
                            c->jp.p, c->seps.p, c->inv.p, s));
    mark(c, 2);
    return FDX_OK;
}

// Cells, moments and groups at the current capacities (no host wait).
int enqueue_tree_groups(fdx_ctx *c) {
    const size_t n = (size_t)c->n;
    const int S = c->nsys;
    hipStream_t s = c->stream;
    HIPCHK(c, tree_build(n, S, c->sys_off.p, c->skey, c->n_leaf, cells_view(c),
                         (uint8_t *)c->tmp_n.p, c->tmp_off.p, c->partial.p, c->st, s));
    mark(c, 3);
    HIPCHK(c, tree_moments(cells_view(c), c->jp.p, s));
    mark(c, 4);
    HIPCHK(c, make_groups(n, S, c->sys_off.p, cells_view(c), c->skey, c->cube.p, c->seps.p,
                          c->n_group, groups_view(c), c->flag.p, c->gcell_at.p, c->gpos.p,
                          c->leaf_lev.p, c->partial.p, c->st, s));
    mark(c, 5);
    return FDX_OK;
}

// Tree part of one evaluation with host checks: retries with larger cell / group capacity
// when the device reports an overflow.  Leaves the status (group count, levels) in c->hst.
int run_tree(fdx_ctx *c, bool sync) {
    c->have_lists = false;
    c->have_counts = false;
    int r = enqueue_keys_sort(c);
    if (r) return r;
    for (int attempt = 0;; attempt++) {
        r = enqueue_tree_groups(c);
        if (r) return r;
        if (!sync) return FDX_OK;
        r = read_status(c);
        if (r) return r;
        const DevStatus &h = c->hst->st;
        if (h.bad_input)
            return fail(c, FDX_EINVAL, "particle data has a non-finite value, a negative mass "
                                       "or eps <= 0");
        bool grow = false;
        uint32_t ncap = c->cell_cap, gcap = c->group_cap;
        if (h.cell_overflow) {
            ncap = (uint32_t)std::min<uint64_t>(2ull * c->cell_cap, 0xFFFFFFF0ull);
            grow = true;
        }
        if (h.group_overflow || h.n_groups > c->group_cap) {
            gcap = h.n_groups + h.n_groups / 8 + 1024;
            grow = true;
        }
        if (!grow) return FDX_OK;
        if (attempt > 8) return fail(c, FDX_EHIP, "tree capacity did not converge");
        r = ensure_tree_buffers(c, ncap, gcap);
        if (r) return r;
        HIPCHK(c, fill_u32((uint32_t *)c->st, 0u, sizeof(DevStatus) / 4, c->stream));
    }
}

// Exact walk, first half: count pass, segment sizes and offsets (device total in
// st->list_total).  gmax bounds the groups (the host count, or the capacity when captured).
static ShortArgs cutoff_args(fdx_ctx *c) {
    ShortArgs sa;
    sa.cube = c->cube.p;
    sa.r_fixed = c->cutoff;
    return sa;
}

int enqueue_count(fdx_ctx *c, size_t gmax) {
    hipStream_t s = c->stream;
    Groups gv = groups_view(c);
    if (c->cutoff > 0)
        HIPCHK(c, walk_short(false, 4, gmax, gv, cells_view(c), cutoff_args(c), c->theta * c->theta,
                             nullptr, nullptr, 0, nullptr, c->cnt_e.p, c->cnt_s.p, c->ovf_list.p,
                             c->st, s));
    else
        HIPCHK(c, walk_runs(false, gmax, gv, cells_view(c), c->theta * c->theta, nullptr,
                            nullptr, 0, nullptr, c->cnt_e.p, c->cnt_s.p, c->ovf_list.p, nullptr,
                            nullptr, c->st, s));
    HIPCHK(c, list_caps(gmax, c->cnt_e.p, c->cnt_s.p, c->lcap.p, c->st, s));
    HIPCHK(c, scan_u32_to_u64(c->lcap.p, c->seg.p, 0, nullptr, &c->st->n_groups_c, c->partial.p,
                              &c->st->list_total, s));
    return FDX_OK;
}

int enqueue_sys_caps(fdx_ctx *c, size_t gmax, const uint32_t *sys_cap) {
    hipStream_t s = c->stream;
    HIPCHK(c, sys_caps(gmax, c->g_sys.p, sys_cap, c->lcap.p, c->st, s));
    HIPCHK(c, scan_u32_to_u64(c->lcap.p, c->seg.p, 0, nullptr, &c->st->n_groups_c, c->partial.p,
                              &c->st->list_total, s));
    return FDX_OK;
}

// Fill pass into the list buffer (its capacity guards every write), then counters.
int enqueue_fill(fdx_ctx *c, size_t gmax, bool spill) {
    hipStream_t s = c->stream;
    Groups gv = groups_view(c);
    if (c->cutoff > 0)
        HIPCHK(c, walk_short(true, 4, gmax, gv, cells_view(c), cutoff_args(c), c->theta * c->theta,
                             c->seg.p, c->lcap.p, c->list_cap, c->list.p, c->cnt_e.p, c->cnt_s.p,
                             c->ovf_list.p, c->st, s));
    else
        HIPCHK(c, walk_runs(true, gmax, gv, cells_view(c), c->theta * c->theta, c->seg.p,
                            c->lcap.p, c->list_cap, c->list.p, c->cnt_e.p, c->cnt_s.p,
                            c->ovf_list.p, nullptr, nullptr, c->st, s, spill));
    return FDX_OK;
}

// Force kernel and return of forces.  G = host group count (direct launch) or 0 with
// persistent kernels (device count).
int enqueue_force(fdx_ctx *c, size_t gmax) {
    hipStream_t s = c->stream;
    const size_t n = (size_t)c->n;
    Groups gv = groups_view(c);
    HIPCHK(c, list_stats(gmax, gv, c->cnt_e.p, c->cnt_s.p, c->st, s));
    const bool persistent = (c->flags & FDX_PERSISTENT) != 0;
    if (persistent)
        // the eight per-XCD runs cut at equal cost from the walk's exact counts: members x
        // (|EPJ| + w |SPJ|), w = a superparticle's cost in particle terms (the inner loops issue
        // 34.5 / 14.25 instructions per quadrupole / particle interaction; a monopole costs
        // about as much as a particle)
        HIPCHK(c, queue_bounds(gmax, gv.count, nullptr, c->cnt_e.p, c->cnt_s.p,
                               (c->flags & FDX_QUAD) ? 2.4f : 1.0f, c->f_cost.p, c->f_pre.p,
                               c->f_bounds.p, c->partial.p, c->st, s));
    mark(c, 6);
    ForceArgs fa;
    fa.g = &gv; fa.jp = c->jp.p; fa.seps = c->seps.p; fa.mom = c->c_mom.p;
    fa.seg = c->seg.p; fa.cap = c->lcap.p; fa.cnt_e = c->cnt_e.p; fa.cnt_s = c->cnt_s.p;
    fa.list = c->list.p; fa.order = nullptr; fa.fs = c->fs.p; fa.st = c->st;
    fa.quad = (c->flags & FDX_QUAD) != 0;
    fa.fp32 = (c->flags & FDX_FP32REL) != 0;
    fa.persistent = persistent;
    fa.bounds = persistent ? c->f_bounds.p : nullptr;
    fa.variant = ext_force_variant(c);
    fa.r_cut = c->cutoff;
    HIPCHK(c, force(gmax, fa, s));
    if (fa.fp32) {
        // groups too wide for group-relative FP32: evaluated again by the FP64 kernel, which
        // overwrites their rows (one persistent pass over the device-side list; empty when no
        // group is wide)
        HIPCHK(c, wide_group_list(gmax, gv, c->wide_list.p, c->st, s));
        ForceArgs fw = fa;
        fw.fp32 = false;
        fw.persistent = true;
        fw.order = c->wide_list.p;
        fw.count = &c->st->wide_groups;
        fw.variant = 5;                    // the FP64 default shape
        HIPCHK(c, force(gmax, fw, s));
    }
    mark(c, 7);
    HIPCHK(c, unsort_forces(n, c->fs.p, c->inv.p, c->ax.p, c->ay.p, c->az.p, c->pot.p, s));
    mark(c, 8);
    return FDX_OK;
}

int enqueue_fused(fdx_ctx *c, size_t gmax, bool capture) {
    hipStream_t s = c->stream;
    const size_t n = (size_t)c->n;
    Groups gv = groups_view(c);
    Cells cv = cells_view(c);
    // queue runs at equal cumulative cost (members x predicted list length, or members)
    const float *y = nullptr;
    if (c->flags & FDX_PREDICTOR) {
        const int r = ext_predicted_lengths(c, gmax, &y);
        if (r) return r;
    }
    HIPCHK(c, queue_bounds(gmax, gv.count, y, nullptr, nullptr, 0.0f, c->f_cost.p, c->f_pre.p,
                           c->f_bounds.p, c->partial.p, c->st, s));
    mark(c, 6);
    FusedArgs fa{};
    fa.g = gv;
    fa.node = cv.node; fa.link = cv.link; fa.ccap = cv.cap;
    fa.jp = c->jp.p; fa.seps = c->seps.p; fa.mom = c->c_mom.p;
    fa.theta2 = c->theta * c->theta;
    fa.bounds = c->f_bounds.p; fa.order = nullptr; fa.count = nullptr;
    fa.cnt_e = c->cnt_e.p; fa.cnt_s = c->cnt_s.p;
    fa.seg = capture ? c->seg.p : nullptr;
    fa.cap = capture ? c->lcap.p : nullptr;
    fa.list = capture ? c->list.p : nullptr;
    fa.fs = c->fs.p; fa.st = c->st;
    const bool fp32 = (c->flags & FDX_FP32REL) != 0, quad = (c->flags & FDX_QUAD) != 0;
    fa.skip_wide = fp32 ? 1 : 0;
    HIPCHK(c, fused(gmax, fa, fp32, quad, c->n_group, s));
    if (fp32) {
        // groups too wide for group-relative FP32: a second pass of the FP64 kernel over the
        // device-side list of them (empty when no group is wide)
        HIPCHK(c, wide_group_list(gmax, gv, c->wide_list.p, c->st, s));
        FusedArgs fw = fa;
        fw.order = c->wide_list.p;
        fw.count = &c->st->wide_groups;
        fw.skip_wide = 0;
        HIPCHK(c, fused(gmax, fw, false, quad, c->n_group, s));
    }
    HIPCHK(c, list_stats(gmax, gv, c->cnt_e.p, c->cnt_s.p, c->st, s));
    mark(c, 7);
    HIPCHK(c, unsort_forces(n, c->fs.p, c->inv.p, c->ax.p, c->ay.p, c->az.p, c->pot.p, s));
    mark(c, 8);
    return FDX_OK;
}

int ensure_list_capacity(fdx_ctx *c, uint64_t total) {
    if (total > c->list_cap || !c->list.p) {
        c->gen++;
        const uint64_t want = total + total / 8 + 1024;
        HIPCHK(c, c->list.ensure(want));
        c->list_cap = want;
    }
    return FDX_OK;
}

// Walk + force + return of forces (eager).  Needs run_tree(sync=true) first.
int run_force(fdx_ctx *c) {
    const uint32_t G = c->hst->st.n_groups;
    int r;
    c->predict_marked = false;
    if (c->flags & FDX_FUSED) {
        const bool capture = c->capture_lists;
        if (capture) {
            // exact list sizes for the entries the fused kernel will store as it evaluates them
            r = enqueue_count(c, G);
            if (!r) r = read_status(c);
            if (r) return r;
            if (c->hst->st.walk_error) return fail(c, FDX_EHIP, "walk stack exhausted");
            r = ensure_list_capacity(c, c->hst->st.list_total);
            if (r) return r;
            c->stats.list_capacity = (int64_t)c->hst->st.list_total;
        } else {
            c->stats.list_capacity = 0;
        }
        c->stats.overflow_groups = 0;
        r = enqueue_fused(c, G, capture);
        if (r) return r;
        c->have_counts = true;
        c->have_lists = capture;
        c->have_force = true;
        return FDX_OK;
    }
    if (c->flags & FDX_PREDICTOR) {
        r = ext_predicted_walk(c, G);
        if (r) return r;
    } else {
        r = enqueue_count(c, G);
        if (r) return r;
        r = read_status(c);
        if (r) return r;
        if (c->hst->st.walk_error) return fail(c, FDX_EHIP, "walk stack exhausted");
        const uint64_t total = c->hst->st.list_total;
        r = ensure_list_capacity(c, total);
        if (r) return r;
        r = enqueue_fill(c, G);
        if (r) return r;
        c->stats.list_capacity = (int64_t)total;
        c->stats.overflow_groups = 0;
    }
    c->have_lists = true;
    c->have_counts = true;
    r = enqueue_force(c, G);
    if (r) return r;
    c->have_force = true;
    return FDX_OK;
}

}  // namespace fdx

namespace fdx {

int setup_eval(fdx_ctx *c, double theta, int n_leaf, int n_group, double eps, int flags) {
    if (!c) return FDX_EINVAL;
    if (!c->have_particles) return fail(c, FDX_ESTATE, "no particles: call fdx_set_particles first");
    if (!(theta > 0.0 && theta <= 1.0)) return fail(c, FDX_EINVAL, "theta must be in (0, 1]");
    if (n_leaf < 1) return fail(c, FDX_EINVAL, "n_leaf must be >= 1");
    if (n_group < 1 || n_group > kMaxGroup) return fail(c, FDX_EINVAL, "n_group must be in [1, %d]", kMaxGroup);
    if (!c->eps_given && !(std::isfinite(eps) && eps > 0.0))
        return fail(c, FDX_EINVAL, "eps must be finite and > 0");
    if ((flags & FDX_FUSED) && n_group > kFusedMaxGroup)
        return fail(c, FDX_EINVAL, "FDX_FUSED takes n_group <= %d", kFusedMaxGroup);
    if (flags & FDX_FUSED) flags |= FDX_PERSISTENT;
    c->theta = theta; c->n_leaf = n_leaf; c->n_group = n_group; c->eps_all = eps;
    c->flags = flags;
    const size_t n = (size_t)c->n, S = (size_t)c->nsys;
    uint32_t ccap = std::max<uint32_t>(c->cell_cap, (uint32_t)std::min<uint64_t>(n + S + 1024, 0xFFFFFFF0ull));
    uint32_t gcap = std::max<uint32_t>(c->group_cap, (uint32_t)(n / 8 + S + 1024));
    return ensure_tree_buffers(c, ccap, gcap);
}

void save_force_params(fdx_ctx *c) {
    fdx_ctx::ForceParams &p = c->last_force;
    p.theta = c->theta; p.eps_all = c->eps_all; p.cutoff = c->cutoff;
    p.n_leaf = c->n_leaf; p.n_group = c->n_group; p.flags = c->flags;
}

void restore_force_params(fdx_ctx *c) {
    const fdx_ctx::ForceParams &p = c->last_force;
    c->theta = p.theta; c->eps_all = p.eps_all; c->cutoff = p.cutoff;
    c->n_leaf = p.n_leaf; c->n_group = p.n_group; c->flags = p.flags;
}

void finish_stats(fdx_ctx *c) {
    fdx_stats &o = c->stats;
    const DevStatus &h = c->hst->st;
    o.n = c->n; o.n_sys = c->nsys;
    o.n_cells = c->hst->lvl[kLevels + 1];
    o.n_groups = h.n_groups;
    int depth = 0;
    for (int l = 0; l <= kLevels; l++)
        if (c->hst->lvl[l + 1] > c->hst->lvl[l]) depth = l;
    o.depth = depth;
    o.n_leaf = c->n_leaf; o.n_group = c->n_group; o.flags = c->flags; o.theta = c->theta;
    o.shape = ext_force_variant(c);
    o.graph_recoveries = c->ext.graph_recoveries;
    o.list_spills = c->ext.list_spills;
}

int sync_timing(fdx_ctx *c) {
    if (!(c->flags & FDX_TIMING)) return FDX_OK;
    HIPCHK(c, hipEventSynchronize(c->ev[8]));
    float t[9] = {};
    for (int k = 0; k < 8; k++) hipEventElapsedTime(&t[k], c->ev[k], c->ev[k + 1]);
    fdx_stats &o = c->stats;
    o.t_keys = t[0]; o.t_sort = t[1]; o.t_tree = t[2]; o.t_moments = t[3]; o.t_groups = t[4];
    o.t_walk = t[5]; o.t_force = t[6]; o.t_unsort = t[7];
    o.t_predict = 0.0;
    if (c->flags & FDX_FUSED) {
        // queue boundaries (and the predictor's network) before the one walk + force launch
        o.t_predict = o.t_walk;
        o.t_walk = 0.0;
    } else if (c->predict_marked) {
        // predicted walk: features + network + capacities (event 5 -> 9), then the walk
        float tp = 0.0f, tw = 0.0f;
        hipEventElapsedTime(&tp, c->ev[5], c->ev[9]);
        hipEventElapsedTime(&tw, c->ev[9], c->ev[6]);
        o.t_predict = tp;
        o.t_walk = tw;
    }
    float tot = 0;
    hipEventElapsedTime(&tot, c->ev[0], c->ev[8]);
    o.t_total = tot;
    return FDX_OK;
}

int read_counters(fdx_ctx *c) {
    HIPCHK(c, hipMemcpyAsync(&c->hst->st, c->st, sizeof(DevStatus), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const DevStatus &h = c->hst->st;
    if (h.walk_error) return fail(c, FDX_EHIP, "walk stack exhausted");
    if ((c->flags & FDX_FUSED) && h.list_overflow)
        return fail(c, FDX_EHIP, "a captured list outgrew its counted size");
    c->stats.n_epj = (int64_t)h.n_epj;
    c->stats.n_spj = (int64_t)h.n_spj;
    c->stats.n_interactions_pp = (int64_t)h.inter_pp;
    c->stats.n_interactions_pc = (int64_t)h.inter_pc;
    c->stats.fp64_groups = (c->flags & FDX_FP32REL) ? (int64_t)h.wide_groups : 0;
    return FDX_OK;
}

}  // namespace fdx

extern "C" {

int fdx_create(fdx_ctx **out, int device, void *hip_stream) {
    FDX_ABI_TRY
    if (!out) return FDX_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return FDX_EINVAL;
    fdx_ctx *c = new (std::nothrow) fdx_ctx();
    if (!c) return FDX_ENOMEM;
    c->device = device;
    if (hipSetDevice(device) != hipSuccess) { delete c; return FDX_EHIP; }
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreate(&c->stream) != hipSuccess) { delete c; return FDX_EHIP; }
        c->own_stream = true;
    }
    if (hipMalloc((void **)&c->st, sizeof(DevStatus)) != hipSuccess ||
        hipHostMalloc((void **)&c->hst, sizeof(HostStatus), hipHostMallocDefault) != hipSuccess) {
        fdx_destroy(c);
        return FDX_ENOMEM;
    }
    memset(c->hst, 0, sizeof(HostStatus));
    for (auto &e : c->ev)
        if (hipEventCreate(&e) != hipSuccess) { fdx_destroy(c); return FDX_EHIP; }
    if (c->partial.ensure(kScanBlocks + 1) != hipSuccess) { fdx_destroy(c); return FDX_ENOMEM; }
    *out = c;
    return FDX_OK;
    FDX_ABI_CATCH(nullptr)
}

int fdx_destroy(fdx_ctx *c) {
    FDX_ABI_TRY
    if (!c) return FDX_OK;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    ext_release(c);
    c->each_buffer([](auto &b) { b.release(); });
    if (c->st) (void)hipFree(c->st);
    if (c->hst) (void)hipHostFree(c->hst);
    for (auto &e : c->ev)
        if (e) (void)hipEventDestroy(e);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return FDX_OK;
    FDX_ABI_CATCH(c)
}

int fdx_set_particles(fdx_ctx *c, int64_t n, const double *x, const double *y, const double *z,
                      const double *vx, const double *vy, const double *vz, const double *m,
                      const double *eps, const int64_t *sys_off, int32_t n_sys, int32_t mem_kind) {
    FDX_ABI_TRY
    if (!c) return FDX_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, FDX_EHIP, "hipSetDevice failed");
    if (n < 0 || n >= (1ll << 31)) return fail(c, FDX_EINVAL, "n must be in [0, 2^31)");
    if (mem_kind != FDX_MEM_HOST && mem_kind != FDX_MEM_DEVICE)
        return fail(c, FDX_EINVAL, "mem_kind must be FDX_MEM_HOST or FDX_MEM_DEVICE");
    if (n > 0 && (!x || !y || !z || !vx || !vy || !vz || !m))
        return fail(c, FDX_EINVAL, "null particle array");
    if (n_sys < 1) return fail(c, FDX_EINVAL, "n_sys must be >= 1");
    std::vector<int64_t> off(n_sys + 1);
    if (sys_off) {
        for (int s = 0; s <= n_sys; s++) off[s] = sys_off[s];
        if (off[0] != 0 || off[n_sys] != n) return fail(c, FDX_EINVAL, "sys_off must run from 0 to n");
        for (int s = 0; s < n_sys; s++)
            if (off[s + 1] < off[s]) return fail(c, FDX_EINVAL, "sys_off must be ascending");
    } else {
        if (n_sys != 1) return fail(c, FDX_EINVAL, "sys_off is null but n_sys != 1");
        off[0] = 0; off[1] = n;
    }
    if (mem_kind == FDX_MEM_HOST && n > 0) {
        for (const double *p : {x, y, z, vx, vy, vz, m})
            if (!finite_all(p, n)) return fail(c, FDX_EINVAL, "non-finite particle data");
        for (int64_t i = 0; i < n; i++)
            if (m[i] < 0) return fail(c, FDX_EINVAL, "negative mass");
        if (eps)
            for (int64_t i = 0; i < n; i++)
                if (!(eps[i] > 0.0) || !std::isfinite(eps[i]))
                    return fail(c, FDX_EINVAL, "eps must be finite and > 0");
    }
    c->eps_per_system = false;
    if (mem_kind == FDX_MEM_HOST && eps && n > 0) {
        bool same = true;
        for (int s = 0; s < n_sys && same; s++)
            same = std::all_of(eps + off[s], eps + off[s + 1],
                               [&](double e) { return e == eps[off[s]]; });
        c->eps_per_system = same;
    }
    c->have_particles = false;
    c->have_force = false;
    c->have_lists = false;
    c->have_counts = false;
    c->gen++;
    ext_invalidate(c);
    c->n = n;
    c->nsys = n_sys;
    c->sys_off_h = off;
    c->eps_given = eps != nullptr;
    c->borrowed = mem_kind == FDX_MEM_DEVICE;
    const size_t N = (size_t)n;
    hipStream_t s = c->stream;
    if (c->borrowed) {
        c->x = (double *)x; c->y = (double *)y; c->z = (double *)z;
        c->vx = (double *)vx; c->vy = (double *)vy; c->vz = (double *)vz;
        c->m = (double *)m; c->eps = (double *)eps;
    } else {
        DBuf<double> *bufs[8] = {&c->ox, &c->oy, &c->oz, &c->ovx, &c->ovy, &c->ovz, &c->om, &c->oeps};
        const double *src[8] = {x, y, z, vx, vy, vz, m, eps};
        double **dst[8] = {&c->x, &c->y, &c->z, &c->vx, &c->vy, &c->vz, &c->m, &c->eps};
        for (int k = 0; k < 8; k++) {
            if (!src[k]) { *dst[k] = nullptr; continue; }
            HIPCHK(c, bufs[k]->ensure(N));
            *dst[k] = bufs[k]->p;
            if (N) HIPCHK(c, hipMemcpyAsync(bufs[k]->p, src[k], N * sizeof(double),
                                            hipMemcpyHostToDevice, s));
        }
    }
    HIPCHK(c, c->sys_off.ensure(n_sys + 1));
    HIPCHK(c, hipMemcpyAsync(c->sys_off.p, off.data(), sizeof(int64_t) * (n_sys + 1),
                             hipMemcpyHostToDevice, s));
    HIPCHK(c, c->sysid.ensure(N));
    HIPCHK(c, sysid_fill(c->sys_off.p, n_sys, c->sysid.p, N, s));
    HIPCHK(c, c->bbox_u.ensure(6 * (size_t)n_sys));
    HIPCHK(c, c->cube.ensure(4 * (size_t)n_sys));
    HIPCHK(c, c->key.ensure(N));
    HIPCHK(c, c->key_alt.ensure(N));
    HIPCHK(c, c->perm.ensure(N));
    HIPCHK(c, c->perm_alt.ensure(N));
    HIPCHK(c, c->inv.ensure(N));
    HIPCHK(c, c->rs_scratch.ensure(radix_scratch_u32(N)));
    if (n_sys > 1 && n_sys <= 65536) HIPCHK(c, c->sys_carry.ensure(2 * N));
    HIPCHK(c, c->jp.ensure(N));
    HIPCHK(c, c->packed.ensure(N));
    HIPCHK(c, c->seps.ensure(N));
    HIPCHK(c, c->flag.ensure(N));
    HIPCHK(c, c->gcell_at.ensure(N));
    HIPCHK(c, c->gpos.ensure(N));
    HIPCHK(c, c->leaf_lev.ensure(N));
    HIPCHK(c, c->fs.ensure(N));
    HIPCHK(c, c->ax.ensure(N));
    HIPCHK(c, c->ay.ensure(N));
    HIPCHK(c, c->az.ensure(N));
    HIPCHK(c, c->pot.ensure(N));
    const bool dev_eps = c->borrowed && eps && n > 0;
    if (dev_eps) {
        HIPCHK(c, fill_u32(&c->st->eps_varies, 0u, 1, s));
        HIPCHK(c, eps_varies(N, c->eps, c->sysid.p, c->sys_off.p, &c->st->eps_varies, s));
        HIPCHK(c, hipMemcpyAsync(&c->hst->st.eps_varies, &c->st->eps_varies, sizeof(uint32_t),
                                 hipMemcpyDeviceToHost, s));
    }
    HIPCHK(c, hipStreamSynchronize(s));   // host arrays may be freed by the caller afterwards
    if (dev_eps) c->eps_per_system = c->hst->st.eps_varies == 0;
    c->have_particles = true;
    c->stats = fdx_stats{};
    return FDX_OK;
    FDX_ABI_CATCH(c)
}

int fdx_build_tree(fdx_ctx *c, int32_t n_leaf, int32_t n_group) {
    FDX_ABI_TRY
    if (!c) return FDX_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, FDX_EHIP, "hipSetDevice failed");
    double eps = c->eps_given ? 0.0 : (c->eps_all > 0 ? c->eps_all : 1.0);
    int r = setup_eval(c, c->theta, n_leaf, n_group, eps, c->flags & ~FDX_TIMING);
    if (r) return r;
    r = run_tree(c, true);
    if (r) return r;
    finish_stats(c);
    return FDX_OK;
    FDX_ABI_CATCH(c)
}

int fdx_calc_force(fdx_ctx *c, double theta, int32_t n_leaf, int32_t n_group, double eps,
                   int32_t flags) {
    FDX_ABI_TRY
    if (!c) return FDX_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, FDX_EHIP, "hipSetDevice failed");
    c->cutoff = 0.0;
    int r = setup_eval(c, theta, n_leaf, n_group, eps, flags);
    if (r) return r;
    r = run_tree(c, true);
    if (r) return r;
    r = run_force(c);
    if (r) return r;
    save_force_params(c);
    finish_stats(c);
    r = sync_timing(c);
    if (r) return r;
    return read_counters(c);
    FDX_ABI_CATCH(c)
}

int fdx_calc_force_cutoff(fdx_ctx *c, double theta, int32_t n_leaf, int32_t n_group, double eps,
                          double r_cut, int32_t flags) {
    FDX_ABI_TRY
    if (!c) return FDX_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, FDX_EHIP, "hipSetDevice failed");
    if (!(std::isfinite(r_cut) && r_cut > 0.0)) return fail(c, FDX_EINVAL, "r_cut must be finite and > 0");
    if (flags & (FDX_QUAD | FDX_PREDICTOR | FDX_GRAPH | FDX_FUSED))
        return fail(c, FDX_EINVAL, "the cutoff kernel is monopole only, without predictor, graph "
                                   "or fused launch");
    int r = setup_eval(c, theta, n_leaf, n_group, eps, flags);
    if (r) return r;
    c->cutoff = r_cut;
    r = run_tree(c, true);
    if (r) return r;
    r = run_force(c);
    if (r) return r;
    save_force_params(c);
    finish_stats(c);
    r = sync_timing(c);
    if (r) return r;
    return read_counters(c);
    FDX_ABI_CATCH(c)
}

int fdx_integrate(fdx_ctx *c, double dt, int32_t n_steps, int32_t flags) {
    FDX_ABI_TRY
    if (!c) return FDX_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, FDX_EHIP, "hipSetDevice failed");
    if (!c->have_force) return fail(c, FDX_ESTATE, "evaluate the force once before integrating");
    if (!std::isfinite(dt) || n_steps < 0) return fail(c, FDX_EINVAL, "bad dt or n_steps");
    restore_force_params(c);
    if ((flags & FDX_GRAPH) && c->cutoff > 0)
        return fail(c, FDX_EINVAL, "graph capture is not available with the cutoff kernel");
    if (flags & FDX_GRAPH) return ext_integrate_graph(c, dt, n_steps);
    const size_t n = (size_t)c->n;
    for (int k = 0; k < n_steps; k++) {
        HIPCHK(c, kick_drift(n, c->x, c->y, c->z, c->vx, c->vy, c->vz, c->ax.p, c->ay.p, c->az.p,
                             dt, c->stream));
        int r = run_tree(c, true);
        if (r) return r;
        r = run_force(c);
        if (r) return r;
        HIPCHK(c, kick(n, c->vx, c->vy, c->vz, c->ax.p, c->ay.p, c->az.p, dt, nullptr, c->stream));
    }
    finish_stats(c);
    if (n_steps > 0) {
        int r = sync_timing(c);
        if (r) return r;
    }
    return read_counters(c);
    FDX_ABI_CATCH(c)
}

int fdx_get_particles(fdx_ctx *c, double *x, double *y, double *z, double *vx, double *vy,
                      double *vz, int32_t mem_kind) {
    FDX_ABI_TRY
    if (!c) return FDX_EINVAL;
    if (!c->have_particles) return fail(c, FDX_ESTATE, "no particles");
    hipMemcpyKind k = mem_kind == FDX_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    const size_t bytes = sizeof(double) * (size_t)c->n;
    double *dst[6] = {x, y, z, vx, vy, vz};
    double *src[6] = {c->x, c->y, c->z, c->vx, c->vy, c->vz};
    for (int i = 0; i < 6; i++)
        if (dst[i] && bytes) HIPCHK(c, hipMemcpyAsync(dst[i], src[i], bytes, k, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return FDX_OK;
    FDX_ABI_CATCH(c)
}

int fdx_get_forces(fdx_ctx *c, double *ax, double *ay, double *az, double *pot, int32_t mem_kind) {
    FDX_ABI_TRY
    if (!c) return FDX_EINVAL;
    if (!c->have_force) return fail(c, FDX_ESTATE, "no force evaluated");
    hipMemcpyKind k = mem_kind == FDX_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    const size_t bytes = sizeof(double) * (size_t)c->n;
    double *dst[4] = {ax, ay, az, pot};
    double *src[4] = {c->ax.p, c->ay.p, c->az.p, c->pot.p};
    for (int i = 0; i < 4; i++)
        if (dst[i] && bytes) HIPCHK(c, hipMemcpyAsync(dst[i], src[i], bytes, k, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return FDX_OK;
    FDX_ABI_CATCH(c)
}

int fdx_get_stats(fdx_ctx *c, fdx_stats *out) {
    FDX_ABI_TRY
    if (!c || !out) return FDX_EINVAL;
    *out = c->stats;
    return FDX_OK;
    FDX_ABI_CATCH(c)
}

int fdx_get_tree(fdx_ctx *c, double *cube, uint64_t *key, uint32_t *perm, int32_t *level,
                 uint64_t *prefix, uint32_t *begin, uint32_t *count, uint32_t *first_child,
                 uint32_t *nchild, uint32_t *parent, double *mom) {
    FDX_ABI_TRY
    if (!c) return FDX_EINVAL;
    if (!c->skey) return fail(c, FDX_ESTATE, "no tree built");
    hipStream_t s = c->stream;
    const size_t n = (size_t)c->n, nc = (size_t)c->stats.n_cells;
    auto cp = [&](void *dst, const void *src, size_t bytes) -> hipError_t {
        if (!dst || !bytes) return hipSuccess;
        return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s);
    };
    HIPCHK(c, cp(cube, c->cube.p, 4 * sizeof(double) * c->nsys));
    HIPCHK(c, cp(key, c->skey, 8 * n));
    HIPCHK(c, cp(perm, c->sperm, 4 * n));
    HIPCHK(c, cp(level, c->c_level.p, 4 * nc));
    HIPCHK(c, cp(prefix, c->c_prefix.p, 8 * nc));
    HIPCHK(c, cp(begin, c->c_begin.p, 4 * nc));
    HIPCHK(c, cp(count, c->c_count.p, 4 * nc));
    HIPCHK(c, cp(first_child, c->c_first.p, 4 * nc));
    HIPCHK(c, cp(nchild, c->c_nchild.p, 4 * nc));
    HIPCHK(c, cp(parent, c->c_parent.p, 4 * nc));
    HIPCHK(c, cp(mom, c->c_mom.p, 80 * nc));
    HIPCHK(c, hipStreamSynchronize(s));
    return FDX_OK;
    FDX_ABI_CATCH(c)
}

int fdx_get_groups(fdx_ctx *c, uint32_t *cell, uint32_t *begin, uint32_t *count, uint32_t *qmin,
                   uint32_t *qmax, double *centre) {
    FDX_ABI_TRY
    if (!c) return FDX_EINVAL;
    if (!c->skey) return fail(c, FDX_ESTATE, "no tree built");
    hipStream_t s = c->stream;
    const size_t G = (size_t)c->stats.n_groups;
    auto cp = [&](void *dst, const void *src, size_t bytes) -> hipError_t {
        if (!dst || !bytes) return hipSuccess;
        return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s);
    };
    HIPCHK(c, cp(cell, c->g_cell.p, 4 * G));
    HIPCHK(c, cp(begin, c->g_begin.p, 4 * G));
    HIPCHK(c, cp(count, c->g_count.p, 4 * G));
    HIPCHK(c, cp(centre, c->g_centre.p, 24 * G));
    std::vector<uint32_t> box(6 * G);
    HIPCHK(c, cp(box.data(), c->g_box.p, 24 * G));
    HIPCHK(c, hipStreamSynchronize(s));
    for (size_t g = 0; g < G; g++)
        for (int a = 0; a < 3; a++) {
            if (qmin) qmin[3 * g + a] = box[6 * g + a];
            if (qmax) qmax[3 * g + a] = box[6 * g + 3 + a];
        }
    return FDX_OK;
    FDX_ABI_CATCH(c)
}

int fdx_get_lists(fdx_ctx *c, uint32_t *n_epj, uint32_t *n_spj, uint32_t *epj, uint32_t *spj) {
    FDX_ABI_TRY
    if (!c) return FDX_EINVAL;
    if (!c->have_counts) return fail(c, FDX_ESTATE, "no walk done on the current groups");
    if ((epj || spj) && !c->have_lists)
        return fail(c, FDX_ESTATE, "the last evaluation (FDX_FUSED) stored no lists: call "
                                   "fdx_set_list_capture(ctx, 1) before it");
    hipStream_t s = c->stream;
    const size_t G = (size_t)c->stats.n_groups;
    std::vector<uint32_t> ce(G), cs(G);
    HIPCHK(c, hipMemcpyAsync(ce.data(), c->cnt_e.p, 4 * G, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipMemcpyAsync(cs.data(), c->cnt_s.p, 4 * G, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    // entries compacted on the device (segments may be far longer than their lists)
    std::vector<uint64_t> oe(G + 1, 0), os(G + 1, 0);
    for (size_t g = 0; g < G; g++) {
        oe[g + 1] = oe[g] + ce[g];
        os[g + 1] = os[g] + cs[g];
        if (n_epj) n_epj[g] = ce[g];
        if (n_spj) n_spj[g] = cs[g];
    }
    if ((epj || spj) && G && (oe[G] || os[G])) {
        DBuf<uint64_t> doe, dos;
        DBuf<uint32_t> de, ds;
        auto run = [&]() -> hipError_t {
            hipError_t e = doe.ensure(G + 1);
            if (e == hipSuccess) e = dos.ensure(G + 1);
            if (e == hipSuccess) e = de.ensure(std::max<uint64_t>(oe[G], 1));
            if (e == hipSuccess) e = ds.ensure(std::max<uint64_t>(os[G], 1));
            if (e == hipSuccess) e = hipMemcpyAsync(doe.p, oe.data(), 8 * (G + 1),
                                                    hipMemcpyHostToDevice, s);
            if (e == hipSuccess) e = hipMemcpyAsync(dos.p, os.data(), 8 * (G + 1),
                                                    hipMemcpyHostToDevice, s);
            if (e == hipSuccess) e = compact_lists(G, c->seg.p, c->lcap.p, c->cnt_e.p, c->cnt_s.p,
                                                   doe.p, dos.p, c->list.p, de.p, ds.p, s);
            if (e == hipSuccess && epj && oe[G])
                e = hipMemcpyAsync(epj, de.p, 4 * oe[G], hipMemcpyDeviceToHost, s);
            if (e == hipSuccess && spj && os[G])
                e = hipMemcpyAsync(spj, ds.p, 4 * os[G], hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            return e;
        };
        const hipError_t e = run();
        doe.release(); dos.release(); de.release(); ds.release();
        if (e != hipSuccess) return fail(c, FDX_EHIP, "get_lists: %s", hipGetErrorString(e));
    }
    return FDX_OK;
    FDX_ABI_CATCH(c)
}

int fdx_set_list_capture(fdx_ctx *c, int32_t on) {
    FDX_ABI_TRY
    if (!c) return FDX_EINVAL;
    c->capture_lists = on != 0;
    return FDX_OK;
    FDX_ABI_CATCH(c)
}

const char *fdx_last_error(const fdx_ctx *c) {
    if (!c) return "null context";
    return c->err;
}

}  // extern "C"
