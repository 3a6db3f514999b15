// SPH density on the tree (short-range interaction with four kinds of cutoff, section
// "Interaction calculation"; Wendland C6 kernel of the paper's SPH application): tree and
// groups as for gravity, candidate lists by the short-range walk (count pass, offsets, one
// read of the total, fill pass), then the density kernel and the return to the caller's order.
#include <cmath>

#include "ctx.h"

namespace fdx {

namespace {

struct SphState {
    DBuf<double> h, sh, hmax, rg, rho_s, rho;
    DBuf<uint32_t> n_s, nngb;
    bool built = false;
    uint64_t gen = 0;
    void release() {
        for (auto *b : {&h, &sh, &hmax, &rg, &rho_s, &rho}) b->release();
        n_s.release();
        nngb.release();
        built = false;
    }
};

SphState *state(fdx_ctx *c) {
    if (!c->ext.sph) c->ext.sph = new SphState();
    return static_cast<SphState *>(c->ext.sph);
}

}  // namespace

void sph_release(fdx_ctx *c) {
    SphState *x = static_cast<SphState *>(c->ext.sph);
    if (!x) return;
    x->release();
    delete x;
    c->ext.sph = nullptr;
}

}  // namespace fdx

using namespace fdx;

extern "C" {

int fdx_calc_density(fdx_ctx *c, int32_t mode, double r_cut, const double *h, int32_t mem_kind,
                     int32_t n_leaf, int32_t n_group, int32_t flags) {
    FDX_ABI_TRY
    if (!c) return FDX_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, FDX_EHIP, "hipSetDevice failed");
    if (!c->have_particles) return fail(c, FDX_ESTATE, "no particles: call fdx_set_particles first");
    if (mode < FDX_CUT_FIXED || mode > FDX_CUT_SYMMETRIC) return fail(c, FDX_EINVAL, "bad cutoff mode");
    if (mode == FDX_CUT_FIXED && !(std::isfinite(r_cut) && r_cut > 0.0))
        return fail(c, FDX_EINVAL, "r_cut must be finite and > 0");
    if (mode != FDX_CUT_FIXED && !h) return fail(c, FDX_EINVAL, "this cutoff mode needs h");
    if (mem_kind != FDX_MEM_HOST && mem_kind != FDX_MEM_DEVICE)
        return fail(c, FDX_EINVAL, "bad mem_kind");
    const double eps = c->eps_given ? 0.0 : (c->eps_all > 0 ? c->eps_all : 1.0);
    int r = setup_eval(c, 0.5, n_leaf, n_group, eps, flags & FDX_TIMING);
    if (r) return r;
    SphState *x = state(c);
    x->built = false;
    hipStream_t s = c->stream;
    const size_t n = (size_t)c->n;
    const double *hsrc = nullptr;
    if (mode != FDX_CUT_FIXED) {
        HIPCHK(c, x->h.ensure(n));
        if (n)
            HIPCHK(c, hipMemcpyAsync(x->h.p, h, n * sizeof(double),
                                     mem_kind == FDX_MEM_HOST ? hipMemcpyHostToDevice
                                                              : hipMemcpyDeviceToDevice, s));
        hsrc = x->h.p;
    }
    r = run_tree(c, true);
    if (r) return r;
    const uint32_t G = c->hst->st.n_groups;
    HIPCHK(c, x->sh.ensure(n));
    HIPCHK(c, x->rho_s.ensure(n));
    HIPCHK(c, x->n_s.ensure(n));
    HIPCHK(c, x->rho.ensure(n));
    HIPCHK(c, x->nngb.ensure(n));
    HIPCHK(c, sph_radius(n, c->sperm, hsrc, r_cut, x->sh.p, c->st, s));
    ShortArgs sa;
    sa.cube = c->cube.p;
    sa.r_fixed = r_cut;
    const Cells cv = cells_view(c);
    const Groups gv = groups_view(c);
    if (mode == FDX_CUT_SCATTER || mode == FDX_CUT_SYMMETRIC) {
        HIPCHK(c, x->hmax.ensure(c->cell_cap));
        HIPCHK(c, sph_cell_hmax(cv, x->sh.p, x->hmax.p, s));
        sa.hmax = x->hmax.p;
    }
    if (mode == FDX_CUT_GATHER || mode == FDX_CUT_SYMMETRIC) {
        HIPCHK(c, x->rg.ensure(std::max<uint32_t>(G, 1)));
        HIPCHK(c, sph_group_hmax(G, gv, x->sh.p, x->rg.p, c->st, s));
        sa.rg = x->rg.p;
    }
    const int kind = mode == FDX_CUT_SCATTER ? 2 : (mode == FDX_CUT_SYMMETRIC ? 3 : 1);
    // count pass, segment sizes and offsets (total in st->list_total), one read, fill pass
    HIPCHK(c, walk_short(false, kind, G, gv, cv, sa, 0.0, nullptr, nullptr, 0, nullptr, c->cnt_e.p,
                         c->cnt_s.p, nullptr, c->st, s));
    HIPCHK(c, list_caps(G, c->cnt_e.p, c->cnt_s.p, c->lcap.p, c->st, s));
    HIPCHK(c, scan_u32_to_u64(c->lcap.p, c->seg.p, 0, nullptr, &c->st->n_groups_c, c->partial.p,
                              &c->st->list_total, s));
    r = read_status(c);
    if (r) return r;
    const DevStatus &hs = c->hst->st;
    if (hs.bad_input) return fail(c, FDX_EINVAL, "h has a non-positive or non-finite value");
    if (hs.walk_error) return fail(c, FDX_EHIP, "walk stack exhausted");
    r = ensure_list_capacity(c, hs.list_total);
    if (r) return r;
    HIPCHK(c, walk_short(true, kind, G, gv, cv, sa, 0.0, c->seg.p, c->lcap.p, c->list_cap, c->list.p,
                         c->cnt_e.p, c->cnt_s.p, nullptr, c->st, s));
    c->have_lists = true;
    c->have_counts = true;
    c->stats.list_capacity = (int64_t)hs.list_total;
    c->stats.overflow_groups = 0;
    HIPCHK(c, list_stats(G, gv, c->cnt_e.p, c->cnt_s.p, c->st, s));
    mark(c, 6);
    HIPCHK(c, sph_density(mode, G, gv, c->seg.p, c->cnt_e.p, c->list.p, c->jp.p, x->sh.p,
                          x->rho_s.p, x->n_s.p, c->st, s));
    mark(c, 7);
    HIPCHK(c, sph_unsort(n, c->inv.p, x->rho_s.p, x->n_s.p, x->rho.p, x->nngb.p, s));
    mark(c, 8);
    finish_stats(c);
    if (flags & FDX_TIMING) {
        r = sync_timing(c);
        if (r) return r;
    }
    r = read_counters(c);
    if (r) return r;
    x->gen = c->gen;
    x->built = true;
    return FDX_OK;
    FDX_ABI_CATCH(c)
}

int fdx_get_density(fdx_ctx *c, double *rho, uint32_t *n_ngb, int32_t mem_kind) {
    FDX_ABI_TRY
    if (!c) return FDX_EINVAL;
    SphState *x = static_cast<SphState *>(c->ext.sph);
    if (!x || !x->built || x->gen != c->gen)
        return fail(c, FDX_ESTATE, "no density computed for the current particles");
    hipMemcpyKind k = mem_kind == FDX_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    const size_t n = (size_t)c->n;
    if (rho && n) HIPCHK(c, hipMemcpyAsync(rho, x->rho.p, n * sizeof(double), k, c->stream));
    if (n_ngb && n) HIPCHK(c, hipMemcpyAsync(n_ngb, x->nngb.p, n * sizeof(uint32_t), k, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return FDX_OK;
    FDX_ABI_CATCH(c)
}

}  // extern "C"
