// Exchange lists between domains (section "Exchange of particles and superparticles",
// long-range mode): the domains are the systems of the particle set, each with its own local
// tree; every ordered pair (sender, receiver) is a walk of the sender's tree against the
// receiver's particle box, split into sub-walks over the sender's top-level frontier and run
// by the group-walk kernels through their selection arguments.
#include <algorithm>
#include <vector>

#include "ctx.h"

namespace fdx {

namespace {

// largest list buffer sized by the per-sender bound (one fill walk); 16 GiB of the GPU's HBM
constexpr uint64_t kExchangeBudgetBytes = 16ull << 30;

struct ExchangeState {
    DBuf<uint32_t> box, start, sel, ne, ns, cap, list, nsel, front, fcount;
    DBuf<uint64_t> seg, total;
    uint64_t list_cap = 0;
    int nsys = 0;
    size_t pairs = 0;
    uint64_t entries = 0, n_epj = 0, n_spj = 0, capacity = 0;
    double ms_tree = 0, ms_lists = 0;
    bool built = false;
    uint64_t gen = 0;            // context generation the lists belong to
    hipEvent_t ev[3] = {};

    void release() {
        for (auto *b : {&box, &start, &sel, &ne, &ns, &cap, &list, &nsel, &front, &fcount})
            b->release();
        seg.release();
        total.release();
        for (auto &e : ev)
            if (e) { (void)hipEventDestroy(e); e = nullptr; }
        list_cap = 0;
        built = false;
    }
};

ExchangeState *state(fdx_ctx *c) {
    if (!c->ext.exch) c->ext.exch = new ExchangeState();
    return static_cast<ExchangeState *>(c->ext.exch);
}

int check_built(fdx_ctx *c) {
    ExchangeState *x = static_cast<ExchangeState *>(c->ext.exch);
    if (!x || !x->built || x->gen != c->gen)
        return fail(c, FDX_ESTATE, "no exchange lists built for the current particles");
    return FDX_OK;
}

}  // namespace

void exchange_release(fdx_ctx *c) {
    ExchangeState *x = static_cast<ExchangeState *>(c->ext.exch);
    if (!x) return;
    x->release();
    delete x;
    c->ext.exch = nullptr;
}

}  // namespace fdx

using namespace fdx;

extern "C" {

int fdx_build_exchange_lists(fdx_ctx *c, double theta, int32_t n_leaf) {
    FDX_ABI_TRY
    if (!c) return FDX_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, FDX_EHIP, "hipSetDevice failed");
    if (!c->have_particles) return fail(c, FDX_ESTATE, "no particles: call fdx_set_particles first");
    if (c->nsys < 2) return fail(c, FDX_EINVAL, "exchange lists need at least two domains");
    for (int s = 0; s < c->nsys; s++)
        if (c->sys_off_h[s + 1] == c->sys_off_h[s])
            return fail(c, FDX_EINVAL, "domain %d is empty", s);
    const size_t P = (size_t)c->nsys * (size_t)(c->nsys - 1);
    if (P > 0x7FFFFFFFull) return fail(c, FDX_EINVAL, "too many domains");
    // the local trees: keys, sort, cells, moments (and groups, unused here); softening is
    // not used by the lists
    const double eps = c->eps_given ? 0.0 : (c->eps_all > 0 ? c->eps_all : 1.0);
    int r = setup_eval(c, theta, n_leaf, kMaxGroup, eps, 0);
    if (r) return r;
    ExchangeState *x = state(c);
    x->built = false;
    hipStream_t s = c->stream;
    for (auto &e : x->ev)
        if (!e) HIPCHK(c, hipEventCreate(&e));
    HIPCHK(c, hipEventRecord(x->ev[0], s));
    r = run_tree(c, true);
    if (r) return r;
    finish_stats(c);
    HIPCHK(c, hipEventRecord(x->ev[1], s));

    const size_t G = exchange_subwalks(c->nsys);
    HIPCHK(c, x->box.ensure(6 * G));
    HIPCHK(c, x->start.ensure(G));
    HIPCHK(c, x->sel.ensure(G));
    HIPCHK(c, x->ne.ensure(G));
    HIPCHK(c, x->ns.ensure(G));
    HIPCHK(c, x->cap.ensure(G));
    HIPCHK(c, x->seg.ensure(G + 1));
    HIPCHK(c, x->total.ensure(1));
    HIPCHK(c, x->nsel.ensure(1));
    HIPCHK(c, x->front.ensure((size_t)kExchangeFrontierMax * c->nsys));
    HIPCHK(c, x->fcount.ensure(c->nsys));
    const Cells cv = cells_view(c);
    const double th2 = c->theta * c->theta;
    HIPCHK(c, exchange_split(c->nsys, cv, c->bbox_u.p, c->cube.p, th2, x->front.p, x->fcount.p,
                             x->box.p, x->start.p, x->cap.p, x->sel.p, x->nsel.p, s));
    HIPCHK(c, fill_u32(x->ne.p, 0u, G, s));
    HIPCHK(c, fill_u32(x->ns.p, 0u, G, s));
    Groups pg{};
    pg.box = x->box.p;
    pg.sys = x->start.p;
    pg.cap = (uint32_t)std::min<size_t>(G, 0xFFFFFFFFu);
    // every list of sender s holds at most n_s entries (they cover disjoint sets of its
    // particles; so does each sub-walk within its start cell): with room for that bound in
    // every segment, one fill walk does; past the budget a count walk sizes them first
    const uint64_t bound = (uint64_t)(c->nsys - 1) * (uint64_t)c->n;
    const bool one_pass = bound * sizeof(uint32_t) <= kExchangeBudgetBytes;
    if (!one_pass) {
        HIPCHK(c, walk(false, G, pg, cv, th2, nullptr, nullptr, 0, nullptr, x->ne.p, x->ns.p,
                       nullptr, x->sel.p, x->nsel.p, c->st, s));
        HIPCHK(c, exchange_caps(G, x->sel.p, x->nsel.p, x->ne.p, x->ns.p, x->cap.p, s));
    }
    HIPCHK(c, scan_u32_to_u64(x->cap.p, x->seg.p, G, nullptr, nullptr, c->partial.p, x->total.p,
                              s));
    uint64_t total = bound;
    if (!one_pass) {
        HIPCHK(c, hipMemcpyAsync(&total, x->total.p, 8, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
    }
    if (total > x->list_cap || !x->list.p) {
        HIPCHK(c, x->list.ensure(total));
        x->list_cap = total;
    }
    HIPCHK(c, walk(true, G, pg, cv, th2, x->seg.p, x->cap.p, x->list_cap, x->list.p, x->ne.p,
                   x->ns.p, nullptr, x->sel.p, x->nsel.p, c->st, s));
    HIPCHK(c, hipEventRecord(x->ev[2], s));
    r = read_status(c);
    if (r) return r;
    const DevStatus &h = c->hst->st;
    if (h.walk_error || h.list_overflow)
        return fail(c, FDX_EHIP, "exchange walk did not complete (stack %u, overflow %u)",
                    h.walk_error, h.list_overflow);
    float t0 = 0, t1 = 0;
    HIPCHK(c, hipEventElapsedTime(&t0, x->ev[0], x->ev[1]));
    HIPCHK(c, hipEventElapsedTime(&t1, x->ev[1], x->ev[2]));
    std::vector<uint32_t> ne(G), ns(G);
    HIPCHK(c, hipMemcpyAsync(ne.data(), x->ne.p, 4 * G, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipMemcpyAsync(ns.data(), x->ns.p, 4 * G, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    x->n_epj = x->n_spj = 0;
    for (size_t g = 0; g < G; g++) { x->n_epj += ne[g]; x->n_spj += ns[g]; }
    x->entries = x->n_epj + x->n_spj;
    x->capacity = total;
    x->nsys = c->nsys;
    x->pairs = P;
    x->ms_tree = t0;
    x->ms_lists = t1;
    x->gen = c->gen;
    x->built = true;
    return FDX_OK;
    FDX_ABI_CATCH(c)
}

int fdx_get_exchange_counts(fdx_ctx *c, uint32_t *n_epj, uint32_t *n_spj) {
    FDX_ABI_TRY
    if (!c) return FDX_EINVAL;
    int r = check_built(c);
    if (r) return r;
    ExchangeState *x = static_cast<ExchangeState *>(c->ext.exch);
    const size_t S = (size_t)x->nsys, G = exchange_subwalks(x->nsys);
    std::vector<uint32_t> ne(G), ns(G);
    HIPCHK(c, hipMemcpyAsync(ne.data(), x->ne.p, 4 * G, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(ns.data(), x->ns.p, 4 * G, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (size_t s = 0; s < S; s++)
        for (size_t q = 0; q < S; q++) {
            uint32_t e = 0, sp = 0;
            if (q != s) {
                const size_t k = s * (S - 1) + (q < s ? q : q - 1);
                for (size_t g = k * kExchangeFrontierMax; g < (k + 1) * kExchangeFrontierMax; g++) {
                    e += ne[g];
                    sp += ns[g];
                }
            }
            if (n_epj) n_epj[s * S + q] = e;
            if (n_spj) n_spj[s * S + q] = sp;
        }
    return FDX_OK;
    FDX_ABI_CATCH(c)
}

int fdx_get_exchange_lists(fdx_ctx *c, uint32_t *epj, uint32_t *spj) {
    FDX_ABI_TRY
    if (!c) return FDX_EINVAL;
    int r = check_built(c);
    if (r) return r;
    ExchangeState *x = static_cast<ExchangeState *>(c->ext.exch);
    const size_t P = exchange_subwalks(x->nsys), n = (size_t)c->n;   // sub-walks, pair-major
    std::vector<uint32_t> ne(P), ns(P), cap(P), perm(n);
    std::vector<uint64_t> seg(P);
    hipStream_t s = c->stream;
    HIPCHK(c, hipMemcpyAsync(ne.data(), x->ne.p, 4 * P, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipMemcpyAsync(ns.data(), x->ns.p, 4 * P, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipMemcpyAsync(cap.data(), x->cap.p, 4 * P, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipMemcpyAsync(seg.data(), x->seg.p, 8 * P, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipMemcpyAsync(perm.data(), c->sperm, 4 * n, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    // each sub-walk's segment: particles from its front, cells from its back; a pair's
    // entries are its sub-walks' in slot order
    std::vector<uint32_t> e(std::max<uint64_t>(x->n_epj, 1)), sp(std::max<uint64_t>(x->n_spj, 1));
    size_t oe = 0, os = 0;
    for (size_t k = 0; k < P; k++) {
        if (epj && ne[k])
            HIPCHK(c, hipMemcpyAsync(e.data() + oe, x->list.p + seg[k], 4 * (size_t)ne[k],
                                     hipMemcpyDeviceToHost, s));
        if (spj && ns[k])
            HIPCHK(c, hipMemcpyAsync(sp.data() + os, x->list.p + seg[k] + cap[k] - ns[k],
                                     4 * (size_t)ns[k], hipMemcpyDeviceToHost, s));
        oe += ne[k];
        os += ns[k];
    }
    HIPCHK(c, hipStreamSynchronize(s));
    if (epj)
        for (size_t i = 0; i < oe; i++) epj[i] = perm[e[i]];
    if (spj)
        for (size_t i = 0; i < os; i++) spj[i] = sp[i];
    return FDX_OK;
    FDX_ABI_CATCH(c)
}

int fdx_get_exchange_stats(fdx_ctx *c, fdx_exchange_stats *out) {
    FDX_ABI_TRY
    if (!c || !out) return FDX_EINVAL;
    int r = check_built(c);
    if (r) return r;
    ExchangeState *x = static_cast<ExchangeState *>(c->ext.exch);
    out->n_domains = x->nsys;
    out->n_pairs = (int64_t)x->pairs;
    out->n_epj = (int64_t)x->n_epj;
    out->n_spj = (int64_t)x->n_spj;
    out->list_capacity = (int64_t)x->capacity;
    out->ms_tree = x->ms_tree;
    out->ms_lists = x->ms_lists;
    return FDX_OK;
    FDX_ABI_CATCH(c)
}

}  // extern "C"
