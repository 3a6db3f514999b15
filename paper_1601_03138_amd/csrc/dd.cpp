// Domain decomposition (section "Domain decomposition"): multisection with cost-weighted
// sampling, and the exchange of particles that follows it.  The current domains are the
// systems of the particle set (virtual processes on one GPU).  The host computes the sample
// counts from the costs; the samples, the three divisions, the destinations, the grouping by
// destination and the reorder of the particle arrays run on the device.
#include <algorithm>
#include <cmath>
#include <utility>
#include <vector>

#include "ctx.h"

namespace fdx {

namespace {

constexpr uint64_t kMaxPairs = 1ull << 24;     // (source, destination) pairs tracked

struct DdState {
    DBuf<int64_t> kofs;
    DBuf<uint64_t> cost;
    DBuf<uint32_t> idx, cell, val, val_alt, start_a, start_b, scratch;
    DBuf<double> sx, sy, sz, faces;
    DBuf<uint64_t> key, key_alt;                   // samples
    DBuf<uint64_t> pkey, pkey_alt;                 // particles
    DBuf<uint32_t> pval, pval_alt, dest, run_lo, run_hi;
    DBuf<double> moved[8];                         // reordered particle arrays (exchange)
    uint32_t *order = nullptr;                     // pval or pval_alt after the sort
    std::vector<int64_t> k;                        // samples per current domain
    std::vector<int64_t> kofs_h;                   // host staging of the sample offsets
    uint32_t start0_h[2] = {0, 0};
    std::vector<int64_t> counts, dom_off;          // send counts [p][d], new offsets
    int nx = 0, ny = 0, nz = 0, nsrc = 0;
    uint64_t D = 0, K = 0;
    int64_t n = 0;
    bool built = false, counts_ready = false, applied = false;
    uint64_t gen = 0;
    hipEvent_t ev[6] = {};

    void release() {
        kofs.release();
        cost.release();
        for (auto *b : {&idx, &cell, &val, &val_alt, &start_a, &start_b, &scratch, &pval,
                        &pval_alt, &dest, &run_lo, &run_hi})
            b->release();
        for (auto *b : {&sx, &sy, &sz, &faces}) b->release();
        for (auto *b : {&key, &key_alt, &pkey, &pkey_alt}) b->release();
        for (auto &b : moved) b.release();
        for (auto &e : ev)
            if (e) { (void)hipEventDestroy(e); e = nullptr; }
        built = false;
    }
};

DdState *state(fdx_ctx *c) {
    if (!c->ext.dd) c->ext.dd = new DdState();
    return static_cast<DdState *>(c->ext.dd);
}

int check_built(fdx_ctx *c) {
    DdState *d = static_cast<DdState *>(c->ext.dd);
    if (!d || !d->built || d->gen != c->gen)
        return fail(c, FDX_ESTATE, "no domain decomposition of the current particles");
    return FDX_OK;
}

int bits_for(uint64_t v) {          // significant bits of v (0 for v = 0)
    int b = 0;
    while (v) { b++; v >>= 1; }
    return b;
}

// send counts and new offsets from the (destination, source) runs of the sorted keys
int ensure_counts(fdx_ctx *c, DdState *d) {
    if (d->counts_ready) return FDX_OK;
    const size_t P = (size_t)d->D * d->nsrc;
    std::vector<uint32_t> lo(P), hi(P);
    HIPCHK(c, hipMemcpyAsync(lo.data(), d->run_lo.p, 4 * P, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(hi.data(), d->run_hi.p, 4 * P, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    d->counts.assign((size_t)d->nsrc * d->D, 0);
    d->dom_off.assign(d->D + 1, 0);
    for (uint64_t dd = 0; dd < d->D; dd++) {
        int64_t col = 0;
        for (int p = 0; p < d->nsrc; p++) {
            const size_t k = (size_t)dd * d->nsrc + p;
            const int64_t v = (int64_t)hi[k] - (int64_t)lo[k];
            d->counts[(size_t)p * d->D + dd] = v;
            col += v;
        }
        d->dom_off[dd + 1] = d->dom_off[dd] + col;
    }
    if (d->dom_off[d->D] != d->n)
        return fail(c, FDX_EHIP, "send counts do not add up to the particle count");
    d->counts_ready = true;
    return FDX_OK;
}

}  // namespace

void dd_release(fdx_ctx *c) {
    DdState *d = static_cast<DdState *>(c->ext.dd);
    if (!d) return;
    d->release();
    delete d;
    c->ext.dd = nullptr;
}

}  // namespace fdx

using namespace fdx;

extern "C" {

int fdx_dd_factor(int32_t n, int32_t *nx, int32_t *ny, int32_t *nz) {
    FDX_ABI_TRY
    if (n < 1 || !nx || !ny || !nz) return FDX_EINVAL;
    int32_t ba = n, bb = 1, bc = 1;            // n x 1 x 1 always exists
    for (int32_t c = 1; (int64_t)c * c * c <= n; c++) {
        if (n % c) continue;
        const int32_t rest = n / c;
        for (int32_t b = c; (int64_t)b * b <= rest; b++) {
            if (rest % b) continue;
            const int32_t a = rest / b;        // a >= b >= c
            if (a - c < ba - bc || (a - c == ba - bc && a - b < ba - bb)) {
                ba = a; bb = b; bc = c;
            }
        }
    }
    *nx = ba; *ny = bb; *nz = bc;
    return FDX_OK;
    FDX_ABI_CATCH(nullptr)
}

int fdx_decompose(fdx_ctx *c, int32_t nx, int32_t ny, int32_t nz, int64_t n_sample,
                  const double *cost, uint64_t seed, int32_t flags) {
    FDX_ABI_TRY
    if (!c) return FDX_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, FDX_EHIP, "hipSetDevice failed");
    if (!c->have_particles) return fail(c, FDX_ESTATE, "no particles: call fdx_set_particles first");
    if (nx < 1 || ny < 1 || nz < 1) return fail(c, FDX_EINVAL, "nx, ny, nz must be >= 1");
    if (n_sample < 1 || n_sample >= (1ll << 31))
        return fail(c, FDX_EINVAL, "n_sample must be in [1, 2^31)");
    if (flags & ~FDX_DD_COST_LISTS) return fail(c, FDX_EINVAL, "unknown flags");
    const bool from_lists = (flags & FDX_DD_COST_LISTS) != 0;
    if (cost && from_lists) return fail(c, FDX_EINVAL, "cost given together with FDX_DD_COST_LISTS");
    const uint64_t D = (uint64_t)nx * (uint64_t)ny * (uint64_t)nz;
    const int nsrc = c->nsys;
    if (D * (uint64_t)nsrc > kMaxPairs)
        return fail(c, FDX_EINVAL, "more than 2^24 (source, destination) pairs");
    if (from_lists && !c->have_lists)
        return fail(c, FDX_ESTATE, "FDX_DD_COST_LISTS needs a walk on the current particles");
    if (cost)
        for (int p = 0; p < nsrc; p++)
            if (!(std::isfinite(cost[p]) && cost[p] >= 0.0))
                return fail(c, FDX_EINVAL, "cost must be finite and >= 0");
    DdState *d = state(c);
    d->built = false;
    hipStream_t s = c->stream;
    HIPCHK(c, hipStreamSynchronize(s));        // the host staging below may still be read
    for (auto &e : d->ev)
        if (!e) HIPCHK(c, hipEventCreate(&e));
    HIPCHK(c, hipEventRecord(d->ev[0], s));

    // costs and sample counts (host)
    std::vector<double> T(nsrc);
    if (cost) {
        for (int p = 0; p < nsrc; p++) T[p] = cost[p];
    } else if (from_lists) {
        HIPCHK(c, d->cost.ensure(nsrc));
        HIPCHK(c, hipMemsetAsync(d->cost.p, 0, 8 * (size_t)nsrc, s));
        const uint32_t G = (uint32_t)std::min<uint64_t>((uint64_t)c->stats.n_groups, c->g_sys.cap);
        HIPCHK(c, dd_cost(G, c->g_sys.p, c->g_count.p, c->cnt_e.p,
                          c->cnt_s.p, d->cost.p, s));
        std::vector<uint64_t> h(nsrc);
        HIPCHK(c, hipMemcpyAsync(h.data(), d->cost.p, 8 * (size_t)nsrc, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        for (int p = 0; p < nsrc; p++) T[p] = (double)h[p];
    } else {
        for (int p = 0; p < nsrc; p++) T[p] = (double)(c->sys_off_h[p + 1] - c->sys_off_h[p]);
    }
    double total = 0.0;
    for (int p = 0; p < nsrc; p++) total += T[p];
    if (!(total > 0.0)) return fail(c, FDX_EINVAL, "the total cost must be > 0");
    d->k.assign(nsrc, 0);
    std::vector<int64_t> &kofs = d->kofs_h;
    kofs.assign(nsrc + 1, 0);
    for (int p = 0; p < nsrc; p++) {
        const int64_t np = c->sys_off_h[p + 1] - c->sys_off_h[p];
        d->k[p] = np == 0 ? 0 : (int64_t)std::floor((double)n_sample * T[p] / total);
        kofs[p + 1] = kofs[p] + d->k[p];
    }
    const uint64_t K = (uint64_t)kofs[nsrc];
    if (K < D)
        return fail(c, FDX_EINVAL, "%llu samples for %llu domains: every domain needs one",
                    (unsigned long long)K, (unsigned long long)D);
    const size_t N = (size_t)c->n;

    // buffers
    HIPCHK(c, d->kofs.ensure(nsrc + 1));
    for (auto *b : {&d->idx, &d->cell, &d->val, &d->val_alt}) HIPCHK(c, b->ensure(K));
    for (auto *b : {&d->sx, &d->sy, &d->sz}) HIPCHK(c, b->ensure(K));
    HIPCHK(c, d->key.ensure(K));
    HIPCHK(c, d->key_alt.ensure(K));
    HIPCHK(c, d->scratch.ensure(radix_scratch_u32(K)));
    HIPCHK(c, d->start_a.ensure(D + 1));
    HIPCHK(c, d->start_b.ensure(D + 1));
    const size_t nfx = nx + 1, nfy = (size_t)nx * (ny + 1), nfz = (size_t)nx * ny * (nz + 1);
    HIPCHK(c, d->faces.ensure(nfx + nfy + nfz));
    for (auto *b : {&d->pval, &d->pval_alt, &d->dest}) HIPCHK(c, b->ensure(N));
    HIPCHK(c, d->pkey.ensure(N));
    HIPCHK(c, d->pkey_alt.ensure(N));
    HIPCHK(c, d->run_lo.ensure(D * nsrc));
    HIPCHK(c, d->run_hi.ensure(D * nsrc));
    HIPCHK(c, hipMemcpyAsync(d->kofs.p, kofs.data(), 8 * (size_t)(nsrc + 1),
                             hipMemcpyHostToDevice, s));
    d->start0_h[0] = 0;
    d->start0_h[1] = (uint32_t)K;
    HIPCHK(c, hipMemcpyAsync(d->start_a.p, d->start0_h, sizeof(d->start0_h), hipMemcpyHostToDevice,
                             s));

    // samples
    HIPCHK(c, dd_sample((uint32_t)K, (uint32_t)nsrc, d->kofs.p, c->sys_off.p, seed, c->x, c->y,
                        c->z, d->idx.p, d->sx.p, d->sy.p, d->sz.p, d->key.p, d->val.p, s));
    HIPCHK(c, hipEventRecord(d->ev[1], s));

    // three divisions: x over all samples, y within slabs, z within columns
    double *bx = d->faces.p, *by = bx + nfx, *bz = by + nfy;
    uint64_t *kin = d->key.p, *kother = d->key_alt.p;
    uint32_t *vin = d->val.p, *vother = d->val_alt.p;
    uint32_t *start_in = d->start_a.p, *start_out = d->start_b.p;
    struct Level { uint32_t nseg, n; const double *coord, *next; double *face; };
    const Level levels[3] = {{1u, (uint32_t)nx, d->sx.p, d->sy.p, bx},
                             {(uint32_t)nx, (uint32_t)ny, d->sy.p, d->sz.p, by},
                             {(uint32_t)(nx * ny), (uint32_t)nz, d->sz.p, nullptr, bz}};
    for (const Level &L : levels) {
        bool alt = false;
        HIPCHK(c, radix_sort(K, kin, kother, vin, vother, L.nseg > 1 ? d->cell.p : nullptr,
                             (int)L.nseg, 64, d->scratch.p, c->partial.p, &alt, s));
        if (alt) { std::swap(kin, kother); std::swap(vin, vother); }
        // sorted samples in (kin, vin); the next level's input goes to (kother, vother)
        HIPCHK(c, dd_cut((uint32_t)K, L.nseg, start_in, L.n, vin, L.coord, L.next, d->cell.p,
                         start_out, L.face, kother, vother, s));
        std::swap(kin, kother);
        std::swap(vin, vother);
        std::swap(start_in, start_out);
    }
    HIPCHK(c, hipEventRecord(d->ev[2], s));

    // destinations, stable grouping by destination, send-count runs
    HIPCHK(c, dd_assign((uint32_t)N, c->x, c->y, c->z, nx, ny, nz, bx, by, bz, d->dest.p,
                        d->pkey.p, d->pval.p, s));
    bool palt = false;
    HIPCHK(c, radix_sort(N, d->pkey.p, d->pkey_alt.p, d->pval.p, d->pval_alt.p, nullptr, 1,
                         bits_for(D - 1), c->rs_scratch.p, c->partial.p, &palt, s));
    d->order = palt ? d->pval_alt.p : d->pval.p;
    const uint64_t *psorted = palt ? d->pkey_alt.p : d->pkey.p;
    HIPCHK(c, hipMemsetAsync(d->run_lo.p, 0, 4 * D * nsrc, s));
    HIPCHK(c, hipMemsetAsync(d->run_hi.p, 0, 4 * D * nsrc, s));
    HIPCHK(c, dd_runs((uint32_t)N, psorted, d->order, c->sysid.p, (uint32_t)nsrc, d->run_lo.p,
                      d->run_hi.p, s));
    HIPCHK(c, hipEventRecord(d->ev[3], s));

    d->nx = nx; d->ny = ny; d->nz = nz; d->nsrc = nsrc;
    d->D = D; d->K = K; d->n = c->n;
    d->counts_ready = false;
    d->applied = false;
    d->built = true;
    d->gen = c->gen;
    return FDX_OK;
    FDX_ABI_CATCH(c)
}

int fdx_get_decomposition(fdx_ctx *c, double *bx, double *by, double *bz, int64_t *send_counts,
                          int64_t *dom_off) {
    FDX_ABI_TRY
    if (!c) return FDX_EINVAL;
    int r = check_built(c);
    if (r) return r;
    DdState *d = state(c);
    const size_t nfx = d->nx + 1, nfy = (size_t)d->nx * (d->ny + 1),
                 nfz = (size_t)d->nx * d->ny * (d->nz + 1);
    std::vector<double> f(nfx + nfy + nfz);
    HIPCHK(c, hipMemcpyAsync(f.data(), d->faces.p, 8 * f.size(), hipMemcpyDeviceToHost, c->stream));
    r = ensure_counts(c, d);          // synchronises the stream
    if (r) return r;
    if (bx) std::copy(f.begin(), f.begin() + nfx, bx);
    if (by) std::copy(f.begin() + nfx, f.begin() + nfx + nfy, by);
    if (bz) std::copy(f.begin() + nfx + nfy, f.end(), bz);
    if (send_counts) std::copy(d->counts.begin(), d->counts.end(), send_counts);
    if (dom_off) std::copy(d->dom_off.begin(), d->dom_off.end(), dom_off);
    return FDX_OK;
    FDX_ABI_CATCH(c)
}

int fdx_get_dd_samples(fdx_ctx *c, int64_t *k_per_domain, uint32_t *sample_idx,
                       uint32_t *sample_domain) {
    FDX_ABI_TRY
    if (!c) return FDX_EINVAL;
    int r = check_built(c);
    if (r) return r;
    DdState *d = state(c);
    if (k_per_domain) std::copy(d->k.begin(), d->k.end(), k_per_domain);
    if (sample_idx)
        HIPCHK(c, hipMemcpyAsync(sample_idx, d->idx.p, 4 * d->K, hipMemcpyDeviceToHost, c->stream));
    if (sample_domain)
        HIPCHK(c, hipMemcpyAsync(sample_domain, d->cell.p, 4 * d->K, hipMemcpyDeviceToHost,
                                 c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return FDX_OK;
    FDX_ABI_CATCH(c)
}

int fdx_get_dd_destinations(fdx_ctx *c, uint32_t *dest, uint32_t *order, int32_t mem_kind) {
    FDX_ABI_TRY
    if (!c) return FDX_EINVAL;
    if (mem_kind != FDX_MEM_HOST && mem_kind != FDX_MEM_DEVICE)
        return fail(c, FDX_EINVAL, "mem_kind must be FDX_MEM_HOST or FDX_MEM_DEVICE");
    int r = check_built(c);
    if (r) return r;
    DdState *d = state(c);
    const hipMemcpyKind k = mem_kind == FDX_MEM_HOST ? hipMemcpyDeviceToHost
                                                     : hipMemcpyDeviceToDevice;
    const size_t N = (size_t)d->n;
    if (dest && N) HIPCHK(c, hipMemcpyAsync(dest, d->dest.p, 4 * N, k, c->stream));
    if (order && N) HIPCHK(c, hipMemcpyAsync(order, d->order, 4 * N, k, c->stream));
    if (mem_kind == FDX_MEM_HOST) HIPCHK(c, hipStreamSynchronize(c->stream));
    return FDX_OK;
    FDX_ABI_CATCH(c)
}

int fdx_exchange_particles(fdx_ctx *c) {
    FDX_ABI_TRY
    if (!c) return FDX_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, FDX_EHIP, "hipSetDevice failed");
    int r = check_built(c);
    if (r) return r;
    DdState *d = state(c);
    if (d->applied) return fail(c, FDX_ESTATE, "the decomposition was already applied");
    r = ensure_counts(c, d);
    if (r) return r;
    hipStream_t s = c->stream;
    const size_t N = (size_t)c->n;
    double *src[8] = {c->x, c->y, c->z, c->vx, c->vy, c->vz, c->m, c->eps};
    DBuf<double> *own[8] = {&c->ox, &c->oy, &c->oz, &c->ovx, &c->ovy, &c->ovz, &c->om, &c->oeps};
    const int narr = c->eps_given ? 8 : 7;
    DdArrays a{}, b{};
    for (int k = 0; k < narr; k++) {
        HIPCHK(c, d->moved[k].ensure(N));
        a.p[k] = src[k];
        b.p[k] = d->moved[k].p;
    }
    HIPCHK(c, hipEventRecord(d->ev[4], s));
    HIPCHK(c, dd_gather((uint32_t)N, d->order, narr, a, b, s));
    HIPCHK(c, hipEventRecord(d->ev[5], s));
    // the reordered arrays become the context's own; its previous own arrays are reused as
    // the next exchange's targets
    double **dst[8] = {&c->x, &c->y, &c->z, &c->vx, &c->vy, &c->vz, &c->m, &c->eps};
    for (int k = 0; k < narr; k++) {
        std::swap(own[k]->p, d->moved[k].p);
        std::swap(own[k]->cap, d->moved[k].cap);
        *dst[k] = own[k]->p;
    }
    if (!c->eps_given) c->eps = nullptr;
    c->borrowed = false;
    const int D = (int)d->D;
    HIPCHK(c, c->sys_off.ensure(D + 1));
    HIPCHK(c, hipMemcpyAsync(c->sys_off.p, d->dom_off.data(), 8 * (size_t)(D + 1),
                             hipMemcpyHostToDevice, s));
    HIPCHK(c, sysid_fill(c->sys_off.p, D, c->sysid.p, N, s));
    HIPCHK(c, c->bbox_u.ensure(6 * (size_t)D));
    HIPCHK(c, c->cube.ensure(4 * (size_t)D));
    if (D > 1 && D <= 65536) HIPCHK(c, c->sys_carry.ensure(2 * N));
    HIPCHK(c, hipStreamSynchronize(s));        // dom_off is a host vector
    c->nsys = D;
    c->sys_off_h = d->dom_off;
    c->have_force = false;
    c->have_lists = false;
    c->have_counts = false;
    c->gen++;
    ext_invalidate(c);
    c->stats = fdx_stats{};
    d->gen = c->gen;
    d->applied = true;
    return FDX_OK;
    FDX_ABI_CATCH(c)
}

int fdx_get_dd_stats(fdx_ctx *c, fdx_dd_stats *out) {
    FDX_ABI_TRY
    if (!c || !out) return FDX_EINVAL;
    int r = check_built(c);
    if (r) return r;
    DdState *d = state(c);
    r = ensure_counts(c, d);
    if (r) return r;
    *out = fdx_dd_stats{};
    out->nx = d->nx; out->ny = d->ny; out->nz = d->nz;
    out->n_domains = (int32_t)d->D;
    out->n_src = d->nsrc;
    out->n_samples = (int64_t)d->K;
    int64_t stay = 0;
    for (int p = 0; p < std::min<int64_t>(d->nsrc, (int64_t)d->D); p++)
        stay += d->counts[(size_t)p * d->D + p];
    out->n_moved = d->n - stay;
    float t[3] = {};
    for (int k = 0; k < 3; k++) HIPCHK(c, hipEventElapsedTime(&t[k], d->ev[k], d->ev[k + 1]));
    out->ms_sample = t[0];
    out->ms_divide = t[1];
    out->ms_assign = t[2];
    if (d->applied) {
        float te = 0;
        HIPCHK(c, hipEventSynchronize(d->ev[5]));
        HIPCHK(c, hipEventElapsedTime(&te, d->ev[4], d->ev[5]));
        out->ms_exchange = te;
    }
    return FDX_OK;
    FDX_ABI_CATCH(c)
}

}  // extern "C"
