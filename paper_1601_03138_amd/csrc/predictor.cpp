// Host side of the learned list-length predictor: weights and normalisation, the training
// driver (own forward/backward/Adam kernels), and the predicted single-pass walk with exact
// re-walk of the groups whose list outgrew its predicted capacity.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <random>
#include <vector>

#include "ctx.h"
#include "mlp.h"
#include "predictor.h"

namespace fdx {

namespace {

struct Pred {
    DBuf<float> P, m, v, grad, gpart, lpart, loss, X, y, mu, sd, mu0, sd1;
    DBuf<float> tX, tT;
    DBuf<uint32_t> idx, ocap, nsel;
    DBuf<uint64_t> ooff, base_total;
    float mu_h[kMlpIn] = {}, sd_h[kMlpIn] = {};
    float margin = 0.0f;
    bool loaded = false;
    int step = 0;
};

Pred *pred_of(fdx_ctx *c) {
    Pred *p = static_cast<Pred *>(c->ext.pred);
    if (!p) {
        p = new Pred();
        c->ext.pred = p;
    }
    return p;
}

int upload_norm(fdx_ctx *c, Pred *p) {
    HIPCHK(c, p->mu.ensure(kMlpIn));
    HIPCHK(c, p->sd.ensure(kMlpIn));
    HIPCHK(c, hipMemcpyAsync(p->mu.p, p->mu_h, sizeof p->mu_h, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(p->sd.p, p->sd_h, sizeof p->sd_h, hipMemcpyHostToDevice, c->stream));
    return FDX_OK;
}

// Grow the list buffer keeping its first `keep` entries.
int grow_list_keep(fdx_ctx *c, uint64_t need, uint64_t keep) {
    if (need <= c->list_cap && c->list.p) return FDX_OK;
    const uint64_t want = need + need / 8 + 1024;
    uint32_t *np = nullptr;
    HIPCHK(c, hipMalloc((void **)&np, want * sizeof(uint32_t)));
    if (keep && c->list.p)
        HIPCHK(c, hipMemcpyAsync(np, c->list.p, keep * sizeof(uint32_t), hipMemcpyDeviceToDevice,
                                 c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->gen++;
    c->list.release();
    c->list.p = np;
    c->list.cap = want;
    c->list_cap = want;
    return FDX_OK;
}

}  // namespace

int ext_predicted_walk(fdx_ctx *c, uint32_t G) {
    Pred *p = pred_of(c);
    if (!p->loaded) return fail(c, FDX_ESTATE, "FDX_PREDICTOR: no predictor trained or loaded");
    hipStream_t s = c->stream;
    Groups gv = groups_view(c);
    Cells cv = cells_view(c);
    const double th2 = c->theta * c->theta;
    HIPCHK(c, p->X.ensure((size_t)c->group_cap * kMlpIn));
    HIPCHK(c, p->y.ensure(c->group_cap));
    // features -> network -> capacities -> segment offsets
    HIPCHK(c, mlp_features(G, gv, cv, c->sys_off.p, p->mu.p, p->sd.p, p->X.p, c->st, s));
    HIPCHK(c, mlp_infer(G, &c->st->n_groups_c, p->X.p, p->P.p, p->y.p, s));
    uint32_t cap_max = 0;
    for (int k = 0; k < c->nsys; k++)
        cap_max = std::max<uint32_t>(cap_max, (uint32_t)(c->sys_off_h[k + 1] - c->sys_off_h[k]));
    HIPCHK(c, pred_caps(G, p->y.p, p->margin, std::max<uint32_t>(cap_max, 1), c->lcap.p, c->st, s));
    mark(c, 9);
    c->predict_marked = (c->flags & FDX_TIMING) != 0;
    HIPCHK(c, scan_u32_to_u64(c->lcap.p, c->seg.p, 0, nullptr, &c->st->n_groups_c, c->partial.p,
                              &c->st->list_total, s));
    int r = read_status(c);
    if (r) return r;
    const uint64_t total = c->hst->st.list_total;
    r = ensure_list_capacity(c, total + total / 8);
    if (r) return r;
    // single walk into the predicted segments; a list that outgrows its segment moves to the
    // space after all segments (the buffer holds total + total / 8) and is walked again there
    HIPCHK(c, walk_runs(true, G, gv, cv, th2, c->seg.p, c->lcap.p, c->list_cap, c->list.p,
                        c->cnt_e.p, c->cnt_s.p, c->ovf_list.p, nullptr, nullptr, c->st, s, true));
    r = read_status(c);
    if (r) return r;
    if (c->hst->st.walk_error) return fail(c, FDX_EHIP, "walk stack exhausted");
    const uint32_t K = c->hst->st.list_overflow;
    const uint32_t spilled = c->hst->st.spilled;
    const uint64_t used = total + c->hst->st.spill_used;   // entries in use (some reserved
                                                            // space may go unused)
    c->ext.list_spills += spilled;
    uint64_t extra = 0;
    if (K) {
        // exact re-walk of the groups that found no room, into segments appended after the
        // relocated lists
        HIPCHK(c, p->nsel.ensure(1));
        HIPCHK(c, p->ocap.ensure(K));
        HIPCHK(c, p->ooff.ensure((size_t)K + 1));
        HIPCHK(c, p->base_total.ensure(2));
        HIPCHK(c, hipMemcpyAsync(p->nsel.p, &c->st->list_overflow, 4, hipMemcpyDeviceToDevice, s));
        const uint64_t base_host = std::min<uint64_t>(used, c->list_cap);
        HIPCHK(c, hipMemcpyAsync(p->base_total.p, &base_host, 8, hipMemcpyHostToDevice, s));
        HIPCHK(c, walk_runs(false, K, gv, cv, th2, nullptr, nullptr, 0, nullptr, c->cnt_e.p,
                            c->cnt_s.p, nullptr, c->ovf_list.p, p->nsel.p, c->st, s));
        HIPCHK(c, ovf_caps(K, p->nsel.p, c->ovf_list.p, c->cnt_e.p, c->cnt_s.p, p->ocap.p, s));
        HIPCHK(c, scan_u32_to_u64(p->ocap.p, p->ooff.p, K, nullptr, nullptr, c->partial.p,
                                  p->base_total.p + 1, s));
        HIPCHK(c, ovf_seg(K, p->nsel.p, c->ovf_list.p, p->ocap.p, p->ooff.p, p->base_total.p,
                          c->seg.p, c->lcap.p, s));
        uint64_t ex = 0;
        HIPCHK(c, hipMemcpyAsync(&ex, p->base_total.p + 1, 8, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        extra = ex;
        const uint64_t keep = std::min<uint64_t>(used, c->list_cap);
        r = grow_list_keep(c, keep + extra, keep);
        if (r) return r;
        HIPCHK(c, walk_runs(true, K, gv, cv, th2, c->seg.p, c->lcap.p, c->list_cap, c->list.p,
                            c->cnt_e.p, c->cnt_s.p, nullptr, c->ovf_list.p, p->nsel.p, c->st, s));
    }
    c->stats.overflow_groups = K + spilled;
    c->stats.list_capacity = (int64_t)(std::min<uint64_t>(used, c->list_cap) + extra);
    return FDX_OK;
}

int ext_predictor_reserve(fdx_ctx *c) {
    Pred *p = pred_of(c);
    if (!p->loaded) return fail(c, FDX_ESTATE, "FDX_PREDICTOR: no predictor trained or loaded");
    HIPCHK(c, p->X.ensure((size_t)c->group_cap * kMlpIn));
    HIPCHK(c, p->y.ensure(c->group_cap));
    return FDX_OK;
}

int ext_predicted_lengths(fdx_ctx *c, size_t gmax, const float **y) {
    const int r = ext_predictor_reserve(c);
    if (r) return r;
    Pred *p = pred_of(c);
    HIPCHK(c, mlp_features(gmax, groups_view(c), cells_view(c), c->sys_off.p, p->mu.p, p->sd.p,
                           p->X.p, c->st, c->stream));
    HIPCHK(c, mlp_infer(gmax, &c->st->n_groups_c, p->X.p, p->P.p, p->y.p, c->stream));
    *y = p->y.p;
    return FDX_OK;
}

void predictor_release(fdx_ctx *c) {
    Pred *p = static_cast<Pred *>(c->ext.pred);
    if (!p) return;
    for (auto *b : {&p->P, &p->m, &p->v, &p->grad, &p->gpart, &p->lpart, &p->loss, &p->X, &p->y,
                    &p->mu, &p->sd, &p->mu0, &p->sd1, &p->tX, &p->tT})
        b->release();
    p->idx.release(); p->ocap.release(); p->nsel.release();
    p->ooff.release(); p->base_total.release();
    delete p;
    c->ext.pred = nullptr;
}

}  // namespace fdx

using namespace fdx;

namespace {

// Xavier-uniform initialisation from a seeded generator (biases zero).
void init_params(std::vector<float> &P, uint64_t seed) {
    std::mt19937_64 rng(seed);
    auto fill = [&](int off, int fan_in, int fan_out, int n) {
        const float a = std::sqrt(6.0f / (float)(fan_in + fan_out));
        std::uniform_real_distribution<float> u(-a, a);
        for (int k = 0; k < n; k++) P[off + k] = u(rng);
    };
    std::fill(P.begin(), P.end(), 0.0f);
    fill(0, kMlpIn, kMlpHidden, kMlpIn * kMlpHidden);
    const int ow2 = kMlpIn * kMlpHidden + kMlpHidden;
    fill(ow2, kMlpHidden, kMlpHidden, kMlpHidden * kMlpHidden);
    const int ow3 = ow2 + kMlpHidden * kMlpHidden + kMlpHidden;
    fill(ow3, kMlpHidden, 1, kMlpHidden);
}

}  // namespace

extern "C" {

int fdx_mlp_params(void) { return kMlpParams; }

// Raw (unstandardised) features of every group of the last tree: X[8 g + k].
int fdx_predictor_features(fdx_ctx *c, float *X) {
    FDX_ABI_TRY
    if (!c || !X) return FDX_EINVAL;
    if (!c->skey) return fail(c, FDX_ESTATE, "no tree built");
    Pred *p = pred_of(c);
    const size_t G = (size_t)c->stats.n_groups;
    HIPCHK(c, p->X.ensure(std::max<size_t>(G, 1) * kMlpIn));
    HIPCHK(c, p->mu0.ensure(kMlpIn));
    HIPCHK(c, p->sd1.ensure(kMlpIn));
    const float zero[kMlpIn] = {0, 0, 0, 0, 0, 0, 0, 0}, one[kMlpIn] = {1, 1, 1, 1, 1, 1, 1, 1};
    HIPCHK(c, hipMemcpyAsync(p->mu0.p, zero, sizeof zero, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(p->sd1.p, one, sizeof one, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, mlp_features(G, groups_view(c), cells_view(c), c->sys_off.p, p->mu0.p, p->sd1.p,
                           p->X.p, c->st, c->stream));
    if (G) HIPCHK(c, hipMemcpyAsync(X, p->X.p, G * kMlpIn * sizeof(float), hipMemcpyDeviceToHost,
                                    c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return FDX_OK;
    FDX_ABI_CATCH(c)
}

// y = MLP_P(X) for n standardised feature rows (host arrays).
int fdx_mlp_forward(fdx_ctx *c, const float *P, const float *X, int64_t n, float *y) {
    FDX_ABI_TRY
    if (!c || !P || !X || !y || n < 0) return FDX_EINVAL;
    Pred *p = pred_of(c);
    DBuf<float> dP, dX, dy;
    int r = FDX_OK;
    auto run = [&]() -> int {
        HIPCHK(c, dP.ensure(kMlpParams));
        HIPCHK(c, dX.ensure((size_t)n * kMlpIn));
        HIPCHK(c, dy.ensure((size_t)n));
        HIPCHK(c, hipMemcpyAsync(dP.p, P, kMlpParams * 4, hipMemcpyHostToDevice, c->stream));
        if (n) HIPCHK(c, hipMemcpyAsync(dX.p, X, (size_t)n * kMlpIn * 4, hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, mlp_infer((size_t)n, nullptr, dX.p, dP.p, dy.p, c->stream));
        if (n) HIPCHK(c, hipMemcpyAsync(y, dy.p, (size_t)n * 4, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        return FDX_OK;
    };
    r = run();
    (void)p;
    dP.release(); dX.release(); dy.release();
    return r;
    FDX_ABI_CATCH(c)
}

// Full-batch gradient of mean((MLP_P(X) - t)^2) with respect to the 4801 parameters.
int fdx_mlp_grad(fdx_ctx *c, const float *P, const float *X, const float *t, int64_t n,
                 float *grad, float *loss) {
    FDX_ABI_TRY
    if (!c || !P || !X || !t || !grad || n < 1) return FDX_EINVAL;
    DBuf<float> dP, dX, dT, gp, lp, dg, dl;
    DBuf<uint32_t> di;
    auto run = [&]() -> int {
        const size_t nb = mlp_train_blocks((size_t)n);
        HIPCHK(c, dP.ensure(kMlpParams));
        HIPCHK(c, dX.ensure((size_t)n * kMlpIn));
        HIPCHK(c, dT.ensure((size_t)n));
        HIPCHK(c, gp.ensure(nb * kMlpParams));
        HIPCHK(c, lp.ensure(nb));
        HIPCHK(c, dg.ensure(kMlpParams));
        HIPCHK(c, dl.ensure(1));
        HIPCHK(c, di.ensure((size_t)n));
        HIPCHK(c, hipMemcpyAsync(dP.p, P, kMlpParams * 4, hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(dX.p, X, (size_t)n * kMlpIn * 4, hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(dT.p, t, (size_t)n * 4, hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, iota_u32(di.p, (size_t)n, c->stream));
        HIPCHK(c, mlp_grad((size_t)n, di.p, dX.p, dT.p, dP.p, gp.p, lp.p, dg.p, dl.p, c->stream));
        HIPCHK(c, hipMemcpyAsync(grad, dg.p, kMlpParams * 4, hipMemcpyDeviceToHost, c->stream));
        if (loss) HIPCHK(c, hipMemcpyAsync(loss, dl.p, 4, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        return FDX_OK;
    };
    int r = run();
    for (auto *b : {&dP, &dX, &dT, &gp, &lp, &dg, &dl}) b->release();
    di.release();
    return r;
    FDX_ABI_CATCH(c)
}

// n_steps Adam steps of the training kernel on host arrays P, m, v (updated in place) with
// the gradients grads[k * 4801 ...], step numbers step0 + 1 ... step0 + n_steps.
int fdx_mlp_adam(fdx_ctx *c, float *P, float *m, float *v, const float *grads, int32_t n_steps,
                 int32_t step0, double lr) {
    FDX_ABI_TRY
    if (!c || !P || !m || !v || !grads || n_steps < 0 || step0 < 0) return FDX_EINVAL;
    if (!(std::isfinite(lr) && lr > 0)) return fail(c, FDX_EINVAL, "lr must be finite and > 0");
    DBuf<float> dP, dm, dv, dg;
    auto run = [&]() -> int {
        const size_t bytes = (size_t)kMlpParams * 4;
        HIPCHK(c, dP.ensure(kMlpParams));
        HIPCHK(c, dm.ensure(kMlpParams));
        HIPCHK(c, dv.ensure(kMlpParams));
        HIPCHK(c, dg.ensure((size_t)std::max(n_steps, 1) * kMlpParams));
        HIPCHK(c, hipMemcpyAsync(dP.p, P, bytes, hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(dm.p, m, bytes, hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(dv.p, v, bytes, hipMemcpyHostToDevice, c->stream));
        if (n_steps)
            HIPCHK(c, hipMemcpyAsync(dg.p, grads, (size_t)n_steps * bytes, hipMemcpyHostToDevice,
                                     c->stream));
        for (int k = 0; k < n_steps; k++)
            HIPCHK(c, mlp_adam(dP.p, dg.p + (size_t)k * kMlpParams, dm.p, dv.p, step0 + k + 1,
                               (float)lr, c->stream));
        HIPCHK(c, hipMemcpyAsync(P, dP.p, bytes, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipMemcpyAsync(m, dm.p, bytes, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipMemcpyAsync(v, dv.p, bytes, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        return FDX_OK;
    };
    const int r = run();
    for (auto *b : {&dP, &dm, &dv, &dg}) b->release();
    return r;
    FDX_ABI_CATCH(c)
}

// Train the predictor on n (raw features, ln list length) samples: standardise with the
// statistics of a seeded 90 % training split, Adam on minibatches of `batch` for `epochs`
// passes, then pick the capacity margin as the 99th percentile of the residual ln t - y on
// the held-out 10 %.  losses[e] = mean training loss of epoch e (optional).
int fdx_predictor_train(fdx_ctx *c, const float *X, const float *t, int64_t n, int32_t epochs,
                        int32_t batch, double lr, int64_t seed, float *losses) {
    FDX_ABI_TRY
    if (!c || !X || !t || n < 16 || epochs < 1 || batch < 1) return FDX_EINVAL;
    Pred *p = pred_of(c);
    hipStream_t s = c->stream;
    std::mt19937_64 rng((uint64_t)seed);
    std::vector<uint32_t> order((size_t)n);
    std::iota(order.begin(), order.end(), 0u);
    std::shuffle(order.begin(), order.end(), rng);
    const size_t ntr = (size_t)(0.9 * (double)n), nte = (size_t)n - ntr;
    // normalisation from the training split
    for (int k = 0; k < kMlpIn; k++) {
        double s1 = 0, s2 = 0;
        for (size_t q = 0; q < ntr; q++) {
            const double v = X[(size_t)order[q] * kMlpIn + k];
            s1 += v; s2 += v * v;
        }
        const double mu = s1 / ntr, var = std::max(0.0, s2 / ntr - mu * mu);
        p->mu_h[k] = (float)mu;
        p->sd_h[k] = (float)(var > 1e-12 ? std::sqrt(var) : 1.0);
    }
    std::vector<float> Xs((size_t)n * kMlpIn);
    for (size_t i = 0; i < (size_t)n; i++)
        for (int k = 0; k < kMlpIn; k++)
            Xs[i * kMlpIn + k] = (X[i * kMlpIn + k] - p->mu_h[k]) / p->sd_h[k];
    std::vector<float> P(kMlpParams);
    init_params(P, (uint64_t)seed ^ 0x9E3779B97F4A7C15ull);
    const size_t B = std::min<size_t>((size_t)batch, ntr);
    const size_t nb = mlp_train_blocks(B);
    HIPCHK(c, p->P.ensure(kMlpParams));
    HIPCHK(c, p->m.ensure(kMlpParams));
    HIPCHK(c, p->v.ensure(kMlpParams));
    HIPCHK(c, p->grad.ensure(kMlpParams));
    HIPCHK(c, p->gpart.ensure(nb * kMlpParams));
    HIPCHK(c, p->lpart.ensure(nb));
    HIPCHK(c, p->loss.ensure(1));
    HIPCHK(c, p->tX.ensure((size_t)n * kMlpIn));
    HIPCHK(c, p->tT.ensure((size_t)n));
    HIPCHK(c, p->idx.ensure((size_t)n));
    HIPCHK(c, hipMemcpyAsync(p->P.p, P.data(), kMlpParams * 4, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(p->tX.p, Xs.data(), Xs.size() * 4, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(p->tT.p, t, (size_t)n * 4, hipMemcpyHostToDevice, s));
    std::vector<float> zeros(kMlpParams, 0.0f);
    HIPCHK(c, hipMemcpyAsync(p->m.p, zeros.data(), kMlpParams * 4, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(p->v.p, zeros.data(), kMlpParams * 4, hipMemcpyHostToDevice, s));
    p->step = 0;
    std::vector<uint32_t> tr(order.begin(), order.begin() + ntr);
    for (int e = 0; e < epochs; e++) {
        std::shuffle(tr.begin(), tr.end(), rng);
        HIPCHK(c, hipMemcpyAsync(p->idx.p, tr.data(), ntr * 4, hipMemcpyHostToDevice, s));
        double esum = 0;
        size_t nbt = 0;
        for (size_t b0 = 0; b0 + B <= ntr; b0 += B) {
            HIPCHK(c, mlp_grad(B, p->idx.p + b0, p->tX.p, p->tT.p, p->P.p, p->gpart.p, p->lpart.p,
                               p->grad.p, p->loss.p, s));
            HIPCHK(c, mlp_adam(p->P.p, p->grad.p, p->m.p, p->v.p, ++p->step, (float)lr, s));
            float l = 0;
            HIPCHK(c, hipMemcpyAsync(&l, p->loss.p, 4, hipMemcpyDeviceToHost, s));
            HIPCHK(c, hipStreamSynchronize(s));
            esum += l;
            nbt++;
        }
        if (losses) losses[e] = (float)(nbt ? esum / nbt : 0.0);
    }
    // margin from the held-out split
    std::vector<float> yh(nte), Xte(nte * kMlpIn);
    for (size_t q = 0; q < nte; q++)
        std::memcpy(&Xte[q * kMlpIn], &Xs[(size_t)order[ntr + q] * kMlpIn], kMlpIn * 4);
    std::vector<float> Ph(kMlpParams);
    HIPCHK(c, hipMemcpyAsync(Ph.data(), p->P.p, kMlpParams * 4, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    int r = fdx_mlp_forward(c, Ph.data(), Xte.data(), (int64_t)nte, yh.data());
    if (r) return r;
    std::vector<float> res(nte);
    for (size_t q = 0; q < nte; q++) res[q] = t[order[ntr + q]] - yh[q];
    std::sort(res.begin(), res.end());
    p->margin = nte ? res[std::min(nte - 1, (size_t)std::ceil(0.99 * (double)nte))] : 0.5f;
    p->margin = std::max(p->margin, 0.0f);
    r = upload_norm(c, p);
    if (r) return r;
    HIPCHK(c, hipStreamSynchronize(s));
    p->loaded = true;
    return FDX_OK;
    FDX_ABI_CATCH(c)
}

// margin: ln of the factor applied to predicted lengths (the trained value when the
// argument is NaN); returns the margin in effect through *out (optional).
int fdx_predictor_margin(fdx_ctx *c, double margin, double *out) {
    FDX_ABI_TRY
    if (!c) return FDX_EINVAL;
    Pred *p = pred_of(c);
    if (!p->loaded) return fail(c, FDX_ESTATE, "no predictor trained or loaded");
    if (!std::isnan(margin)) p->margin = (float)margin;
    if (out) *out = p->margin;
    return FDX_OK;
    FDX_ABI_CATCH(c)
}

static const char kMagic[8] = {'F', 'D', 'X', 'M', 'L', 'P', '1', 0};

int fdx_predictor_save(fdx_ctx *c, const char *path) {
    FDX_ABI_TRY
    if (!c || !path) return FDX_EINVAL;
    Pred *p = pred_of(c);
    if (!p->loaded) return fail(c, FDX_ESTATE, "no predictor trained or loaded");
    std::vector<float> P(kMlpParams);
    HIPCHK(c, hipMemcpy(P.data(), p->P.p, kMlpParams * 4, hipMemcpyDeviceToHost));
    FILE *f = std::fopen(path, "wb");
    if (!f) return fail(c, FDX_EINVAL, "cannot open %s", path);
    bool ok = std::fwrite(kMagic, 1, 8, f) == 8 && std::fwrite(p->mu_h, 4, kMlpIn, f) == kMlpIn &&
              std::fwrite(p->sd_h, 4, kMlpIn, f) == kMlpIn && std::fwrite(&p->margin, 4, 1, f) == 1 &&
              std::fwrite(P.data(), 4, kMlpParams, f) == (size_t)kMlpParams;
    ok = (std::fclose(f) == 0) && ok;
    return ok ? FDX_OK : fail(c, FDX_EINVAL, "write failed: %s", path);
    FDX_ABI_CATCH(c)
}

int fdx_predictor_load(fdx_ctx *c, const char *path) {
    FDX_ABI_TRY
    if (!c || !path) return FDX_EINVAL;
    Pred *p = pred_of(c);
    FILE *f = std::fopen(path, "rb");
    if (!f) return fail(c, FDX_EINVAL, "cannot open %s", path);
    char mg[8];
    std::vector<float> P(kMlpParams);
    float mu[kMlpIn], sd[kMlpIn], margin = 0;
    bool ok = std::fread(mg, 1, 8, f) == 8 && std::memcmp(mg, kMagic, 8) == 0 &&
              std::fread(mu, 4, kMlpIn, f) == kMlpIn && std::fread(sd, 4, kMlpIn, f) == kMlpIn &&
              std::fread(&margin, 4, 1, f) == 1 &&
              std::fread(P.data(), 4, kMlpParams, f) == (size_t)kMlpParams;
    std::fclose(f);
    if (!ok) return fail(c, FDX_EINVAL, "not a predictor file: %s", path);
    std::memcpy(p->mu_h, mu, sizeof mu);
    std::memcpy(p->sd_h, sd, sizeof sd);
    p->margin = margin;
    HIPCHK(c, p->P.ensure(kMlpParams));
    HIPCHK(c, hipMemcpy(p->P.p, P.data(), kMlpParams * 4, hipMemcpyHostToDevice));
    int r = upload_norm(c, p);
    if (r) return r;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    p->loaded = true;
    return FDX_OK;
    FDX_ABI_CATCH(c)
}

}  // extern "C"
