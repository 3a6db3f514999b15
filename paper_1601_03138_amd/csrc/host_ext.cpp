// Host extensions of the force path: force-kernel shape choice and autotuner, and HIP-graph
// capture of leapfrog steps.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "ctx.h"
#include "predictor.h"

namespace fdx {

int ext_force_variant(fdx_ctx *c) {
    // shapes used when none is set or tuned: FP32 nt512_ipl1_pf_w8 for the direct launch and
    // nt512_ipl1_w8 (no register prefetch: no spills in the persistent loop) for the
    // persistent launch, FP64 nt256_ipl2 (no prefetch; also the shape of the wide-group
    // hand-off).  At N = 2^24 the autotuner finds nt512_ipl2 about 1.3 % faster for FP32.
    const bool f32 = (c->flags & FDX_FP32REL) != 0;
    const int dflt = f32 ? ((c->flags & FDX_PERSISTENT) ? 9 : 8) : 5;
    int v = c->ext.variant[f32] >= 0 ? c->ext.variant[f32] : dflt;
    if (force_variant_capacity(v) < c->n_group) v = 3;
    return v;
}

// ---------------------------------------------------------------------------------------
// Graph-captured leapfrog step: kick + drift, the whole force evaluation (walk into a
// fixed-capacity list buffer, persistent force kernel over per-XCD queues), kick.  With
// several systems every group's segment is sized by its system: min(particles of the system,
// percent / 100 x the longest list the system had in the evaluation before the capture + 64;
// a list that outgrows it moves to the buffer's spare quarter inside the walk), and one
// fill walk builds the lists, if the segments fit the list budget; otherwise a count walk
// sizes them first.  Capacities are fixed at capture time with a margin; a step whose tree,
// groups or lists do not fit is reported by the device status: its final kick is skipped, the
// host redoes force and kick eagerly with larger buffers (and a doubled list percentage) and
// captures again.
struct GraphState {
    hipStream_t gs = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // everything the captured launches depend on
    uint64_t gen = 0;
    double dt = 0, theta = 0, eps_all = 0;
    int flags = 0, n_leaf = 0, n_group = 0, variant = 0, nsys = 0;
    int64_t n = -1;
    bool sized = false;           // segments sized per system (no count walk)
    DBuf<uint32_t> sys_cap, lmax;
    void drop() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    }
};

static int capture_step(fdx_ctx *c, GraphState *g, double dt) {
    const size_t n = (size_t)c->n;
    g->drop();
    HIPCHK(c, hipStreamBeginCapture(g->gs, hipStreamCaptureModeRelaxed));
    int r = FDX_OK;
    auto step = [&]() -> int {
        HIPCHK(c, kick_drift(n, c->x, c->y, c->z, c->vx, c->vy, c->vz, c->ax.p, c->ay.p, c->az.p,
                             dt, g->gs));
        int q = enqueue_keys_sort(c);
        if (!q) q = enqueue_tree_groups(c);
        if (c->flags & FDX_FUSED) {
            if (!q) q = enqueue_fused(c, c->group_cap, false);
        } else {
            if (!q) q = g->sized ? enqueue_sys_caps(c, c->group_cap, g->sys_cap.p)
                                 : enqueue_count(c, c->group_cap);
            if (!q) q = enqueue_fill(c, c->group_cap, g->sized);
            if (!q) q = enqueue_force(c, c->group_cap);
        }
        if (q) return q;
        HIPCHK(c, kick(n, c->vx, c->vy, c->vz, c->ax.p, c->ay.p, c->az.p, dt, c->st, g->gs));
        return FDX_OK;
    };
    r = step();
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(g->gs, &graph);
    if (r) {
        if (graph) (void)hipGraphDestroy(graph);
        return r;
    }
    if (e != hipSuccess) return fail(c, FDX_EHIP, "graph capture failed: %s", hipGetErrorString(e));
    g->graph = graph;
    e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        g->drop();
        return fail(c, FDX_EHIP, "graph instantiate failed: %s", hipGetErrorString(e));
    }
    g->gen = c->gen;
    g->dt = dt;
    g->theta = c->theta;
    g->eps_all = c->eps_all;
    g->flags = c->flags;
    g->n_leaf = c->n_leaf;
    g->n_group = c->n_group;
    g->variant = ext_force_variant(c);
    g->nsys = c->nsys;
    g->n = c->n;
    return FDX_OK;
}

static bool graph_stale(fdx_ctx *c, GraphState *g, double dt) {
    return !g->exec || g->gen != c->gen || g->dt != dt || g->theta != c->theta ||
           g->eps_all != c->eps_all || g->flags != c->flags || g->n_leaf != c->n_leaf ||
           g->n_group != c->n_group || g->variant != ext_force_variant(c) ||
           g->nsys != c->nsys || g->n != c->n;
}

void ext_invalidate(fdx_ctx *c) {
    GraphState *g = static_cast<GraphState *>(c->ext.graph);
    if (g) g->drop();
}

// list entries (4 B each) the per-system segments may take: 16 GiB
constexpr uint64_t kSizedBudget = 1ull << 32;

// capacities with headroom for the drift of one step; chooses the segment sizing.  The
// per-system statistics are read from the current groups and lists before any buffer is
// grown: growing reallocates the group arrays and drops their contents.
static int graph_headroom(fdx_ctx *c, GraphState *g) {
    const DevStatus h = c->hst->st;         // the last evaluation's tree and lists
    const uint32_t ncell = c->hst->lvl[kLevels + 1];
    const int S = c->nsys;
    const uint64_t pct = c->ext.graph_margin_pct;
    const bool try_sized = S > 1 && c->have_lists && pct > 0 && !(c->flags & FDX_FUSED);
    std::vector<uint32_t> st2;              // [longest list per system, groups per system]
    if (try_sized) {
        HIPCHK(c, g->lmax.ensure(2 * (size_t)S));
        HIPCHK(c, fill_u32(g->lmax.p, 0u, 2 * (size_t)S, c->stream));
        HIPCHK(c, sys_lmax(c->group_cap, c->g_sys.p, c->cnt_e.p, c->cnt_s.p, g->lmax.p,
                           g->lmax.p + S, c->st, c->stream));
        st2.resize(2 * (size_t)S);
        HIPCHK(c, hipMemcpyAsync(st2.data(), g->lmax.p, 8 * (size_t)S, hipMemcpyDeviceToHost,
                                 c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    c->have_lists = false;                  // buffers may be reallocated below
    c->have_counts = false;
    uint32_t ccap = std::max<uint32_t>(c->cell_cap, ncell + ncell / 4 + 1024);
    uint32_t gcap = std::max<uint32_t>(c->group_cap, h.n_groups + h.n_groups / 4 + 1024);
    int r = ensure_tree_buffers(c, ccap, gcap);
    if (r) return r;
    if (c->flags & FDX_FUSED) {
        // one walk + force launch: no list buffer; the predictor's buffers (if used) are sized
        // now, outside the capture
        g->sized = false;
        return (c->flags & FDX_PREDICTOR) ? ext_predictor_reserve(c) : FDX_OK;
    }
    uint64_t need = h.list_total;
    g->sized = false;
    if (try_sized) {
        std::vector<uint32_t> cap(S);
        uint64_t total = 0;
        for (int s = 0; s < S; s++) {
            const uint64_t ns = (uint64_t)(c->sys_off_h[s + 1] - c->sys_off_h[s]);
            cap[s] = (uint32_t)std::min<uint64_t>(ns, pct * st2[s] / 100 + 64);
            total += (uint64_t)st2[S + s] * cap[s];
        }
        if (total + total / 4 + 4096 <= kSizedBudget) {
            HIPCHK(c, g->sys_cap.ensure(S));
            HIPCHK(c, hipMemcpyAsync(g->sys_cap.p, cap.data(), 4 * (size_t)S,
                                     hipMemcpyHostToDevice, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));     // cap is a host vector
            g->sized = true;
            need = total;
        }
    }
    return ensure_list_capacity(c, need + need / 4 + 4096);
}

int ext_integrate_graph(fdx_ctx *c, double dt, int n_steps) {
    GraphState *g = static_cast<GraphState *>(c->ext.graph);
    if (!g) {
        g = new GraphState();
        c->ext.graph = g;
    }
    if (!g->gs) HIPCHK(c, hipStreamCreate(&g->gs));
    hipStream_t user = c->stream;
    const int user_flags = c->flags;
    HIPCHK(c, hipStreamSynchronize(user));
    c->stream = g->gs;
    // the predicted walk reads its totals back on the host, so it is not captured; the fused
    // launch uses the predictor on the device only and keeps it
    c->flags = (user_flags | FDX_PERSISTENT) &
               ~(FDX_TIMING | ((user_flags & FDX_FUSED) ? 0 : FDX_PREDICTOR));
    const size_t n = (size_t)c->n;
    int r = FDX_OK;
    for (int k = 0; k < n_steps && !r; k++) {
        if (graph_stale(c, g, dt)) {
            r = graph_headroom(c, g);
            if (!r) r = capture_step(c, g, dt);
            if (r) break;
        }
        hipError_t e = hipGraphLaunch(g->exec, g->gs);
        if (e != hipSuccess) { r = fail(c, FDX_EHIP, "graph launch: %s", hipGetErrorString(e)); break; }
        r = read_status(c);
        if (r) break;
        const DevStatus h = c->hst->st;
        c->ext.list_spills += h.spilled;
        if (h.bad_input) { r = fail(c, FDX_EINVAL, "non-finite particle data"); break; }
        // the replay's lists (or the eager redo's); the fused launch stores counts only
        c->have_lists = !(c->flags & FDX_FUSED);
        c->have_counts = true;
        if (status_incomplete(h)) {
            // positions and velocities hold kick + drift; redo force and kick eagerly
            r = run_tree(c, true);
            if (!r) r = run_force(c);
            if (r) break;
            hipError_t ek = hipSuccess;
            ek = kick(n, c->vx, c->vy, c->vz, c->ax.p, c->ay.p, c->az.p, dt, nullptr, g->gs);
            if (ek != hipSuccess) { r = fail(c, FDX_EHIP, "kick: %s", hipGetErrorString(ek)); break; }
            r = read_status(c);
            if (r) break;
            c->ext.graph_recoveries++;
            if (g->sized && h.list_overflow && c->ext.graph_margin_pct < (1u << 20))
                c->ext.graph_margin_pct *= 2;
            g->drop();
        }
    }
    if (!r) {
        finish_stats(c);
        hipError_t e = hipStreamSynchronize(g->gs);
        if (e != hipSuccess) r = fail(c, FDX_EHIP, "sync: %s", hipGetErrorString(e));
    }
    c->stream = user;
    c->flags = user_flags;
    if (!r) r = read_counters(c);
    return r;
}

void ext_release(fdx_ctx *c) {
    GraphState *g = static_cast<GraphState *>(c->ext.graph);
    if (g) {
        g->drop();
        g->sys_cap.release();
        g->lmax.release();
        if (g->gs) (void)hipStreamDestroy(g->gs);
        delete g;
        c->ext.graph = nullptr;
    }
    predictor_release(c);
    exchange_release(c);
    sph_release(c);
    dd_release(c);
}

}  // namespace fdx

using namespace fdx;

extern "C" {

int fdx_autotune_shapes(void) { return force_variants(); }

const char *fdx_shape_name(int32_t shape) {
    return shape < 0 || shape >= force_variants() ? "" : force_variant_name(shape);
}

int fdx_set_graph_list_margin(fdx_ctx *c, int32_t percent) {
    FDX_ABI_TRY
    if (!c) return FDX_EINVAL;
    if (percent < 0) return fail(c, FDX_EINVAL, "percent must be >= 0");
    c->ext.graph_margin_pct = (uint32_t)percent;
    ext_invalidate(c);
    return FDX_OK;
    FDX_ABI_CATCH(c)
}

int fdx_set_shape(fdx_ctx *c, int32_t shape) {
    FDX_ABI_TRY
    if (!c) return FDX_EINVAL;
    if (shape < -1 || shape >= force_variants()) return fail(c, FDX_EINVAL, "shape out of range");
    c->ext.variant[0] = c->ext.variant[1] = shape;
    return FDX_OK;
    FDX_ABI_CATCH(c)
}

int fdx_autotune(fdx_ctx *c, double theta, int32_t n_leaf, double eps, int32_t flags,
                 const int32_t *n_group_cand, int32_t n_cand, int32_t reps, double *times_ms,
                 int32_t *best_n_group, int32_t *best_shape) {
    FDX_ABI_TRY
    if (!c) return FDX_EINVAL;
    if (!n_group_cand || n_cand < 1 || reps < 1) return fail(c, FDX_EINVAL, "no candidates");
    const int nv = force_variants();
    double best = 1e300;
    int bg = -1, bv = -1;
    // the search sets the shape of the precision it times; the other keeps its own
    const bool f32 = (flags & FDX_FP32REL) != 0;
    int &slot = c->ext.variant[f32];
    const int saved = slot;
    // FDX_GRAPH: time graph-captured leapfrog steps of dt = 0 (x += 0 v, v += 0 a: the state
    // does not change), which is what a graph-replayed run executes per step
    const bool graph = (flags & FDX_GRAPH) != 0;
    flags &= ~(FDX_TIMING | FDX_PREDICTOR | FDX_GRAPH);
    if (graph) flags |= FDX_PERSISTENT;
    // the caller's last force evaluation, re-done at the end so that forces, lists and the
    // parameters fdx_integrate uses are the caller's again, not the last candidate's
    const bool had_force = c->have_force;
    const fdx_ctx::ForceParams caller = c->last_force;
    // shapes whose registers spill are not timed when a shape that does not spill can take
    // the group size: they move their spills through memory on every tile, and a tie decided
    // by timing noise would pick them
    std::vector<int> spills(nv);
    for (int v = 0; v < nv; v++)
        spills[v] = force_variant_scratch(f32, (flags & FDX_QUAD) != 0,
                                          (flags & FDX_PERSISTENT) != 0, v) > 0;
    for (int k = 0; k < n_cand; k++) {
        bool clean = false;
        for (int v = 0; v < nv; v++)
            clean |= force_variant_capacity(v) >= n_group_cand[k] && !spills[v];
        // the fused launch has no separate force-kernel shape: one timing per group size
        const bool fused = (flags & FDX_FUSED) != 0;
        for (int v = 0; v < nv; v++) {
            double t = NAN;
            const bool fits = fused ? (v == 0 && n_group_cand[k] <= kFusedMaxGroup)
                                    : force_variant_capacity(v) >= n_group_cand[k] &&
                                          !(clean && spills[v]);
            if (fits) {
                slot = v;
                int r = fdx_calc_force(c, theta, n_leaf, n_group_cand[k], eps, flags);
                if (!r && graph) r = fdx_integrate(c, 0.0, 1, FDX_GRAPH);     // capture
                if (r) { slot = saved; return r; }
                std::vector<double> ts;
                for (int q = 0; q < reps; q++) {
                    auto t0 = std::chrono::steady_clock::now();
                    r = graph ? fdx_integrate(c, 0.0, 1, FDX_GRAPH)
                              : fdx_calc_force(c, theta, n_leaf, n_group_cand[k], eps, flags);
                    if (r) { slot = saved; return r; }
                    auto t1 = std::chrono::steady_clock::now();
                    ts.push_back(std::chrono::duration<double, std::milli>(t1 - t0).count());
                }
                std::sort(ts.begin(), ts.end());
                t = ts[ts.size() / 2];
                if (t < best) { best = t; bg = n_group_cand[k]; bv = v; }
            }
            if (times_ms) times_ms[(size_t)k * nv + v] = t;
        }
    }
    slot = bv;
    if (had_force) {
        const int r = caller.cutoff > 0
            ? fdx_calc_force_cutoff(c, caller.theta, caller.n_leaf, caller.n_group,
                                    caller.eps_all, caller.cutoff, caller.flags)
            : fdx_calc_force(c, caller.theta, caller.n_leaf, caller.n_group, caller.eps_all,
                             caller.flags);
        if (r) return r;
    } else {
        c->have_force = false;      // the candidates' evaluations were not the caller's
    }
    if (best_n_group) *best_n_group = bg;
    if (best_shape) *best_shape = bv;
    return FDX_OK;
    FDX_ABI_CATCH(c)
}

// Autotuner results recorded in a text file, one JSON object per line:
//   {"key": "<arch>|n2^<k>|sys2^<k>|theta=<g>|leaf=<n>|flags=<f>|cand=<a,b,..>|reps=<r>",
//    "n_group": <g>, "shape": <v>}
// The last line with the same key wins; lines that do not parse are ignored.
int fdx_autotune_cached(fdx_ctx *c, const char *path, double theta, int32_t n_leaf, double eps,
                        int32_t flags, const int32_t *n_group_cand, int32_t n_cand, int32_t reps,
                        int32_t *best_n_group, int32_t *best_shape, int32_t *from_cache) {
    FDX_ABI_TRY
    if (!c) return FDX_EINVAL;
    if (!path || !n_group_cand || n_cand < 1 || reps < 1)
        return fail(c, FDX_EINVAL, "null path or no candidates");
    if (!c->have_particles) return fail(c, FDX_ESTATE, "no particles: call fdx_set_particles first");
    hipDeviceProp_t prop;
    HIPCHK(c, hipGetDeviceProperties(&prop, c->device));
    auto lg = [](int64_t v) { int k = 0; while (v > 1) { v >>= 1; k++; } return k; };
    const int32_t fkey = flags & (FDX_QUAD | FDX_FP32REL | FDX_PERSISTENT | FDX_GRAPH);
    char head[256];
    snprintf(head, sizeof(head), "%s|n2^%d|sys2^%d|theta=%.9g|leaf=%d|flags=%d|cand=",
             prop.gcnArchName, lg(c->n), lg(c->nsys), theta, n_leaf, fkey);
    std::string key = head;
    for (int k = 0; k < n_cand; k++) key += (k ? "," : "") + std::to_string(n_group_cand[k]);
    key += "|reps=" + std::to_string(reps);
    if (from_cache) *from_cache = 0;
    // look the key up
    int g_hit = -1, v_hit = -1;
    if (FILE *f = fopen(path, "r")) {
        char line[1024];
        const std::string want = "{\"key\": \"" + key + "\", ";
        while (fgets(line, sizeof(line), f)) {
            if (strncmp(line, want.c_str(), want.size()) != 0) continue;
            int g = -1, v = -1;
            if (sscanf(line + want.size(), "\"n_group\": %d, \"shape\": %d}", &g, &v) == 2 &&
                g >= 1 && g <= kMaxGroup && v >= 0 && v < force_variants() &&
                force_variant_capacity(v) >= g) {
                g_hit = g;
                v_hit = v;
            }
        }
        fclose(f);
    }
    if (g_hit > 0) {
        c->ext.variant[(flags & FDX_FP32REL) != 0] = v_hit;
        if (best_n_group) *best_n_group = g_hit;
        if (best_shape) *best_shape = v_hit;
        if (from_cache) *from_cache = 1;
        return FDX_OK;
    }
    int32_t bg = -1, bv = -1;
    int r = fdx_autotune(c, theta, n_leaf, eps, flags, n_group_cand, n_cand, reps, nullptr, &bg,
                         &bv);
    if (r) return r;
    FILE *f = fopen(path, "a");
    if (!f) return fail(c, FDX_EINVAL, "cannot append to %s", path);
    fprintf(f, "{\"key\": \"%s\", \"n_group\": %d, \"shape\": %d}\n", key.c_str(), bg, bv);
    const bool ok = fclose(f) == 0;
    if (!ok) return fail(c, FDX_EINVAL, "cannot write %s", path);
    if (best_n_group) *best_n_group = bg;
    if (best_shape) *best_shape = bv;
    return FDX_OK;
    FDX_ABI_CATCH(c)
}

}  // extern "C"
