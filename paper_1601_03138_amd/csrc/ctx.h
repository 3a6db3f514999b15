// Host-side context of the Barnes-Hut library (shared by the C ABI and the host extensions:
// predictor, autotuner, graph capture).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/fdx.h"
#include "abi_guard.h"
#include "fdx_internal.h"
#include "host_ext.h"

namespace fdx {

template <class T>
struct DBuf {
    T *p = nullptr;
    size_t cap = 0;
    bool fixed = false;      // memory the buffer does not own: never grown or freed
    hipError_t ensure(size_t n) {
        if (n == 0) n = 1;
        if (n <= cap) return hipSuccess;
        if (fixed) return hipErrorOutOfMemory;
        release();
        hipError_t e = hipMalloc((void **)&p, n * sizeof(T));
        if (e != hipSuccess) { p = nullptr; cap = 0; return e; }
        cap = n;
        return hipSuccess;
    }
    void release() {
        if (p && !fixed) (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
};

struct HostStatus {
    DevStatus st;
    uint32_t lvl[kLevels + 2];
};

}  // namespace fdx

struct fdx_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    char err[512] = {};           // message of the last failed call (fixed size: writing it
                                  // never allocates)

    // particles (caller's order)
    int64_t n = 0;
    int nsys = 0;
    bool have_particles = false, borrowed = false, eps_given = false;
    // every system's particles share one eps: the sorted gather takes it from the system's first
    // particle instead of reading eps through the permutation (the same result, one random
    // read per particle less)
    bool eps_per_system = false;
    std::vector<int64_t> sys_off_h;
    fdx::DBuf<double> ox, oy, oz, ovx, ovy, ovz, om, oeps;       // owned copies
    double *x = nullptr, *y = nullptr, *z = nullptr, *vx = nullptr, *vy = nullptr,
           *vz = nullptr, *m = nullptr, *eps = nullptr;    // active arrays
    fdx::DBuf<int64_t> sys_off;
    fdx::DBuf<uint32_t> sysid;

    // keys and order
    fdx::DBuf<uint64_t> bbox_u, key, key_alt;
    fdx::DBuf<double> cube;
    fdx::DBuf<uint32_t> perm, perm_alt, inv, rs_scratch;
    fdx::DBuf<uint16_t> sys_carry;                               // 2n: sort carry (several systems)
    fdx::DBuf<uint64_t> partial;
    uint64_t *skey = nullptr;
    uint32_t *sperm = nullptr;
    fdx::DBuf<double4> jp, packed;
    fdx::DBuf<double> seps;

    // tree
    fdx::DBuf<uint32_t> c_level, c_begin, c_count, c_first, c_nchild, c_parent, c_lvl;
    fdx::DBuf<uint64_t> c_prefix;
    fdx::DBuf<uint4> c_node;
    fdx::DBuf<uint2> c_link;
    fdx::DBuf<double> c_mom;
    fdx::DBuf<uint32_t> tmp_n, tmp_off;
    uint32_t cell_cap = 0;

    // groups
    fdx::DBuf<uint32_t> g_cell, g_begin, g_count, g_sys, g_box, flag, gcell_at, gpos;
    fdx::DBuf<uint32_t> g_wide, wide_list;     // groups evaluated in FP64 by the FP32 path
    fdx::DBuf<uint8_t> leaf_lev;               // level of every sorted particle's leaf
    fdx::DBuf<double> g_centre;
    uint32_t group_cap = 0;

    // lists
    fdx::DBuf<uint32_t> cnt_e, cnt_s, lcap, list, ovf_list;
    fdx::DBuf<uint64_t> seg;
    uint64_t list_cap = 0;

    // one-launch walk + force: cost per group, its prefix sums, the eight queue runs
    fdx::DBuf<uint32_t> f_cost, f_bounds;
    fdx::DBuf<uint64_t> f_pre;
    bool capture_lists = false;    // FDX_FUSED: also store the lists (fdx_set_list_capture)
    bool have_counts = false;      // cnt_e / cnt_s belong to the current groups

    // forces
    fdx::DBuf<double4> fs;
    fdx::DBuf<double> ax, ay, az, pot;
    bool have_force = false;
    bool have_lists = false;       // the lists belong to the current groups (last walk)

    // status
    fdx::DevStatus *st = nullptr;
    fdx::HostStatus *hst = nullptr;

    // last parameters
    double theta = 0.5, eps_all = 0.0;
    int n_leaf = 8, n_group = 64, flags = 0, variant = -1;
    double cutoff = 0.0;           // > 0: the last evaluation was the TreePM cutoff kernel
    // parameters of the last fdx_calc_force / fdx_calc_force_cutoff: fdx_integrate steps with
    // these (the tree-only, density, exchange-list and autotuner calls set the fields above
    // for their own passes)
    struct ForceParams {
        double theta = 0.5, eps_all = 0.0, cutoff = 0.0;
        int n_leaf = 8, n_group = 64, flags = 0;
    } last_force;
    fdx_stats stats{};
    hipEvent_t ev[12] = {};
    bool predict_marked = false;   // event 9 holds the end of the predictor's network

    fdx::HostExt ext;   // predictor, autotuner, graph state

    // every device buffer of the context (fdx_destroy frees them; the no-allocation entry
    // point marks them fixed so that a buffer it did not carve fails instead of allocating)
    template <class F>
    void each_buffer(F f) {
        f(ox); f(oy); f(oz); f(ovx); f(ovy); f(ovz); f(om); f(oeps);
        f(sys_off); f(sysid);
        f(bbox_u); f(key); f(key_alt); f(cube);
        f(perm); f(perm_alt); f(inv); f(rs_scratch); f(sys_carry); f(partial);
        f(jp); f(packed); f(seps);
        f(c_level); f(c_begin); f(c_count); f(c_first); f(c_nchild); f(c_parent); f(c_lvl);
        f(c_prefix); f(c_node); f(c_link); f(c_mom); f(tmp_n); f(tmp_off);
        f(g_cell); f(g_begin); f(g_count); f(g_sys); f(g_box); f(flag); f(gcell_at); f(gpos);
        f(g_wide); f(wide_list); f(leaf_lev); f(g_centre);
        f(cnt_e); f(cnt_s); f(lcap); f(list); f(ovf_list); f(seg);
        f(f_cost); f(f_bounds); f(f_pre);
        f(fs); f(ax); f(ay); f(az); f(pot);
    }
    // bumped by every fdx_set_particles and every reallocation of a buffer a captured graph
    // refers to; a graph captured under another generation is never replayed
    uint64_t gen = 0;
};

namespace fdx {

int fail(fdx_ctx *c, int code, const char *fmt, ...);

// FDX_ABI_CATCH handler: status code of the exception in flight, message into c->err
inline int abi_exception(fdx_ctx *c) noexcept {
    return classify_exception(c ? c->err : nullptr, c ? sizeof c->err : 0);
}

#define HIPCHK(ctx, expr)                                                                     \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return ::fdx::fail(ctx, e_ == hipErrorOutOfMemory ? FDX_ENOMEM : FDX_EHIP,         \
                               "%s: %s (%s)", #expr, hipGetErrorString(e_), __func__);       \
    } while (0)

Cells cells_view(fdx_ctx *c);
Groups groups_view(fdx_ctx *c);
void mark(fdx_ctx *c, int k);
int read_status(fdx_ctx *c);
int run_tree(fdx_ctx *c, bool sync);
int run_force(fdx_ctx *c);
int enqueue_keys_sort(fdx_ctx *c);
int enqueue_tree_groups(fdx_ctx *c);
int enqueue_count(fdx_ctx *c, size_t gmax);
int enqueue_fill(fdx_ctx *c, size_t gmax, bool spill = false);
// segments sized per system (sys_cap, device array indexed by system), no count walk
int enqueue_sys_caps(fdx_ctx *c, size_t gmax, const uint32_t *sys_cap);
int enqueue_force(fdx_ctx *c, size_t gmax);
// walk + force in one launch, then the return of forces (capture: lists into c->list)
int enqueue_fused(fdx_ctx *c, size_t gmax, bool capture);
int ensure_list_capacity(fdx_ctx *c, uint64_t total);
int setup_eval(fdx_ctx *c, double theta, int n_leaf, int n_group, double eps, int flags);
void save_force_params(fdx_ctx *c);
void restore_force_params(fdx_ctx *c);
void finish_stats(fdx_ctx *c);
int sync_timing(fdx_ctx *c);
int read_counters(fdx_ctx *c);
int ensure_tree_buffers(fdx_ctx *c, uint32_t cell_cap, uint32_t group_cap);

}  // namespace fdx
