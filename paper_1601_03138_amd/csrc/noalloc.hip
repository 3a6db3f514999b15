// fdx_calc_force_noalloc: one force evaluation that allocates nothing, for callers that cannot
// call the device allocator (code under HIP graph capture, tight serving loops, harnesses that
// forbid it).
//
// It runs the same launches as fdx_calc_force on one system, with every buffer the library
// would own -- keys, sort scratch, sorted particles, cells, moments, groups, interaction lists,
// device status -- carved out of one file-scope device array of kScratchBytes.  The caller
// passes the particle arrays and the four output arrays in device memory.  Each device holds
// its own copy of the array from the first call on it until the process ends; its address on
// a device is taken once with hipGetSymbolAddress and used from then on (the array's name is
// a host-side stand-in and is never passed to a kernel).  Every call on one device shares that
// array: calls that overlap on one device -- two host threads, or two streams -- race on it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "ctx.h"

using namespace fdx;

namespace {

constexpr size_t kScratchBytes = 128ull << 20;       // 128 MiB per device
constexpr int64_t kMaxParticles = 1 << 17;           // 131072
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mutex;
void *g_scratch[kMaxDevices] = {};

// device address of the scratch array on the current device (taken once per device)
int scratch_ptr(int dev, void **out, char *err, size_t errlen) {
    if (dev < 0 || dev >= kMaxDevices) {
        snprintf(err, errlen, "device %d out of range", dev);
        return FDX_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            snprintf(err, errlen, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
            return FDX_EHIP;
        }
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return FDX_OK;
}

// bump allocation over the scratch array, 256-byte aligned; the buffers it hands out are
// fixed: growing one fails instead of allocating
struct Carver {
    unsigned char *base;
    size_t used = 0, size;
    bool ok = true;
    template <class T>
    void take(DBuf<T> &b, size_t n) {
        if (n == 0) n = 1;
        const size_t off = (used + 255) & ~(size_t)255;
        const size_t bytes = n * sizeof(T);
        if (off + bytes > size) { ok = false; return; }
        b.p = reinterpret_cast<T *>(base + off);
        b.cap = n;
        b.fixed = true;
        used = off + bytes;
    }
    template <class T>
    void rest(DBuf<T> &b, uint64_t *count) {
        const size_t off = (used + 255) & ~(size_t)255;
        const size_t n = off < size ? (size - off) / sizeof(T) : 0;
        *count = n;
        if (n == 0) { ok = false; return; }
        b.p = reinterpret_cast<T *>(base + off);
        b.cap = n;
        b.fixed = true;
        used = size;
    }
};

}  // namespace

extern "C" {

int fdx_calc_force_noalloc(int device, void *hip_stream, int64_t n, const double *x,
                           const double *y, const double *z, const double *m, const double *eps,
                           double eps_all, double theta, int32_t n_leaf, int32_t n_group,
                           int32_t flags, double *ax, double *ay, double *az, double *pot,
                           char *err, int32_t err_len) {
    FDX_ABI_TRY
    char msg[256] = {};
    auto out = [&](int code) {
        if (err && err_len > 0) snprintf(err, (size_t)err_len, "%s", msg);
        return code;
    };
    if (n < 0 || n > kMaxParticles) {
        snprintf(msg, sizeof msg, "n = %lld outside [0, %lld]", (long long)n,
                 (long long)kMaxParticles);
        return out(FDX_EINVAL);
    }
    if (flags & ~(FDX_QUAD | FDX_FP32REL | FDX_PERSISTENT)) {
        snprintf(msg, sizeof msg, "flags may hold FDX_QUAD, FDX_FP32REL and FDX_PERSISTENT only");
        return out(FDX_EINVAL);
    }
    if (n > 0 && (!x || !y || !z || !m || !ax || !ay || !az || !pot)) {
        snprintf(msg, sizeof msg, "null particle or output array");
        return out(FDX_EINVAL);
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        snprintf(msg, sizeof msg, "device %d does not exist", device);
        return out(FDX_EINVAL);
    }
    if (hipSetDevice(device) != hipSuccess) {
        snprintf(msg, sizeof msg, "hipSetDevice(%d) failed", device);
        return out(FDX_EHIP);
    }
    void *base = nullptr;
    int r = scratch_ptr(device, &base, msg, sizeof msg);
    if (r) return out(r);
    if (n == 0) return out(FDX_OK);

    // a context on the stack whose buffers all live in the scratch array
    fdx_ctx c;
    c.device = device;
    c.stream = (hipStream_t)hip_stream;
    c.n = n;
    c.nsys = 1;
    c.borrowed = true;
    c.eps_given = eps != nullptr;
    c.x = const_cast<double *>(x); c.y = const_cast<double *>(y); c.z = const_cast<double *>(z);
    c.m = const_cast<double *>(m); c.eps = const_cast<double *>(eps);
    HostStatus hst{};
    c.hst = &hst;
    const size_t N = (size_t)n, S = 1;
    // cells: room for chains of single-child cells above tight clumps (the eager path grows
    // its cell arrays on demand instead)
    const uint32_t ccap = (uint32_t)(2 * N + S + 1024), gcap = (uint32_t)(N / 8 + S + 1024);
    Carver cv{static_cast<unsigned char *>(base), 0, kScratchBytes};
    DBuf<DevStatus> st;
    cv.take(st, 1);
    c.st = st.p;
    cv.take(c.partial, kScanBlocks + 1);
    cv.take(c.sys_off, S + 1);
    cv.take(c.sysid, N);
    cv.take(c.bbox_u, 6 * S);
    cv.take(c.cube, 4 * S);
    cv.take(c.key, N);
    cv.take(c.key_alt, N);
    cv.take(c.perm, N);
    cv.take(c.perm_alt, N);
    cv.take(c.inv, N);
    cv.take(c.rs_scratch, radix_scratch_u32(std::max<size_t>(N, gcap)));
    cv.take(c.jp, N);
    cv.take(c.packed, N);
    cv.take(c.seps, N);
    cv.take(c.flag, N);
    cv.take(c.gcell_at, N);
    cv.take(c.gpos, N);
    cv.take(c.leaf_lev, N);
    cv.take(c.fs, N);
    // cells
    cv.take(c.c_level, ccap); cv.take(c.c_begin, ccap); cv.take(c.c_count, ccap);
    cv.take(c.c_first, ccap); cv.take(c.c_nchild, ccap); cv.take(c.c_parent, ccap);
    cv.take(c.c_prefix, ccap); cv.take(c.c_node, ccap); cv.take(c.c_link, ccap);
    cv.take(c.c_mom, 10 * (size_t)ccap);
    cv.take(c.c_lvl, kLevels + 2);
    cv.take(c.tmp_n, N + S + 1);
    cv.take(c.tmp_off, std::max(N + S + 2, tree_scratch_u32(N)));
    c.cell_cap = ccap;
    // groups
    cv.take(c.g_cell, gcap); cv.take(c.g_begin, gcap); cv.take(c.g_count, gcap);
    cv.take(c.g_sys, gcap); cv.take(c.g_box, 6 * (size_t)gcap);
    cv.take(c.g_centre, 3 * (size_t)gcap); cv.take(c.g_wide, gcap); cv.take(c.wide_list, gcap);
    cv.take(c.cnt_e, gcap); cv.take(c.cnt_s, gcap); cv.take(c.lcap, gcap);
    cv.take(c.seg, (size_t)gcap + 1); cv.take(c.ovf_list, gcap);
    // per-XCD queue runs of the persistent force kernel
    cv.take(c.f_cost, gcap); cv.take(c.f_pre, (size_t)gcap + 1); cv.take(c.f_bounds, 9);
    c.group_cap = gcap;
    // interaction lists: the rest of the array
    uint64_t list_room = 0;
    cv.rest(c.list, &list_room);
    c.list_cap = list_room;
    if (!cv.ok) {
        snprintf(msg, sizeof msg, "the scratch array (%zu bytes) cannot hold the buffers of "
                 "%lld particles", kScratchBytes, (long long)n);
        return out(FDX_ENOMEM);
    }
    // outputs: the caller's arrays
    c.ax.p = ax; c.ay.p = ay; c.az.p = az; c.pot.p = pot;
    c.ax.cap = c.ay.cap = c.az.cap = c.pot.cap = N;
    // every other buffer stays empty and fixed: growing one fails (FDX_ENOMEM) instead of
    // allocating
    c.each_buffer([](auto &b) { b.fixed = true; });

    const auto hip_fail = [&](hipError_t e, const char *what) {
        snprintf(msg, sizeof msg, "%s: %s", what, hipGetErrorString(e));
        return out(e == hipErrorOutOfMemory ? FDX_ENOMEM : FDX_EHIP);
    };
    hipError_t e = fill_u64(reinterpret_cast<uint64_t *>(c.sys_off.p), 0, 1, c.stream);
    if (e == hipSuccess) e = fill_u64(reinterpret_cast<uint64_t *>(c.sys_off.p) + 1, (uint64_t)n, 1,
                                      c.stream);
    if (e == hipSuccess) e = sysid_fill(c.sys_off.p, 1, c.sysid.p, N, c.stream);
    if (e != hipSuccess) return hip_fail(e, "set-up");
    c.have_particles = true;

    r = setup_eval(&c, theta, n_leaf, n_group, eps_all, flags);
    if (!r) r = run_tree(&c, true);
    if (!r) {
        const uint32_t G = c.hst->st.n_groups;
        r = enqueue_count(&c, G);
        if (!r) r = read_status(&c);
        if (!r && c.hst->st.walk_error) r = fail(&c, FDX_EHIP, "walk stack exhausted");
        if (!r && c.hst->st.list_total > c.list_cap)
            r = fail(&c, FDX_ENOMEM, "the interaction lists need %llu entries, the scratch "
                     "array has room for %llu", (unsigned long long)c.hst->st.list_total,
                     (unsigned long long)c.list_cap);
        if (!r) r = enqueue_fill(&c, G);
        if (!r) r = enqueue_force(&c, G);
        if (!r) r = read_status(&c);
        if (!r && status_incomplete(c.hst->st))
            r = fail(&c, FDX_EHIP, "the device reported an incomplete evaluation");
    }
    if (r) {
        if (r == FDX_ENOMEM && !strstr(c.err, "interaction lists"))
            snprintf(msg, sizeof msg, "the cells or groups do not fit the scratch array (%s)", c.err);
        else
            snprintf(msg, sizeof msg, "%s", c.err);
        return out(r);
    }
    return out(FDX_OK);
    FDX_ABI_CATCH(nullptr)
}

}  // extern "C"
