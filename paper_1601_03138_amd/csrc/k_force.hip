// Particle-particle and particle-superparticle force kernels over the shared group lists.
//
// The paper asks for an interaction routine that takes many i-particles and many
// j-particles at once so each j is reused from fast memory (section "Design concept of
// FDPS"), with particles (EPJ) and superparticles (SPJ) as two sums (equation geqL).  Here
// one workgroup evaluates one group: j entries are gathered tile by tile into LDS, JT entries
// per tile (JT <= NT; with PF the next tile's global loads are issued before the current tile
// is computed), and thread t owns IPL i-particles and one slice of every tile.  The group's n_i particles map onto
// tps = ceil(n_i / IPL) threads per slice and floor(NT / tps) slices, so nearly all lanes
// carry a real i-particle whatever n_i is.  Slices are combined at the end in slice order,
// so the result is deterministic.
//
// Particle term (equation ParticleParticleNbody, G = 1):
//   a_i += m_j (r_j - r_i) / (|r_j - r_i|^2 + eps_i^2)^{3/2},  phi_i -= m_j / (...)^{1/2}
// Superparticle term (equation ParticleSuperparticleNbody with the superparticle at r'_j,
// extended to the quadrupole; r = r_i - X, R^2 = |r|^2 + eps_i^2):
//   phi_i -= M/R + (1/2) r.Q.r / R^5
//   a_i   += -M r / R^3 + Q r / R^5 - (5/2) (r.Q.r) r / R^7
// Each group's own particles are in its particle list (its leaves are always opened), so
// the self pair adds exactly 0 to a_i (r = 0) and -m_i/eps_i to phi_i, which is removed after
// the loop.
//
// FP32 variant: positions are taken relative to the centre of the group's cell in FP64 and
// rounded to FP32 when a tile is staged; the inner loop is FP32 (hardware reciprocal square
// root); each slice sums a tile plainly and adds the tile total into a Kahan-compensated
// accumulator; outputs are FP64.
// FP64 variant: the same loop in FP64; 1/sqrt from the hardware estimate refined by one
// Newton-Raphson step.
#include "dev_util.h"
#include "fdx_internal.h"
#include "interact.h"

namespace fdx {

namespace {

struct KArgs {
    const uint32_t *gbegin, *gcount;
    const double *gcentre;
    const double4 *jp;
    const double *seps;
    const double *mom;
    const uint64_t *seg;
    const uint32_t *cap, *cnt_e, *cnt_s, *list;
    const uint32_t *order;
    const uint32_t *bounds;  // persistent: per-XCD runs [bounds[x], bounds[x+1]) (or null)
    const uint32_t *ngroups;
    double4 *fs;
    DevStatus *st;
    uint32_t G;              // groups (direct launch); persistent kernels read *ngroups
    double cut_s;            // cutoff kernel: 2 / r_cut
};

// Kahan accumulator (FP32) or plain sum (FP64)
template <class T> struct Acc {
    T s = 0;
    __device__ __forceinline__ void add(T v) { s += v; }
    __device__ __forceinline__ double val() const { return (double)s; }
};
template <> struct Acc<float> {
    float s = 0.f, c = 0.f;
    __device__ __forceinline__ void add(float v) {
        float y = v - c;
        float t = s + y;
        c = (t - s) - y;
        s = t;
    }
    __device__ __forceinline__ double val() const { return (double)s - (double)c; }
};

template <class T, int NT, int IPL, int JT>
struct Smem {
    using V = typename V4<T>::t;
    union {
        V e[JT];                        // particle tile
        V s[3 * JT];                    // superparticle tile (A, B, C per entry)
        double red[NT * IPL * 4];       // per-thread slice partials
    };
    uint32_t slot;
};

template <class T, bool QUAD, int NT, int IPL, bool PF, bool CUT, int JT>
__device__ __forceinline__ void force_group(const KArgs &a, uint32_t gi, Smem<T, NT, IPL, JT> &sm) {
    static_assert(JT <= NT && NT % JT == 0, "a tile holds at most one entry per thread");
    using V = typename V4<T>::t;
    const int tid = threadIdx.x;
    // the group's values are the same in every lane: held in scalar registers
    gi = uniform_u32(gi);
    const uint32_t gb = uniform_u32(a.gbegin[gi]), ni = uniform_u32(a.gcount[gi]);
    const uint32_t ne = uniform_u32(a.cnt_e[gi]), ns = uniform_u32(a.cnt_s[gi]);
    const uint32_t capg = uniform_u32(a.cap[gi]);
    const uint32_t *epj = a.list + uniform_u64(a.seg[gi]);
    const uint32_t *spj = epj + capg - ns;
    const bool fp32 = sizeof(T) == 4;
    const double cx = fp32 ? uniform_f64(a.gcentre[3 * gi]) : 0.0;
    const double cy = fp32 ? uniform_f64(a.gcentre[3 * gi + 1]) : 0.0;
    const double cz = fp32 ? uniform_f64(a.gcentre[3 * gi + 2]) : 0.0;
    const T cut_s = (T)a.cut_s;

    uint32_t tps = (ni + IPL - 1) / IPL;
    tps = tps < 1 ? 1 : (tps > (uint32_t)NT ? (uint32_t)NT : tps);
    const uint32_t nslice = NT / tps;
    const uint32_t slice = tid / tps, li = tid % tps;
    const bool active = slice < nslice;

    T xi[IPL], yi[IPL], zi[IPL], e2[IPL];
    Acc<T> ax[IPL], ay[IPL], az[IPL], ph[IPL];
#pragma unroll
    for (int k = 0; k < IPL; k++) {
        const uint32_t i = li + k * tps;
        const uint32_t r = gb + (i < ni ? i : 0);
        const double4 p = a.jp[r];
        xi[k] = (T)(p.x - cx); yi[k] = (T)(p.y - cy); zi[k] = (T)(p.z - cz);
        const double e = a.seps[r];
        e2[k] = (T)(e * e);
    }

    // particle tiles: one entry per thread per tile (PF: the next tile is loaded into
    // registers while the current one is computed)
    {
        double4 nxt = make_double4(0, 0, 0, 0);
        if (PF && (uint32_t)tid < min((uint32_t)JT, ne)) nxt = a.jp[epj[tid]];
        for (uint32_t t0 = 0; t0 < ne; t0 += JT) {
            const uint32_t nt = min((uint32_t)JT, ne - t0);
            __syncthreads();
            if ((uint32_t)tid < nt) {
                if (!PF) nxt = a.jp[epj[t0 + tid]];
                V v;
                v.x = (T)(nxt.x - cx); v.y = (T)(nxt.y - cy); v.z = (T)(nxt.z - cz); v.w = (T)nxt.w;
                sm.e[tid] = v;
            }
            __syncthreads();
            if (PF && tid < JT && t0 + JT + tid < ne) nxt = a.jp[epj[t0 + JT + tid]];
            if (active) {
                T tx[IPL], ty[IPL], tz[IPL], tp[IPL];
#pragma unroll
                for (int k = 0; k < IPL; k++) tx[k] = ty[k] = tz[k] = tp[k] = 0;
                // a contiguous run of kmain entries per slice (block-uniform trip count,
                // constant LDS stride), then the nt mod nslice leftover entries one per slice
                const uint32_t kmain = nt / nslice;
                const V *run = sm.e + slice * kmain;
                // FP32 with two i-particles per lane: those already give two independent
                // chains; unrolled 4 (and the superparticle loop 2) the kernel held 98 VGPRs,
                // 2 and 1 hold 72 (6 waves per SIMD instead of 4)
#pragma unroll (IPL == 2 && sizeof(T) == 4 ? 2 : 4)
                for (uint32_t q = 0; q < kmain; q++) {
                    const V J = run[q];
#pragma unroll
                    for (int k = 0; k < IPL; k++)
                        pp<T, CUT>(J, xi[k], yi[k], zi[k], e2[k], tx[k], ty[k], tz[k], tp[k], cut_s);
                }
                const uint32_t j = kmain * nslice + slice;
                if (j < nt) {
                    const V J = sm.e[j];
#pragma unroll
                    for (int k = 0; k < IPL; k++)
                        pp<T, CUT>(J, xi[k], yi[k], zi[k], e2[k], tx[k], ty[k], tz[k], tp[k], cut_s);
                }
#pragma unroll
                for (int k = 0; k < IPL; k++) {
                    ax[k].add(tx[k]); ay[k].add(ty[k]); az[k].add(tz[k]); ph[k].add(tp[k]);
                }
            }
        }
    }

    // superparticle tiles
    {
        const double *o = nullptr;
        double m0 = 0, m1 = 0, m2 = 0, m3 = 0, q0 = 0, q1 = 0, q2 = 0, q3 = 0, q4 = 0, q5 = 0;
        auto fetch = [&](uint32_t k) {
            o = a.mom + 10 * (size_t)spj[k];
            m0 = o[0]; m1 = o[1]; m2 = o[2]; m3 = o[3];
            if (QUAD) { q0 = o[4]; q1 = o[5]; q2 = o[6]; q3 = o[7]; q4 = o[8]; q5 = o[9]; }
        };
        if (PF && (uint32_t)tid < min((uint32_t)JT, ns)) fetch(tid);
        for (uint32_t t0 = 0; t0 < ns; t0 += JT) {
            const uint32_t nt = min((uint32_t)JT, ns - t0);
            __syncthreads();
            if ((uint32_t)tid < nt) {
                if (!PF) fetch(t0 + tid);
                V A;
                A.x = (T)(m1 - cx); A.y = (T)(m2 - cy); A.z = (T)(m3 - cz); A.w = (T)m0;
                sm.s[3 * tid] = A;
                if (QUAD) {
                    V B, C;
                    B.x = (T)q0; B.y = (T)q1; B.z = (T)q2; B.w = (T)q3;
                    C.x = (T)q4; C.y = (T)q5; C.z = 0; C.w = 0;
                    sm.s[3 * tid + 1] = B;
                    sm.s[3 * tid + 2] = C;
                }
            }
            __syncthreads();
            if (PF && tid < JT && t0 + JT + tid < ns) fetch(t0 + JT + tid);
            if (active) {
                T tx[IPL], ty[IPL], tz[IPL], tp[IPL];
#pragma unroll
                for (int k = 0; k < IPL; k++) tx[k] = ty[k] = tz[k] = tp[k] = 0;
                const uint32_t kmain = nt / nslice;
                const V *run = sm.s + 3 * slice * kmain;
                // (FP32, two i-particles per lane: not unrolled, as above)
#pragma unroll (IPL == 2 && sizeof(T) == 4 ? 1 : 2)
                for (uint32_t q = 0; q < kmain; q++) {
                    const V A = run[3 * q];
                    V B, C;
                    if (QUAD) { B = run[3 * q + 1]; C = run[3 * q + 2]; } else { B = A; C = A; }
#pragma unroll
                    for (int k = 0; k < IPL; k++)
                        pc<T, QUAD, CUT>(A, B, C, xi[k], yi[k], zi[k], e2[k], tx[k], ty[k], tz[k], tp[k],
                                         cut_s);
                }
                const uint32_t j = kmain * nslice + slice;
                if (j < nt) {
                    const V A = sm.s[3 * j];
                    V B, C;
                    if (QUAD) { B = sm.s[3 * j + 1]; C = sm.s[3 * j + 2]; } else { B = A; C = A; }
#pragma unroll
                    for (int k = 0; k < IPL; k++)
                        pc<T, QUAD, CUT>(A, B, C, xi[k], yi[k], zi[k], e2[k], tx[k], ty[k], tz[k], tp[k],
                                         cut_s);
                }
#pragma unroll
                for (int k = 0; k < IPL; k++) {
                    ax[k].add(tx[k]); ay[k].add(ty[k]); az[k].add(tz[k]); ph[k].add(tp[k]);
                }
            }
        }
    }

    // combine slices in slice order (FP64), remove the self term of the potential
    __syncthreads();
    if (active) {
#pragma unroll
        for (int k = 0; k < IPL; k++) {
            double *o = sm.red + 4 * ((size_t)k * NT + tid);
            // slice 0 carries the potential's self term (added first, in FP64); only slots
            // that hold a particle of the group read its mass (a slot past n_i does not)
            const uint32_t i = li + k * tps;
            double self = 0.0;
            if (!CUT && slice == 0 && i < ni) self = (double)((T)a.jp[gb + i].w * rsqrt_t(e2[k]));
            o[0] = ax[k].val(); o[1] = ay[k].val(); o[2] = az[k].val(); o[3] = self + ph[k].val();
        }
    }
    __syncthreads();
    // one thread per (component, i-particle slot) sums that component over the slices in
    // slice order -- the same order for every launch shape that shares tps -- so a small
    // group's many slices are combined by 4 x tps threads instead of tps
#pragma unroll 1
    for (uint32_t t = (uint32_t)tid; t < 4u * IPL * tps; t += NT) {
        const uint32_t c = t & 3u, slot = t >> 2;
        const uint32_t k = IPL == 1 ? 0u : slot / tps, lk = slot - k * tps;
        const uint32_t i = lk + k * tps;
        if (i >= ni) continue;
        double v = 0;
        const double *o = sm.red + 4 * ((size_t)k * NT + lk) + c;
#pragma unroll 1
        for (uint32_t q = 0; q < nslice; q++) v += o[4 * (size_t)q * tps];
        const uint32_t r = gb + i;
        reinterpret_cast<double *>(a.fs + r)[c] = (CUT && c == 3) ? 0.0 : v;
    }
    __syncthreads();
}

// OCC: minimum waves per SIMD the register allocation must allow (1 = no constraint).
template <class T, bool QUAD, int NT, int IPL, bool PF, int OCC, bool CUT, int JT>
__global__ void __launch_bounds__(NT, OCC)
k_force_direct(KArgs a) {
    __shared__ Smem<T, NT, IPL, JT> sm;
    // XCD-aware order: consecutive blocks go round-robin over the 8 XCDs, so hand each XCD a
    // contiguous run of groups (neighbouring groups share most of their lists -> L2 reuse).
    const uint32_t G = a.G;
    const uint32_t chunk = (G + 7) / 8;
    const uint32_t q = (blockIdx.x % 8) * chunk + blockIdx.x / 8;
    if (q >= G) return;
    force_group<T, QUAD, NT, IPL, PF, CUT, JT>(a, a.order ? a.order[q] : q, sm);
}

// Persistent variant: a fixed grid pops work from device counters.  Without an explicit list
// the groups are split into eight contiguous runs in tree order (at equal cumulative cost when
// bounds are given, else of equal group counts), one queue per XCD
// (consecutive workgroups are dispatched round-robin over the 8 XCDs, so workgroup b runs on
// XCD b % 8); a workgroup pops from its own XCD's queue, keeping neighbouring groups -- which
// share most of their lists -- in one L2, and once that queue is empty takes slots from the
// other XCDs' queues, which balances the load.  With an explicit list (order + device count)
// it pops one shared queue.
template <class T, bool QUAD, int NT, int IPL, bool PF, int OCC, bool CUT, int JT>
__global__ void __launch_bounds__(NT, OCC)
k_force_persistent(KArgs a) {
    __shared__ Smem<T, NT, IPL, JT> sm;
    const uint32_t G = *a.ngroups;
    const uint32_t x = blockIdx.x % 8u, chunk = (G + 7u) / 8u;
    for (;;) {
        if (threadIdx.x == 0) {
            uint32_t slot = kNone;
            if (a.order) {
                slot = atomicAdd(&a.st->queue_head, 1u);
            } else {
                for (uint32_t t = 0; t < 8u && slot == kNone; t++) {
                    const uint32_t q = (x + t) & 7u;
                    const uint32_t lo = a.bounds ? a.bounds[q] : q * chunk;
                    const uint32_t hi = a.bounds ? a.bounds[q + 1] : min(G, lo + chunk);
                    if (lo >= hi) continue;
                    const uint32_t k = atomicAdd(&a.st->xcd_head[q], 1u);
                    if (k < hi - lo) slot = lo + k;
                }
            }
            sm.slot = slot;
        }
        __syncthreads();
        const uint32_t slot = sm.slot;
        __syncthreads();
        if (slot >= G) break;
        force_group<T, QUAD, NT, IPL, PF, CUT, JT>(a, a.order ? a.order[slot] : slot, sm);
    }
}

template <class T, bool QUAD, int NT, int IPL, bool PF, int OCC = 1, bool CUT = false, int JT = NT>
hipError_t launch(const KArgs &k, bool persistent, hipStream_t s) {
    if (persistent) {
        int dev = 0, ncu = 256;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
        int per_cu = 0;
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void *>(k_force_persistent<T, QUAD, NT, IPL, PF, OCC, CUT, JT>), NT, 0);
        if (per_cu < 1) per_cu = 1;
        size_t grid = (size_t)ncu * per_cu;
        if (k.G && grid > k.G) grid = k.G;
        hipLaunchKernelGGL((k_force_persistent<T, QUAD, NT, IPL, PF, OCC, CUT, JT>), dim3((unsigned)grid), dim3(NT),
                           0, s, k);
    } else {
        if (k.G == 0) return hipSuccess;
        const uint32_t chunk = (k.G + 7) / 8;
        hipLaunchKernelGGL((k_force_direct<T, QUAD, NT, IPL, PF, OCC, CUT, JT>), dim3(8 * chunk), dim3(NT), 0, s, k);
    }
    return hipGetLastError();
}

struct Variant { int nt, ipl; bool pf; const char *name; };
// the j-tile equals the workgroup size unless the name says otherwise (_jtN: N entries per tile)
constexpr Variant kVariants[] = {
    {256, 1, true, "nt256_ipl1_pf"}, {256, 2, true, "nt256_ipl2_pf"},
    {512, 1, true, "nt512_ipl1_pf"}, {512, 2, true, "nt512_ipl2_pf"},
    {256, 1, false, "nt256_ipl1"},   {256, 2, false, "nt256_ipl2"},
    {512, 1, false, "nt512_ipl1"},   {512, 2, false, "nt512_ipl2"},
    {512, 1, true, "nt512_ipl1_pf_w8"}, {512, 1, false, "nt512_ipl1_w8"},
    {256, 1, false, "nt256_ipl1_jt64"}, {256, 1, false, "nt256_ipl1_jt128"},
    {512, 1, false, "nt512_ipl1_w8_jt128"}, {512, 1, false, "nt512_ipl1_w8_jt256"}};
constexpr int kNumVariants = 14;

// FP32: register allocation held to 64 VGPRs, 8 waves per SIMD (4 workgroups per CU)
template <class T> constexpr int kW8 = sizeof(T) == 4 ? 8 : 1;

template <class T, bool QUAD>
hipError_t launch_v(const KArgs &k, bool persistent, int v, hipStream_t s) {
    switch (v) {
        case 0: return launch<T, QUAD, 256, 1, true>(k, persistent, s);
        case 1: return launch<T, QUAD, 256, 2, true>(k, persistent, s);
        case 2: return launch<T, QUAD, 512, 1, true>(k, persistent, s);
        case 3: return launch<T, QUAD, 512, 2, true>(k, persistent, s);
        case 4: return launch<T, QUAD, 256, 1, false>(k, persistent, s);
        case 5: return launch<T, QUAD, 256, 2, false>(k, persistent, s);
        case 6: return launch<T, QUAD, 512, 1, false>(k, persistent, s);
        case 7: return launch<T, QUAD, 512, 2, false>(k, persistent, s);
        case 8: return launch<T, QUAD, 512, 1, true, kW8<T>>(k, persistent, s);
        case 9: return launch<T, QUAD, 512, 1, false, kW8<T>>(k, persistent, s);
        case 10: return launch<T, QUAD, 256, 1, false, 1, false, 64>(k, persistent, s);
        case 11: return launch<T, QUAD, 256, 1, false, 1, false, 128>(k, persistent, s);
        case 12: return launch<T, QUAD, 512, 1, false, kW8<T>, false, 128>(k, persistent, s);
        default: return launch<T, QUAD, 512, 1, false, kW8<T>, false, 256>(k, persistent, s);
    }
}

// private (scratch) bytes per lane of one kernel instance: > 0 means registers spill
template <class T, bool QUAD, int NT, int IPL, bool PF, int OCC = 1, int JT = NT>
int scratch_of(bool persistent) {
    hipFuncAttributes at{};
    const void *f = persistent
        ? reinterpret_cast<const void *>(k_force_persistent<T, QUAD, NT, IPL, PF, OCC, false, JT>)
        : reinterpret_cast<const void *>(k_force_direct<T, QUAD, NT, IPL, PF, OCC, false, JT>);
    if (hipFuncGetAttributes(&at, f) != hipSuccess) return -1;
    return (int)at.localSizeBytes;
}

template <class T, bool QUAD>
int scratch_v(bool persistent, int v) {
    switch (v) {
        case 0: return scratch_of<T, QUAD, 256, 1, true>(persistent);
        case 1: return scratch_of<T, QUAD, 256, 2, true>(persistent);
        case 2: return scratch_of<T, QUAD, 512, 1, true>(persistent);
        case 3: return scratch_of<T, QUAD, 512, 2, true>(persistent);
        case 4: return scratch_of<T, QUAD, 256, 1, false>(persistent);
        case 5: return scratch_of<T, QUAD, 256, 2, false>(persistent);
        case 6: return scratch_of<T, QUAD, 512, 1, false>(persistent);
        case 7: return scratch_of<T, QUAD, 512, 2, false>(persistent);
        case 8: return scratch_of<T, QUAD, 512, 1, true, kW8<T>>(persistent);
        case 9: return scratch_of<T, QUAD, 512, 1, false, kW8<T>>(persistent);
        case 10: return scratch_of<T, QUAD, 256, 1, false, 1, 64>(persistent);
        case 11: return scratch_of<T, QUAD, 256, 1, false, 1, 128>(persistent);
        case 12: return scratch_of<T, QUAD, 512, 1, false, kW8<T>, 128>(persistent);
        default: return scratch_of<T, QUAD, 512, 1, false, kW8<T>, 256>(persistent);
    }
}

}  // namespace

int force_variant_scratch(bool fp32, bool quad, bool persistent, int v) {
    if (v < 0 || v >= kNumVariants) return -1;
    if (fp32) return quad ? scratch_v<float, true>(persistent, v) : scratch_v<float, false>(persistent, v);
    return quad ? scratch_v<double, true>(persistent, v) : scratch_v<double, false>(persistent, v);
}

int force_variants() { return kNumVariants; }
const char *force_variant_name(int v) {
    return kVariants[v < 0 || v >= kNumVariants ? 0 : v].name;
}
int force_variant_capacity(int v) {
    const Variant &x = kVariants[v < 0 || v >= kNumVariants ? 0 : v];
    return x.nt * x.ipl;
}

hipError_t force(size_t G, const ForceArgs &fa, hipStream_t s) {
    KArgs k;
    k.gbegin = fa.g->begin; k.gcount = fa.g->count; k.gcentre = fa.g->centre;
    k.jp = fa.jp; k.seps = fa.seps; k.mom = fa.mom;
    k.seg = fa.seg; k.cap = fa.cap; k.cnt_e = fa.cnt_e; k.cnt_s = fa.cnt_s;
    k.list = fa.list;
    k.order = fa.order; k.bounds = fa.bounds;
    k.ngroups = fa.count ? fa.count : &fa.st->n_groups_c;
    k.fs = fa.fs; k.st = fa.st;
    k.G = (uint32_t)G;
    k.cut_s = fa.r_cut > 0 ? 2.0 / fa.r_cut : 0.0;
    if (fa.r_cut > 0) {                // tree part of TreePM: monopole with the S2 cutoff
        if (!fa.fp32) return launch<double, false, 256, 2, false, 1, true>(k, fa.persistent, s);
        // the persistent loop holds the 64-register budget only without the register prefetch
        return fa.persistent ? launch<float, false, 512, 1, false, 8, true>(k, true, s)
                             : launch<float, false, 512, 1, true, 8, true>(k, false, s);
    }
    const int v = fa.variant;
    if (fa.fp32) return fa.quad ? launch_v<float, true>(k, fa.persistent, v, s)
                                : launch_v<float, false>(k, fa.persistent, v, s);
    return fa.quad ? launch_v<double, true>(k, fa.persistent, v, s)
                   : launch_v<double, false>(k, fa.persistent, v, s);
}

}  // namespace fdx
