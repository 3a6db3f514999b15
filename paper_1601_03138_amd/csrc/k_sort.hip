// Stable LSD radix sort of (63-bit key, u32 index) pairs, then stably by system id, so the
// result is ordered by (system, key, original index).  8-bit digits; per pass: per-tile
// digit histograms, a device-wide exclusive scan over (digit, tile), and a scatter in which
// each wave ranks its elements with ballot-based multisplit so the order is stable, and the
// tile is reordered in LDS so each digit's run is written contiguously.  With several
// systems (at most 2^16) and a carry buffer, a 16-bit copy of each element's system id
// travels with it through the key passes, so the system-id passes read their digit in
// order instead of gathering it through the permutation.
#include "dev_util.h"
#include "fdx_internal.h"

namespace fdx {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / kWave;     // 4
constexpr int kItems = 8;                    // rounds of 64 per wave
constexpr int kWaveTile = kItems * kWave;    // 512 elements per wave
constexpr int kTile = kWaves * kWaveTile;    // 2048 elements per block
constexpr int kRadix = 256;

// digit source: the key, the system id gathered through the index, or the carried system id
enum { kDigitKey = 0, kDigitSysGather = 1, kDigitSysCarried = 2 };

template <int SRC>
__device__ __forceinline__ uint32_t digit_of(uint64_t k, uint32_t v, uint32_t sc,
                                             const uint32_t *sysid, int shift) {
    if (SRC == kDigitSysGather) return (sysid[v] >> shift) & (kRadix - 1);
    if (SRC == kDigitSysCarried) return (sc >> shift) & (kRadix - 1);
    return (uint32_t)(k >> shift) & (kRadix - 1);
}

template <int SRC>
__global__ void __launch_bounds__(kThreads)
k_rs_hist(const uint64_t *key, const uint32_t *val, const uint16_t *sc, const uint32_t *sysid,
          size_t n, int shift, uint32_t nblocks, uint32_t *counts) {
    __shared__ uint32_t h[kRadix];
    h[threadIdx.x] = 0;
    __syncthreads();
    const size_t base = (size_t)blockIdx.x * kTile;
#pragma unroll 4
    for (int r = 0; r < kTile / kThreads; r++) {
        size_t i = base + (size_t)r * kThreads + threadIdx.x;
        if (i < n) {
            uint32_t d;
            if (SRC == kDigitKey) d = digit_of<kDigitKey>(key[i], 0, 0, nullptr, shift);
            else if (SRC == kDigitSysGather) d = digit_of<SRC>(0, val[i], 0, sysid, shift);
            else d = digit_of<SRC>(0, 0, sc[i], nullptr, shift);
            atomicAdd(&h[d], 1u);
        }
    }
    __syncthreads();
    counts[(size_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Scatter of one tile: every element's rank among the tile's elements of its digit (ballot
// multisplit per wave, waves in order), the elements laid out in LDS in digit order, then
// each digit's run written to its global range with consecutive threads on consecutive
// addresses.  CARRY moves the 16-bit system ids along (sc_in -> sc_out).
template <int SRC, bool CARRY>
__global__ void __launch_bounds__(kThreads)
k_rs_scatter(const uint64_t *key_in, const uint32_t *val_in, const uint16_t *sc_in,
             const uint32_t *sysid, size_t n, int shift, uint32_t nblocks, const uint32_t *offs,
             uint64_t *key_out, uint32_t *val_out, uint16_t *sc_out) {
    static_assert(SRC != kDigitSysCarried || CARRY, "carried digits are staged with the carry");
    __shared__ uint64_t sk[kTile];
    __shared__ uint32_t sv[kTile];
    __shared__ uint16_t ss[CARRY ? kTile : 1];
    __shared__ uint32_t wcnt[kWaves][kRadix];     // per wave and digit: count, then offset
    __shared__ uint32_t lstart[kRadix];           // first LDS slot of each digit
    __shared__ uint32_t gstart[kRadix];           // global position of that slot
    __shared__ uint64_t scan_tmp[kWaves];
    for (int k = threadIdx.x; k < kWaves * kRadix; k += kThreads) (&wcnt[0][0])[k] = 0;
    __syncthreads();
    const int w = threadIdx.x / kWave, lane = lane_id();
    const uint64_t lt = lanemask_lt();
    const size_t base = (size_t)blockIdx.x * kTile + (size_t)w * kWaveTile;
    uint64_t kk[kItems];
    uint32_t vv[kItems], rk[kItems], cc[kItems];
#pragma unroll
    for (int r = 0; r < kItems; r++) {
        const size_t i = base + (size_t)r * kWave + lane;
        const bool valid = i < n;
        uint64_t k = 0;
        uint32_t v = 0, d = 0, c = 0;
        if (valid) {
            k = key_in[i];
            v = val_in[i];
            if (CARRY || SRC == kDigitSysCarried) c = sc_in[i];
            d = digit_of<SRC>(k, v, c, sysid, shift);
        }
        uint64_t m = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            uint64_t bal = __ballot((d >> b) & 1u);
            m &= ((d >> b) & 1u) ? bal : ~bal;
        }
        const uint32_t before = (uint32_t)__popcll(m & lt);
        const uint32_t cnt = (uint32_t)__popcll(m);
        const uint32_t prev = valid ? wcnt[w][d] : 0u;
        wave_barrier();
        if (valid && before == 0) wcnt[w][d] = prev + cnt;
        wave_barrier();
        kk[r] = k;
        vv[r] = v;
        cc[r] = c;
        rk[r] = valid ? (d << 16) | (prev + before) : 0xFFFFFFFFu;
    }
    __syncthreads();
    {
        const int d = threadIdx.x;                 // kThreads == kRadix
        uint32_t tot = 0;
#pragma unroll
        for (int ww = 0; ww < kWaves; ww++) {
            const uint32_t c = wcnt[ww][d];
            wcnt[ww][d] = tot;
            tot += c;
        }
        uint64_t btot;
        lstart[d] = (uint32_t)block_excl_scan<kThreads>(tot, scan_tmp, &btot);
        gstart[d] = offs[(size_t)d * nblocks + blockIdx.x];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kItems; r++) {
        if (rk[r] != 0xFFFFFFFFu) {
            const uint32_t d = rk[r] >> 16;
            const uint32_t slot = lstart[d] + wcnt[w][d] + (rk[r] & 0xFFFFu);
            sk[slot] = kk[r];
            sv[slot] = vv[r];
            if (CARRY) ss[slot] = (uint16_t)cc[r];
        }
    }
    __syncthreads();
    const size_t b0 = (size_t)blockIdx.x * kTile;
    const uint32_t cnt = (uint32_t)min((size_t)kTile, n - b0);
    for (uint32_t j = threadIdx.x; j < cnt; j += kThreads) {
        const uint64_t k = sk[j];
        const uint32_t v = sv[j];
        const uint32_t c = CARRY ? (uint32_t)ss[j] : 0u;
        const uint32_t d = digit_of<SRC>(k, v, c, sysid, shift);
        const uint32_t pos = gstart[d] + (j - lstart[d]);
        key_out[pos] = k;
        val_out[pos] = v;
        if (CARRY) sc_out[pos] = (uint16_t)c;
    }
}

static_assert(kThreads == kRadix, "one thread per digit in the offset step");

}  // namespace

size_t radix_scratch_u32(size_t n) {
    size_t nblocks = (n + kTile - 1) / kTile;
    if (nblocks < 1) nblocks = 1;
    return 2 * (size_t)kRadix * nblocks;      // counts + scanned offsets
}

// 16-bit system ids in input order (the carry's starting copy)
__global__ void k_carry_init(size_t n, const uint32_t *sysid, uint16_t *sc) {
    for (size_t i = gtid(); i < n; i += gstride()) sc[i] = (uint16_t)sysid[i];
}

template <int SRC, bool CARRY>
static void rs_pass(uint32_t nblocks, hipStream_t s, const uint64_t *kin, const uint32_t *vin,
                    const uint16_t *cin, const uint32_t *sysid, size_t n, int shift,
                    uint32_t *counts, const uint32_t *offs, uint64_t *kout, uint32_t *vout,
                    uint16_t *cout, bool hist) {
    if (hist)
        hipLaunchKernelGGL(k_rs_hist<SRC>, dim3(nblocks), dim3(kThreads), 0, s, kin, vin, cin,
                           sysid, n, shift, nblocks, counts);
    else
        hipLaunchKernelGGL((k_rs_scatter<SRC, CARRY>), dim3(nblocks), dim3(kThreads), 0, s, kin,
                           vin, cin, sysid, n, shift, nblocks, offs, kout, vout, cout);
}

hipError_t radix_sort(size_t n, uint64_t *key, uint64_t *key_alt, uint32_t *val,
                      uint32_t *val_alt, const uint32_t *sysid, int nsys, int key_bits,
                      uint32_t *scratch, uint64_t *partial, bool *result_in_alt, hipStream_t s,
                      uint16_t *carry) {
    *result_in_alt = false;
    if (n <= 1) return hipSuccess;
    const uint32_t nblocks = (uint32_t)((n + kTile - 1) / kTile);
    const size_t ncount = (size_t)kRadix * nblocks;
    uint32_t *counts = scratch, *offs = scratch + ncount;
    uint64_t *kin = key, *kout = key_alt;
    uint32_t *vin = val, *vout = val_alt;
    int sys_passes = 0;
    for (int b = 0; (1ll << b) < (long long)nsys; b += 8) sys_passes++;
    const int key_passes = (key_bits + 7) / 8;
    const int passes = key_passes + sys_passes;  // key bytes, then system id bytes
    const bool carried = sys_passes > 0 && carry && nsys <= 65536;
    uint16_t *cin = carried ? carry : nullptr, *cout = carried ? carry + n : nullptr;
    if (carried) {
        const size_t b = (n + kThreads - 1) / kThreads;
        hipLaunchKernelGGL(k_carry_init, dim3((unsigned)(b < 16384 ? b : 16384)), dim3(kThreads),
                           0, s, n, sysid, cin);
    }
    for (int p = 0; p < passes; p++) {
        const bool sysp = p >= key_passes;
        const int shift = sysp ? 8 * (p - key_passes) : 8 * p;
        for (int phase = 0; phase < 2; phase++) {
            const bool hist = phase == 0;
            if (!sysp && carried)
                rs_pass<kDigitKey, true>(nblocks, s, kin, vin, cin, sysid, n, shift, counts, offs,
                                         kout, vout, cout, hist);
            else if (!sysp)
                rs_pass<kDigitKey, false>(nblocks, s, kin, vin, cin, sysid, n, shift, counts,
                                          offs, kout, vout, cout, hist);
            else if (carried)
                rs_pass<kDigitSysCarried, true>(nblocks, s, kin, vin, cin, sysid, n, shift,
                                                counts, offs, kout, vout, cout, hist);
            else
                rs_pass<kDigitSysGather, false>(nblocks, s, kin, vin, cin, sysid, n, shift,
                                                counts, offs, kout, vout, cout, hist);
            if (hist) {
                hipError_t e = scan_u32_to_u32(counts, offs, ncount, nullptr, nullptr, partial,
                                               nullptr, s);
                if (e != hipSuccess) return e;
            }
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        uint64_t *tk = kin; kin = kout; kout = tk;
        uint32_t *tv = vin; vin = vout; vout = tv;
        uint16_t *tc = cin; cin = cout; cout = tc;
    }
    *result_in_alt = (kin == key_alt);
    return hipSuccess;
}

}  // namespace fdx
