// Device-side helpers shared by the gfx950 kernels (wave64 primitives, key bit tricks).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fdx {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
    return (1ull << lane_id()) - 1ull;
}

// Order-preserving map of an FP64 value to u64 (so min/max reduce to integer atomics).
__device__ __forceinline__ uint64_t dbl_to_ord(double d) {
    uint64_t b = (uint64_t)__double_as_longlong(d);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double ord_to_dbl(uint64_t u) {
    uint64_t b = (u >> 63) ? (u & 0x7FFFFFFFFFFFFFFFull) : ~u;
    return __longlong_as_double((long long)b);
}

// Spread the low 21 bits of v so that bit b lands on bit 3b.
__device__ __forceinline__ uint64_t spread3(uint64_t v) {
    v &= 0x1FFFFFull;
    v = (v | (v << 32)) & 0x1F00000000FFFFull;
    v = (v | (v << 16)) & 0x1F0000FF0000FFull;
    v = (v | (v << 8)) & 0x100F00F00F00F00Full;
    v = (v | (v << 4)) & 0x10C30C30C30C30C3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}
// Inverse of spread3: gather bits 0, 3, 6, ... into the low 21 bits.
__device__ __forceinline__ uint32_t compact3(uint64_t v) {
    v &= 0x1249249249249249ull;
    v = (v ^ (v >> 2)) & 0x10C30C30C30C30C3ull;
    v = (v ^ (v >> 4)) & 0x100F00F00F00F00Full;
    v = (v ^ (v >> 8)) & 0x1F0000FF0000FFull;
    v = (v ^ (v >> 16)) & 0x1F00000000FFFFull;
    v = (v ^ (v >> 32)) & 0x1FFFFFull;
    return (uint32_t)v;
}

// Inclusive prefix sum over the 64 lanes of a wave.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    const int l = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint32_t t = __shfl_up(v, d, kWave);
        if (l >= d) v += t;
    }
    return v;
}

// Exclusive prefix sum over the wave of small non-negative counts, one bit plane at a time:
// prefix = sum_b 2^b * (number of lower lanes with bit b set), from a ballot per bit and
// mbcnt (no cross-lane data movement).  *total receives the wave total.  Loops only over the
// bit planes in use, so counts below 16 cost four ballots.
__device__ __forceinline__ uint32_t wave_excl_scan_small(uint32_t v, uint32_t *total) {
    uint32_t pre = 0, tot = 0;
    for (int b = 0; b < 32; b++) {
        if (!__ballot((v >> b) != 0u)) break;
        const uint64_t m = __ballot((v >> b) & 1u);
        const uint32_t below = __builtin_amdgcn_mbcnt_hi(
            (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        pre += below << b;
        tot += (uint32_t)__popcll(m) << b;
    }
    *total = tot;
    return pre;
}

// Inclusive prefix sum over the 64 lanes with DPP lane moves (all lanes must be active):
// shifts by 1, 2, 4, 8 within each row of 16 lanes (lanes shifted in from outside the row
// read 0), then row 15's total added to rows 1 and 3 (row_bcast:15) and lane 31's to rows 2
// and 3 (row_bcast:31).
__device__ __forceinline__ uint32_t wave_incl_scan_dpp(uint32_t x) {
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false);   // row_shr:1
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false);   // row_shr:2
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false);   // row_shr:4
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false);   // row_shr:8
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);   // row_bcast:15
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);   // row_bcast:31
    return x;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

// Minimum / maximum over the 64 lanes, returned to every lane (all lanes must be active): the
// lane moves of wave_incl_scan_dpp with min / max in place of the sum (lanes shifted in from
// outside a row, and the rows a broadcast skips, read the operation's identity), after which
// lane 63 holds the result.
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t x) {
    constexpr int id = -1;                                                          // 0xFFFFFFFF
    x = min(x, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)x, 0x111, 0xf, 0xf, false));
    x = min(x, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)x, 0x112, 0xf, 0xf, false));
    x = min(x, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)x, 0x114, 0xf, 0xf, false));
    x = min(x, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)x, 0x118, 0xf, 0xf, false));
    x = min(x, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)x, 0x142, 0xa, 0xf, false));
    x = min(x, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)x, 0x143, 0xc, 0xf, false));
    return (uint32_t)__builtin_amdgcn_readlane((int)x, kWave - 1);
}
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t x) {
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false));
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false));
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false));
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false));
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false));
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false));
    return (uint32_t)__builtin_amdgcn_readlane((int)x, kWave - 1);
}
// Minimum / maximum over each 16-lane row, held by the row's last lane (lanes 15, 31, 47, 63;
// the other lanes hold prefix results): the four row_shr moves of wave_min_u32 / wave_max_u32
// without the broadcasts across rows.  All lanes must be active.
__device__ __forceinline__ uint32_t row_min_u32(uint32_t x) {
    constexpr int id = -1;
    x = min(x, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)x, 0x111, 0xf, 0xf, false));
    x = min(x, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)x, 0x112, 0xf, 0xf, false));
    x = min(x, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)x, 0x114, 0xf, 0xf, false));
    x = min(x, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)x, 0x118, 0xf, 0xf, false));
    return x;
}
__device__ __forceinline__ uint32_t row_max_u32(uint32_t x) {
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false));
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false));
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false));
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false));
    return x;
}
// one DPP lane move of a 64-bit value (both halves from the same lane; identity all ones)
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint64_t dpp_move_u64_max_id(uint64_t u) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)(uint32_t)u, CTRL,
                                                              ROW_MASK, 0xf, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)(uint32_t)(u >> 32), CTRL,
                                                              ROW_MASK, 0xf, false);
    return (uint64_t)lo | ((uint64_t)hi << 32);
}
// minimum of non-negative doubles (or +inf) over the 64 lanes, as wave_min_u32 on the bit
// patterns (ordered like the values for non-negative doubles)
__device__ __forceinline__ double wave_min_nonneg_f64(double v) {
    uint64_t u = (uint64_t)__double_as_longlong(v), o;
    o = dpp_move_u64_max_id<0x111, 0xf>(u); u = o < u ? o : u;
    o = dpp_move_u64_max_id<0x112, 0xf>(u); u = o < u ? o : u;
    o = dpp_move_u64_max_id<0x114, 0xf>(u); u = o < u ? o : u;
    o = dpp_move_u64_max_id<0x118, 0xf>(u); u = o < u ? o : u;
    o = dpp_move_u64_max_id<0x142, 0xa>(u); u = o < u ? o : u;
    o = dpp_move_u64_max_id<0x143, 0xc>(u); u = o < u ? o : u;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, kWave - 1);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), kWave - 1);
    return __longlong_as_double((long long)((uint64_t)lo | ((uint64_t)hi << 32)));
}
// the same over each 16-lane row, held by the row's last lane
__device__ __forceinline__ double row_min_nonneg_f64(double v) {
    uint64_t u = (uint64_t)__double_as_longlong(v), o;
    o = dpp_move_u64_max_id<0x111, 0xf>(u); u = o < u ? o : u;
    o = dpp_move_u64_max_id<0x112, 0xf>(u); u = o < u ? o : u;
    o = dpp_move_u64_max_id<0x114, 0xf>(u); u = o < u ? o : u;
    o = dpp_move_u64_max_id<0x118, 0xf>(u); u = o < u ? o : u;
    return __longlong_as_double((long long)u);
}

// Exclusive prefix sum over a block of NT threads (NT a multiple of 64, <= 1024); returns the
// thread's exclusive prefix and writes the block total to *total.  Needs NT/64 words of LDS.
template <int NT>
__device__ __forceinline__ uint64_t block_excl_scan(uint64_t v, uint64_t *lds, uint64_t *total) {
    const int l = lane_id(), w = threadIdx.x / kWave;
    uint64_t x = v;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint64_t t = __shfl_up(x, d, kWave);
        if (l >= d) x += t;
    }
    if (l == kWave - 1) lds[w] = x;
    __syncthreads();
    uint64_t base = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < NT / kWave; k++) {
        uint64_t s = lds[k];
        if (k < w) base += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return base + x - v;
}

// a value that every lane of the wave holds, moved to a scalar register
__device__ __forceinline__ uint32_t uniform_u32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}
__device__ __forceinline__ uint64_t uniform_u64(uint64_t v) {
    return (uint64_t)uniform_u32((uint32_t)v) | ((uint64_t)uniform_u32((uint32_t)(v >> 32)) << 32);
}
__device__ __forceinline__ double uniform_f64(double v) {
    return __longlong_as_double((long long)uniform_u64((uint64_t)__double_as_longlong(v)));
}

// A 64-bit kernel argument copied into a scalar register pair of its own.  Arguments arrive
// in wide scalar tuples, and when the allocator spills such a tuple into vector lanes it
// reloads the whole tuple wherever one member is read: an argument read in a hot loop then
// costs one readlane per tuple register on every pass.  The copy is one s_mov_b64 that the
// compiler cannot fold back into the tuple (a readfirstlane of a scalar value it does).
template <class T>
__device__ __forceinline__ T own_sgpr_pair(T v) {
    static_assert(sizeof(T) == 8, "a 64-bit value");
    T r;
    asm("s_mov_b64 %0, %1" : "=s"(r) : "s"(v));
    return r;
}

__device__ __forceinline__ void wave_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Grid-stride index helpers.
__device__ __forceinline__ size_t gtid() { return (size_t)blockIdx.x * blockDim.x + threadIdx.x; }
__device__ __forceinline__ size_t gstride() { return (size_t)gridDim.x * blockDim.x; }

}  // namespace fdx
