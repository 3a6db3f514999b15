// Order in which the waves of the group walk by runs (k_walk.hip) take the runs: the launch
// rule and the wave -> run slot mapping, plain C++ so that a host program can check them.
//
// The workgroups go to the eight XCDs in turn (workgroup b to XCD b mod 8).  The waves of XCD
// x take the runs of every eighth chunk of `chunk` consecutive runs, x-th first, so the waves
// walking at once on one XCD work on neighbouring groups and share the cells in that XCD's
// L2, while every XCD still gets its share of the dense and the sparse regions.  A wave takes
// one run per W = all waves of the grid (its slot, then slot + W, ...).
#pragma once

#include <cstddef>
#include <cstdint>

#if defined(__HIPCC__)
#define FDX_WALK_ORDER_HD __host__ __device__
#else
#define FDX_WALK_ORDER_HD
#endif

namespace fdx {

constexpr uint32_t kWalkOrderWaves = 4;    // waves per workgroup of the walk
constexpr uint32_t kXcdChunk = 1024;       // most runs per chunk

// Grid and chunk for `items` runs, starting from a grid of grid0 workgroups: the chunk is a
// power of two, at most kXcdChunk, at most 1/48 of the runs (every XCD gets six chunks or
// more) and at most one XCD's waves (W / 8 = grid / 2); the grid is rounded up to a multiple
// of 8 and of 2 chunk, which makes the slots a permutation of 0..W-1.
inline void walk_order_launch(size_t items, size_t grid0, size_t *grid, uint32_t *chunk) {
    uint32_t c = kXcdChunk;
    while (c > 1 && (2 * (size_t)c > grid0 || 48 * (size_t)c > items)) c >>= 1;
    const size_t m = 2 * (size_t)c < 8 ? 8 : 2 * (size_t)c;
    *grid = (grid0 + m - 1) / m * m;
    *chunk = c;
}

// slot of wave w of workgroup b in a grid of nb workgroups (the plain order b * waves + w
// when the grid does not fit the rule, or chunk is 0)
FDX_WALK_ORDER_HD inline uint32_t walk_order_slot(uint32_t b, uint32_t w, uint32_t nb,
                                                   uint32_t chunk) {
    if (chunk == 0 || nb % 8u != 0 || nb % (2u * chunk) != 0) return b * kWalkOrderWaves + w;
    const uint32_t x = b % 8u, local = (b / 8u) * kWalkOrderWaves + w;
    return ((local / chunk) * 8u + x) * chunk + local % chunk;
}

}  // namespace fdx
