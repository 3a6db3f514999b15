// The opening test of the group walk (k_walk.hip, k_fused.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace fdx {

// The opening test: a cell of side S (level l: S = 2^(22-l) half-grid units) whose centre
// lies at distance D from the box [bmin, bmax] (half-grid units) is accepted iff
// S^2 < theta^2 D^2; D^2 is an exact integer in FP64 and the product is rounded once.
__device__ __forceinline__ bool cell_accepted(const uint4 nd, int bminx, int bminy, int bminz,
                                              int bmaxx, int bmaxy, int bmaxz, double theta2) {
    const int lv = (int)(nd.w & 0xFFu);
    const int cx = (int)nd.x, cy = (int)nd.y, cz = (int)nd.z;
    const int dx = max(0, max(bminx - cx, cx - bmaxx));
    const int dy = max(0, max(bminy - cy, cy - bmaxy));
    const int dz = max(0, max(bminz - cz, cz - bmaxz));
    const double D2 = (double)dx * (double)dx + (double)dy * (double)dy +
                      (double)dz * (double)dz;                         // exact integers
    const double S2 = __longlong_as_double((long long)(1023 + 2 * (22 - lv)) << 52);
    return S2 < __dmul_rn(theta2, D2);
}

}  // namespace fdx
