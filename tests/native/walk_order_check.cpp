// Host check of the group walk's run order (walk_order.h): for run counts from 1 to past one
// grid-wide round, the launch rule gives a grid of a multiple of 8 and of 2 chunk workgroups,
// the slots of all waves are a permutation of 0..W-1, one round covers every run up to the
// grid cap, and every XCD's chunks hold runs.  Prints one line per failure and "ok" at the end.
#include <cstdio>
#include <vector>

#include "walk_order.h"

using namespace fdx;

int main() {
    const size_t counts[] = {1, 2, 3, 7, 8, 31, 100, 513, 1000, 3500, 14000, 49151, 49152,
                             56250, 65535, 65536, 65537, 88000, 262144};
    int bad = 0;
    for (size_t items : counts) {
        size_t grid0 = (items + kWalkOrderWaves - 1) / kWalkOrderWaves;
        grid0 = grid0 < 1 ? 1 : (grid0 > 16384 ? 16384 : grid0);
        size_t grid = 0;
        uint32_t chunk = 0;
        walk_order_launch(items, grid0, &grid, &chunk);
        if (chunk < 1 || (chunk & (chunk - 1)) || chunk > kXcdChunk || grid % 8 ||
            grid % (2 * chunk) || grid > 16384) {
            printf("rule %zu: grid %zu chunk %u\n", items, grid, chunk);
            bad++;
            continue;
        }
        const size_t W = grid * kWalkOrderWaves;
        std::vector<int> seen(W, 0);
        std::vector<size_t> per_xcd(8, 0);
        for (uint32_t b = 0; b < grid; b++)
            for (uint32_t w = 0; w < kWalkOrderWaves; w++) {
                const uint32_t s = walk_order_slot(b, w, (uint32_t)grid, chunk);
                if (s >= W) { printf("slot %zu: %u >= %zu\n", items, s, W); bad++; continue; }
                seen[s]++;
                if (s < items) per_xcd[b % 8]++;
            }
        for (size_t s = 0; s < W; s++)
            if (seen[s] != 1) { printf("perm %zu: slot %zu seen %d times\n", items, s, seen[s]); bad++; break; }
        if (W < (items < 65536 ? items : 65536)) { printf("cover %zu: W %zu\n", items, W); bad++; }
        // with at least 48 chunks of runs every XCD's waves take part
        if (items >= 48 * (size_t)chunk)
            for (int x = 0; x < 8; x++)
                if (per_xcd[x] == 0) { printf("xcd %zu: XCD %d idle\n", items, x); bad++; }
        // the plain order when the rule does not hold
        if (walk_order_slot(5, 3, 12, 4) != 5 * kWalkOrderWaves + 3) { printf("plain\n"); bad++; }
    }
    printf(bad ? "failures %d\n" : "ok\n", bad);
    return bad ? 1 : 0;
}
