// Host-side check of the tiled update's work list (tile::build_schedule):
// every (tile column, plane) is covered exactly once, segments are
// non-empty and inside the grid, each block's list is contiguous from its
// first entry, and the largest block cost equals the reported cost.  Prints
// one line per case: columns nz resident tz grid nseg cost ideal split, and
// the number of segments of an odd number of planes that another segment of
// the same block follows.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "tslb_tiles.h"

using namespace tslb::tile;

static int check(int columns, int nz, int resident) {
    const Schedule s = build_schedule(columns, nz, resident);
    std::vector<int> seen((size_t)columns * nz, 0);
    long long worst = 0, odd_then_more = 0;
    if (s.grid % 8 != 0 || s.grid > resident || s.nseg < 1 || s.seg.size() != (size_t)s.grid * s.nseg) return 1;
    for (int b = 0; b < s.grid; ++b) {
        long long cost = 0;
        bool ended = false;
        for (int k = 0; k < s.nseg; ++k) {
            const int4 q = s.seg[(size_t)b * s.nseg + k];
            if (q.x < 0) {
                ended = true;
                continue;
            }
            if (ended) return 2;  // an entry after the end marker
            if (((q.z - q.y) & 1) && k + 1 < s.nseg && s.seg[(size_t)b * s.nseg + k + 1].x >= 0) ++odd_then_more;
            if (q.x >= columns || q.y < 0 || q.z > nz || q.y >= q.z) return 3;
            for (int z = q.y; z < q.z; ++z) seen[(size_t)q.x * nz + z] += 1;
            cost += q.z - q.y + 2;
        }
        if (cost > worst) worst = cost;
    }
    for (int v : seen)
        if (v != 1) return 4;
    if (worst != s.cost) return 5;
    const long long ideal = ((long long)columns * nz + resident - 1) / resident + 2;
    printf("%d %d %d %d %d %d %lld %lld %d %lld\n", columns, nz, resident, s.tz, s.grid, s.nseg, s.cost, ideal, s.split,
           odd_then_more);
    return 0;
}

int main() {
    const int cases[][3] = {
        {176, 256, 256}, {96, 192, 256}, {344, 512, 256}, {259, 600, 256}, {6, 64, 256}, {1, 1, 256},
        {1, 3, 256},     {2, 1, 8},      {16, 5, 256},    {1376, 1023, 256}, {7, 300, 16}, {33, 17, 40},
        {20, 457, 256},
    };
    for (const auto& c : cases) {
        const int rc = check(c[0], c[1], c[2]);
        if (rc) {
            printf("FAIL %d %d %d: %d\n", c[0], c[1], c[2], rc);
            return rc;
        }
    }
    return 0;
}
