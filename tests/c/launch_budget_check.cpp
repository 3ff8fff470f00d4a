// Host-only check of the LDS each render launch asks for: for every launch
// shape (the plans' candidates and the direct shape), every number of tile
// sums a render mode reduces, every residency setting the library accepts
// and several per-CU / per-workgroup LDS limits, the workgroup's static plus
// reserved dynamic LDS stays within what one workgroup may allocate, and
// the reservation caps residency at the request (settings of up to 8
// workgroups per CU, the range the library and its autotuner use) where
// that limit allows.  Prints "ok" and
// exits 0, or prints the first violation and exits 1.
#include <stdio.h>

#include "launch_budget.hpp"

using namespace drr;

static int check(const LdsLimits& lim, const ShapeInfo& sh, int nsum, size_t extra, int wg)
{
    const int waves = sh.wx * sh.wy;
    const size_t stat = tile_sum_lds_bytes(nsum, waves) + extra;
    const size_t dyn = occupancy_lds_bytes(lim, wg, stat);
    const size_t total = stat + dyn;
    if (stat + kLdsMargin <= lim.per_block && total > lim.per_block) {
        printf("over the per-workgroup limit: per_cu %zu per_block %zu shape {%d,%d,%d} "
               "nsum %d extra %zu wg %d: static %zu + dynamic %zu\n",
               lim.per_cu, lim.per_block, sh.tw, sh.wx, sh.wy, nsum, extra, wg, stat, dyn);
        return 1;
    }
    if (wg > 0 && wg <= 8 && dyn > 0) {
        // residency the reservation allows (LDS is allocated in 512-byte
        // units) equals the request where the per-workgroup cap did not bind
        const size_t alloc = (total + 511) / 512 * 512;
        const size_t resident = lim.per_cu / alloc;
        const bool capped = dyn == lim.per_block - (stat + kLdsMargin);
        if (!capped && resident != (size_t)wg) {
            printf("residency %zu against the requested %d: per_cu %zu per_block %zu "
                   "shape {%d,%d,%d} nsum %d\n",
                   resident, wg, lim.per_cu, lim.per_block, sh.tw, sh.wx, sh.wy, nsum);
            return 1;
        }
    }
    if (wg <= 0 && dyn != 0) {
        printf("no limit requested but %zu bytes reserved\n", dyn);
        return 1;
    }
    return 0;
}

int main()
{
    const LdsLimits limits[] = {
        {160 * 1024, 160 * 1024}, {160 * 1024, 64 * 1024}, {64 * 1024, 64 * 1024},
        {64 * 1024, 32 * 1024},   {96 * 1024, 96 * 1024},
    };
    ShapeInfo shapes[kNumShapes + 1];
    for (int i = 0; i < kNumShapes; ++i) shapes[i] = kShapes[i];
    shapes[kNumShapes] = kDirectShape;
    long cases = 0;
    for (const LdsLimits& lim : limits)
        for (const ShapeInfo& sh : shapes)
            for (int nsum = 0; nsum <= kMaxTileSums; ++nsum)
                for (size_t extra = 0; extra <= 16; extra += 16)
                    for (int wg = -1; wg <= 64; ++wg) {
                        if (check(lim, sh, nsum, extra, wg)) return 1;
                        ++cases;
                    }
    printf("ok %ld cases\n", cases);
    return 0;
}
