// Launch shapes of the render kernels and the LDS each launch asks for.
//
// Plain C++ (no HIP): host-only tests compile this header on its own and
// check, for every shape and residency setting, that a launch never asks
// for more LDS than one workgroup may allocate (a larger request is
// rejected when the dispatch starts, and that aborts the queue).
#pragma once

#include <stddef.h>

namespace drr {

// A launch shape: pixels per wave row (a wave covers tw x 64/tw pixels) and
// waves per workgroup along w and along h.
struct ShapeInfo {
    int tw, wx, wy;
};

// Candidate shapes of the plans (autotuner codes 0..kNumShapes-1).
constexpr ShapeInfo kShapes[] = {
    {8, 2, 2},    // 0: 16 x 16 px, 8 x 8 wave tiles
    {8, 1, 1},    // 1:  8 x  8 px
    {8, 1, 4},    // 2:  8 x 32 px
    {16, 1, 4},   // 3: 16 x 16 px, 16 x 4 wave tiles
    {4, 4, 1},    // 4: 16 x 16 px,  4 x 16 wave tiles
    {8, 4, 1},    // 5: 32 x  8 px
    {4, 1, 4},    // 6:  4 x 64 px,  4 x 16 wave tiles
    {2, 2, 2},    // 7:  4 x 64 px,  2 x 32 wave tiles
    {1, 4, 1},    // 8:  4 x 64 px,  1 x 64 wave tiles
};
constexpr int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);

// Shape of the direct (non-plan) entry points: 4 x 16-pixel wave tiles
// (4 columns, 16 rows), 4 waves side by side (16 x 16 pixels, 256 threads).
// Of nine shapes timed on the 256-pose CT batch this one was the fastest for
// the image mode and level with the best for the fused gradient.
#ifndef DRR_DIRECT_SHAPE
#define DRR_DIRECT_SHAPE {4, 4, 1}
#endif
constexpr ShapeInfo kDirectShape = DRR_DIRECT_SHAPE;

// Largest number of FP64 sums a render workgroup reduces per tile (the fused
// -ZNCC objective: I, I^2, T, T^2, IT, J[7], TJ[7], IJ[7]).
constexpr int kMaxTileSums = 26;

// Static LDS of a render kernel whose `waves`-wave workgroup reduces `nsum`
// FP64 sums per tile (one slot per wave and sum; at least one double).
constexpr size_t tile_sum_lds_bytes(int nsum, int waves)
{
    return sizeof(double) * (size_t)(nsum > 0 ? nsum : 1) * (size_t)waves;
}

// Bytes kept free of each workgroup's share of the CU for the allocation
// granularity of LDS.
constexpr size_t kLdsMargin = 512;

struct LdsLimits {
    size_t per_cu, per_block;
};

// Dynamic LDS to reserve per workgroup so that `wg_per_cu` workgroups are
// resident on a CU (0 or less: no limit), for a kernel that already uses
// `static_bytes` of LDS.  The workgroup's whole allocation (static +
// dynamic) is its share of the CU less the margin, and never more than one
// workgroup may allocate.  With LDS allocated in 512-byte units this admits
// exactly `wg_per_cu` workgroups for settings of up to 8; larger settings,
// or a cap that binds, can admit more.
inline size_t occupancy_lds_bytes(const LdsLimits& lim, int wg_per_cu, size_t static_bytes)
{
    if (wg_per_cu <= 0) return 0;
    const size_t share = lim.per_cu / (size_t)wg_per_cu;
    const size_t used = static_bytes + kLdsMargin;
    const size_t dyn = share > used ? share - used : 0;
    const size_t cap = lim.per_block > used ? lim.per_block - used : 0;
    return dyn < cap ? dyn : cap;
}

}  // namespace drr
