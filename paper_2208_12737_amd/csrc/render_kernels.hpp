// Render kernels: one workgroup renders one tile of one pose's detector.
//
// A wave covers a TW x (64/TW) block of pixels, one ray per lane; a
// workgroup is WX x WY waves.  Neighbouring lanes trace neighbouring rays,
// so at any step the wave's gathers fall in a compact footprint of the
// volume and share cache lines.
//
// Modes
//   kImage    image only
//   kCount    image + per-pixel count of positive-length segments (gathers)
//   kJac      image + per-pixel Jacobian d image / d pose (7 floats)
//   kRetrace  sum over the tile of g * Jacobian (g = upstream image gradient)
//   kNcc      image (optional) + per-tile sums for the ZNCC loss and its
//             pose gradient: I, I^2, T, T^2, IT, J[7], T J[7], I J[7]
//   kNccLoss  image (optional) + per-tile sums for the ZNCC loss only:
//             I, I^2, T, T^2, IT
//   kJacDet   image + per-pixel d image / d (delta_x, delta_y, offset_u,
//             offset_v) (4 floats)
//   kL2       image (optional) + per-tile sums for the mean squared
//             difference and its pose gradient: (I-T)^2, (I-T) J[7]
//   kL2Loss   image (optional) + per-tile sum of (I-T)^2
#pragma once

#include "launch_budget.hpp"
#include "siddon.hpp"

namespace drr {

enum Mode { kImage = 0, kCount = 1, kJac = 2, kRetrace = 3, kNcc = 4, kNccLoss = 5,
            kJacDet = 6, kL2 = 7, kL2Loss = 8 };

constexpr int kNccSums = 26;
static_assert(kNccSums <= kMaxTileSums, "tile sums exceed the LDS budget");

template <int MODE>
struct ModeTraits {
    static constexpr bool jac =
        MODE == kJac || MODE == kRetrace || MODE == kNcc || MODE == kJacDet || MODE == kL2;
    static constexpr bool count = MODE == kCount;
    static constexpr int nsum =
        MODE == kRetrace ? 7
        : MODE == kNcc   ? kNccSums
        : MODE == kNccLoss ? 5
        : MODE == kL2    ? 8
        : MODE == kL2Loss ? 1
                         : 0;
};

// Gather pipeline depth (crossings the merge runs ahead of the
// accumulation) of a launch that fills the GPU: the image and count modes
// run about 1% faster at depth 2 (fewer lines in flight per wave, a higher
// L2 hit rate), every mode with a Jacobian or a loss reduction is faster at
// depth 4.  Small launches use depth 4 in every mode.  Results do not depend
// on the depth.
template <int MODE>
constexpr int full_depth()
{
    return (MODE == kImage || MODE == kCount) ? 2 : 4;
}

// Per-tile outputs.  `aux` is the upstream image gradient (kRetrace) or the
// target image (kNcc, kNccLoss, kL2, kL2Loss) of this pose; `partial` receives the tile's sums.
struct TileOut {
    float* image;      // [H][W] of this pose, may be NULL in kRetrace/kNcc
    float* jac;        // [H][W][7]
    int32_t* counts;   // [H][W]
    const float* aux;  // [H][W]
    double* partial;   // nsum doubles
};

template <int TW, int WX, int WY>
struct TileShape {
    static constexpr int th = 64 / TW;
    static constexpr int px_w = TW * WX;   // pixels per workgroup tile, along w
    static constexpr int px_h = th * WY;   // along h
    static constexpr int threads = 64 * WX * WY;
};

// Fixed-order workgroup reduction of NS per-lane values into out[0..NS).
template <int NS, int NWAVES>
__device__ inline void block_sums(double (&vals)[NS], double* lds, double* out)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        double s = wave_sum(vals[k]);
        if (lane == 0) lds[wave * NS + k] = s;
    }
    __syncthreads();
    if ((int)threadIdx.x < NS) {
        double acc = 0.0;
        for (int wv = 0; wv < NWAVES; ++wv) acc += lds[wv * NS + threadIdx.x];
        out[threadIdx.x] = acc;
    }
    __syncthreads();
}

// Always inlined: an out-of-line call (the plan kernels have two call sites
// per instance) passes the volume and detector fields in vector registers and
// turns their uses into per-lane loads.
// LEAN: for kernels that carry more state of their own (the persistent plan
// kernels, short of scalar registers), the pose's trigonometry is evaluated
// per lane and rebuilt in the Jacobian tail rather than kept through the
// loop, and the Jacobian loop is the masked one only (see trace()); the
// results are the same bits.
template <int TW, int WX, int WY, int MODE, int DEPTH, bool LEAN = false>
__device__ __forceinline__ void render_tile(const VolArgs& V, const DetArgs& D,
                                            const float* __restrict__ pose, int tx, int ty,
                                            const TileOut& o, double* lds)
{
    using S = TileShape<TW, WX, WY>;
    using T = ModeTraits<MODE>;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wx = wave % WX, wy = wave / WX;
    const int w = (tx * WX + wx) * TW + lane % TW;
    const int h = (ty * WY + wy) * S::th + lane / TW;
    const bool inside = (w < D.W) && (h < D.H);

    const PoseTrig q = LEAN ? pose_trig_per_lane(pose) : pose_trig(pose);
    const Mat3 R = rotation(q.ct, q.st, q.cp, q.sp, q.cg, q.sg, -1);
    const double u = ((double)w + 0.5 - 0.5 * (double)D.W) * (double)D.dx + D.ou;
    const double v = ((double)h + 0.5 - 0.5 * (double)D.H) * (double)D.dy + D.ov;
    double s[3], d[3];
    ray_of(q, R, u, v, s, d);

    // Copy of the volume for this pose: by the principal axis of its
    // central ray (the direction of -R e_x), the same for the whole tile.
    int principal = 0;
    {
        const double c0 = fabs(R.m[0][0]), c1 = fabs(R.m[1][0]), c2 = fabs(R.m[2][0]);
        principal = (c1 > c0 && c1 >= c2) ? 1 : ((c2 > c0 && c2 > c1) ? 2 : 0);
    }
    // (selects, not indexing: a dynamic index into the argument block would
    // be lowered to a scratch copy of it)
    const int copy = __builtin_amdgcn_readfirstlane(
        principal == 0 ? V.copy_for[0] : (principal == 1 ? V.copy_for[1] : V.copy_for[2]));
    const __amdgpu_buffer_rsrc_t rsrc = make_rsrc(V, copy);
    int32_t pitch[3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
        pitch[c] = __builtin_amdgcn_readfirstlane(
            copy == 0 ? V.pitch[0][c] : (copy == 1 ? V.pitch[1][c] : V.pitch[2][c]));

    RayAcc r;
    r.sum = 0.0;
    r.a0 = r.a1 = r.a2 = r.b0 = r.b1 = r.b2 = 0.0f;
    r.nseg = 0;
    r.valid = true;
    // Axis whose Jacobian sums are derived from the identities: the
    // principal axis of the wave's first ray.  The wave's rays are a few
    // pixels apart, so |d| / |d_c| stays below ~sqrt(3) for all of them,
    // however wide the detector's fan.
    const double e0 = fabs(d[0]), e1 = fabs(d[1]), e2 = fabs(d[2]);
    const int derived =
        __builtin_amdgcn_readfirstlane((e0 >= e1 && e0 >= e2) ? 0 : (e1 >= e2 ? 1 : 2));
    if (inside) {
        if (!T::jac)
            r = trace<false, T::count, 0, DEPTH>(V, rsrc, pitch, s, d);
        else if (derived == 0)
            r = trace<T::jac, T::count, 0, DEPTH, !LEAN>(V, rsrc, pitch, s, d);
        else if (derived == 1)
            r = trace<T::jac, T::count, 1, DEPTH, !LEAN>(V, rsrc, pitch, s, d);
        else
            r = trace<T::jac, T::count, 2, DEPTH, !LEAN>(V, rsrc, pitch, s, d);
    }

    const double L = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    const float E = r.valid ? (float)(L * r.sum) : __builtin_nanf("");
    const int64_t pix = (int64_t)h * D.W + w;

    float J[7], Jp[4];
    if (T::jac) {
        const PoseTrig qt = LEAN ? pose_trig_per_lane(launder(pose)) : q;
        if (inside && r.valid) {
            ray_jacobian(r, qt, u, v, J, MODE == kJacDet ? Jp : nullptr,
                         (double)w + 0.5 - 0.5 * (double)D.W, (double)h + 0.5 - 0.5 * (double)D.H);
        } else {
#pragma unroll
            for (int j = 0; j < 7; ++j) J[j] = inside ? __builtin_nanf("") : 0.0f;
            Jp[0] = Jp[1] = Jp[2] = Jp[3] = inside ? __builtin_nanf("") : 0.0f;
        }
    }

    if (inside) {
        if (o.image) o.image[pix] = E;
        if (MODE == kCount) o.counts[pix] = r.nseg;
        if (MODE == kJac) {
#pragma unroll
            for (int j = 0; j < 7; ++j) o.jac[pix * 7 + j] = J[j];
        }
        if (MODE == kJacDet) {
#pragma unroll
            for (int j = 0; j < 4; ++j) o.jac[pix * 4 + j] = Jp[j];
        }
    }

    if (MODE == kRetrace) {
        const float g = inside ? o.aux[pix] : 0.0f;
        double vals[7];
#pragma unroll
        for (int j = 0; j < 7; ++j) vals[j] = inside ? (double)g * (double)J[j] : 0.0;
        block_sums<7, WX * WY>(vals, lds, o.partial);
    }
    if (MODE == kNcc) {
        const double I = inside ? (double)E : 0.0;
        const double Tv = inside ? (double)o.aux[pix] : 0.0;
        double vals[kNccSums];
        vals[0] = I;
        vals[1] = I * I;
        vals[2] = Tv;
        vals[3] = Tv * Tv;
        vals[4] = I * Tv;
#pragma unroll
        for (int j = 0; j < 7; ++j) {
            const double Jj = inside ? (double)J[j] : 0.0;
            vals[5 + j] = Jj;
            vals[12 + j] = Tv * Jj;
            vals[19 + j] = I * Jj;
        }
        block_sums<kNccSums, WX * WY>(vals, lds, o.partial);
    }
    if (MODE == kNccLoss) {
        const double I = inside ? (double)E : 0.0;
        const double Tv = inside ? (double)o.aux[pix] : 0.0;
        double vals[5] = {I, I * I, Tv, Tv * Tv, I * Tv};
        block_sums<5, WX * WY>(vals, lds, o.partial);
    }
    if constexpr (MODE == kL2 || MODE == kL2Loss) {
        const double r_ = inside ? (double)E - (double)o.aux[pix] : 0.0;
        double vals[T::nsum];
        vals[0] = r_ * r_;
        if constexpr (MODE == kL2) {
#pragma unroll
            for (int j = 0; j < 7; ++j) vals[1 + j] = inside ? r_ * (double)J[j] : 0.0;
        }
        block_sums<T::nsum, WX * WY>(vals, lds, o.partial);
    }
}

// Pose and tile of workgroup `bid` of a flat launch.  Hardware dispatch
// deals consecutive workgroup ids to the 8 XCDs in turn.  When a pose's tile
// count divides by 8, the XCDs advance through the poses together, each
// taking a contiguous band of every pose's tiles (neighbouring tiles share
// its L2, and the poses being traced at once are few, which spares the
// Infinity Cache); otherwise each XCD takes a contiguous range of the
// launch's tiles.  Which workgroup traces a tile never changes a result.
__device__ inline void pose_tile(uint32_t bid, uint32_t total, uint32_t tiles, int* b, int* t)
{
    if (tiles % 8u == 0u) {
        const uint32_t k = bid % tiles;
        *b = (int)(bid / tiles);
        *t = (int)((k % 8u) * (tiles / 8u) + k / 8u);
    } else {
        const uint32_t logical = xcd_logical(bid, total);
        *b = (int)(logical / tiles);
        *t = (int)(logical % tiles);
    }
}

// Flat launch: grid = wg_per_pose * n_poses workgroups, XCD-aware ordering.
template <int TW, int WX, int WY, int MODE, int DEPTH>
__global__ __launch_bounds__(64 * WX * WY) void render_flat(
    VolArgs V, DetArgs D, const float* __restrict__ poses, int tiles_x, int wg_per_pose,
    float* image, float* jac, int32_t* counts, const float* aux, int64_t aux_stride,
    double* partials)
{
    using T = ModeTraits<MODE>;
    __shared__ double lds[(T::nsum > 0 ? T::nsum : 1) * WX * WY];
    static_assert(sizeof(lds) == tile_sum_lds_bytes(T::nsum, WX * WY), "static LDS budget");
    int b, t;
    pose_tile(blockIdx.x, gridDim.x, (uint32_t)wg_per_pose, &b, &t);
    const int ty = t / tiles_x, tx = t % tiles_x;
    const int64_t hw = (int64_t)D.H * D.W;
    TileOut o;
    o.image = image ? image + b * hw : nullptr;
    o.jac = jac ? jac + b * hw * (MODE == kJacDet ? 4 : 7) : nullptr;
    o.counts = counts ? counts + b * hw : nullptr;
    o.aux = aux ? aux + b * aux_stride : nullptr;
    o.partial = T::nsum > 0 ? partials + ((int64_t)b * wg_per_pose + t) * T::nsum : nullptr;
    render_tile<TW, WX, WY, MODE, DEPTH>(V, D, poses + 7 * b, tx, ty, o, lds);
}

}  // namespace drr
