// Device-side Siddon-Jacobs ray traversal for gfx950.
//
// One ray per lane.  The plane crossings of Eq. 3 are produced in increasing
// order by a three-way merge kept in registers (the iterative form of
// Sec. 2.2): each axis holds the parameter of its next crossing and the
// parametric step between its planes; the smallest of the three ends the
// current segment (Eq. 2), and the axes that attain it advance.  Crossing
// state is FP64 so that segment lengths, taken as differences of crossing
// parameters, keep their relative accuracy; voxel values are FP32 and the
// path sum is accumulated in FP64.
//
// The packed volume is the caller's grid surrounded by a one-voxel border
// of zeros, read through a raw buffer resource: a rounding-induced step one
// voxel past the last crossing lands in the border (value 0), and any offset
// beyond the buffer reads 0 instead of faulting.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace drr {

constexpr uint32_t kBufferDword3 = 0x00020000u;  // gfx9 raw buffer, 32-bit data

// Crossing parameters are advanced by repeated addition, so a plane that
// coincides with the exit (or with another plane) can land a few ulps away
// from it and open a sliver segment.  The segment counter (gathers per ray)
// ignores segments shorter than this many units of alpha -- 2^-36 of the
// source-detector distance, about 1.5e-8 mm at 1 m.  The path sum itself
// always includes every segment.
constexpr double kSliver = 0x1p-36;

// Gather pipeline depth (crossings the merge runs ahead of the
// accumulation) of the small launches, which leave a SIMD with few waves to
// hide the latency of the gathers.  The depth changes only when loads are
// issued, never the order of the arithmetic: results are bitwise the same at
// any depth.
constexpr int kDeepDepth = 4;
// Depth of launches that leave each SIMD a single wave.
#ifndef DRR_TINY_DEPTH
#define DRR_TINY_DEPTH 6
#endif
constexpr int kTinyDepth = DRR_TINY_DEPTH;

// A packed volume: one or three copies of the zero-bordered grid, each in
// its own memory order.  pitch[q][c] is the byte distance between
// neighbouring voxels along axis c in copy q; copy_for[c] names the copy read
// by poses whose central ray runs mostly along axis c.
struct VolArgs {
    const float* packed;
    double spacing[3];
    double origin[3];
    int32_t n[3];
    uint32_t copy_bytes;
    int32_t pitch[3][3];
    int32_t copy_for[3];
};

struct DetArgs {
    double dx, dy;   // pitch
    double ou, ov;   // principal-point offset
    int32_t H, W;
};

// ------------------------------------------------------------------ geometry

struct Mat3 {
    double m[3][3];
};

__device__ inline Mat3 mul(const Mat3& a, const Mat3& b)
{
    Mat3 c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            c.m[i][j] = a.m[i][0] * b.m[0][j] + a.m[i][1] * b.m[1][j] + a.m[i][2] * b.m[2][j];
    return c;
}

// Rz(theta) Ry(phi) Rx(gamma); `which` = 0/1/2 differentiates one factor.
__device__ inline Mat3 rotation(double ct, double st, double cp, double sp, double cg, double sg,
                                int which)
{
    Mat3 z = {{{ct, -st, 0.0}, {st, ct, 0.0}, {0.0, 0.0, 1.0}}};
    Mat3 y = {{{cp, 0.0, sp}, {0.0, 1.0, 0.0}, {-sp, 0.0, cp}}};
    Mat3 x = {{{1.0, 0.0, 0.0}, {0.0, cg, -sg}, {0.0, sg, cg}}};
    if (which == 0) z = Mat3{{{-st, -ct, 0.0}, {ct, -st, 0.0}, {0.0, 0.0, 0.0}}};
    if (which == 1) y = Mat3{{{-sp, 0.0, cp}, {0.0, 0.0, 0.0}, {-cp, 0.0, -sp}}};
    if (which == 2) x = Mat3{{{0.0, 0.0, 0.0}, {0.0, -sg, -cg}, {0.0, cg, -sg}}};
    return mul(mul(z, y), x);
}

struct PoseTrig {
    double ct, st, cp, sp, cg, sg;
    double rho;
    double t[3];
};

// Value of x in lane `lane` of the wave (a scalar, uniform result).
__device__ inline double lane_value(double x, int lane)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
    return __hiloint2double(hi, lo);
}

// The pose's trigonometry, once per wave: lanes 0, 1 and 2 evaluate the sine
// and cosine of the three angles in one vector sincos, and every lane reads
// the results back as wave-uniform (scalar) values.  Every lane of the wave
// must be active.
__device__ inline PoseTrig pose_trig(const float* __restrict__ pose)
{
    const int lane = (int)(threadIdx.x & 63);
    const float ang = lane == 0 ? pose[0] : (lane == 1 ? pose[1] : pose[2]);
    double sn, cs;
    sincos((double)ang, &sn, &cs);
    PoseTrig q;
    q.st = lane_value(sn, 0);
    q.ct = lane_value(cs, 0);
    q.sp = lane_value(sn, 1);
    q.cp = lane_value(cs, 1);
    q.sg = lane_value(sn, 2);
    q.cg = lane_value(cs, 2);
    q.t[0] = pose[3];
    q.t[1] = pose[4];
    q.t[2] = pose[5];
    q.rho = 0.5 * (double)pose[6];
    return q;
}

// The same, evaluated by every lane (vector registers).  Kernels short of
// scalar registers use this form: there the wave-uniform values above would
// be spilled to vector registers while the traversal runs.
__device__ inline PoseTrig pose_trig_per_lane(const float* __restrict__ pose)
{
    PoseTrig q;
    sincos((double)pose[0], &q.st, &q.ct);
    sincos((double)pose[1], &q.sp, &q.cp);
    sincos((double)pose[2], &q.sg, &q.cg);
    q.t[0] = pose[3];
    q.t[1] = pose[4];
    q.t[2] = pose[5];
    q.rho = 0.5 * (double)pose[6];
    return q;
}

// Source s and direction d = p - s for detector coordinates (u, v).
__device__ inline void ray_of(const PoseTrig& q, const Mat3& R, double u, double v, double s[3],
                              double d[3])
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        s[c] = q.rho * R.m[c][0] + q.t[c];
        d[c] = -2.0 * q.rho * R.m[c][0] + u * R.m[c][1] + v * R.m[c][2];
    }
}

// ------------------------------------------------------------------ traversal

// Per-ray result.  sum = E / |d|.  For the Jacobian, crossings are grouped by
// the axis of their plane: A_c = sum of (V_before - V_after) over the c-plane
// crossings, B_c = sum of alpha (V_before - V_after).  Ends clamped to the
// ray's own [0, 1] do not move with the pose and belong to no axis.  Two axes
// are summed in the loop; the third follows from sum_k (V_before - V_after)
// = 0 and sum_k alpha_k (V_before - V_after) = E/|d| over all crossings.  That third axis carries the rounding
// error of the other two, which the tail multiplies by |d| / |d_c|, so it is
// the principal axis of the wave's first ray (|d| / |d_c| <= ~sqrt(3) for
// the wave's rays); deriving an axis whose planes a ray runs almost parallel
// to would multiply the error by millions.
struct RayAcc {
    double sum;
    float a0, a1, a2, b0, b1, b2;
    int32_t nseg;
    bool valid;  // false: non-finite geometry (result NaN)
};

// Volume value at a byte offset into the packed buffer (0 beyond its end).
__device__ inline float ld(const __amdgpu_buffer_rsrc_t& r, uint32_t byte_off)
{
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)byte_off, 0, 0));
}

// min of two non-NaN doubles.  fmin() would first quiet possible signalling
// NaNs of loop-carried operands (an extra instruction per operand); the
// crossing parameters are never NaN (non-finite rays are rejected before
// the loop), so the bare instruction is exact here.
__device__ inline double min_nn(double a, double b)
{
    double r;
    asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// DERIVED is the axis whose Jacobian sums come from the identities rather
// than the loop: the principal axis of the wave's first ray, so that
// |d| / |d_DERIVED| stays small for every ray of the wave.  (A template
// argument: with a run-time axis the compiler selects between the per-lane
// crossing masks with several VALU instructions per step.)
// FOLDED_LOOP: compile the Jacobian loop without the exit mask for waves
// whose rays all fold their exit (see `clip`); without it every wave takes
// the masked loop, which gives the same bits at some 2 VALU instructions
// more per step and a few registers fewer.
template <bool JAC, bool COUNT, int DERIVED, int DEPTH, bool FOLDED_LOOP = true>
__device__ inline RayAcc trace(const VolArgs& V, const __amdgpu_buffer_rsrc_t& rsrc,
                               const int32_t pitch[3], const double s[3], const double d[3])
{
    static_assert(DEPTH >= 1 && DEPTH <= 12, "gather pipeline depth 1..12");
    static_assert(DEPTH >= 2 || !JAC, "the Jacobian sums need a pipeline depth of at least 2");
    static_assert(!(JAC && COUNT), "the folded Jacobian loop does not count segments");
    constexpr int derived = DERIVED;
    RayAcc r;
    r.sum = 0.0;
    r.a0 = r.a1 = r.a2 = r.b0 = r.b1 = r.b2 = 0.0f;
    r.nseg = 0;
    r.valid = true;

    bool finite = true;
#pragma unroll
    for (int c = 0; c < 3; ++c) finite = finite && isfinite(s[c]) && isfinite(d[c]);
    if (!finite) {
        r.valid = false;
        return r;
    }

    // Entry and exit parameters (Sec. 2.3), clamped to [0, 1].
    double amin = 0.0, amax = 1.0;
    int amin_ax = -1, amax_ax = -1;
    // Bound on how far the exit face's parameter, as the loop reaches it by
    // repeated steps, can lie from amax: the plane positions and the
    // divisions round within a few ulps of the largest coordinate involved
    // (scaled by 1 / |d_c| into alpha), and each of at most n_c + 4 steps
    // rounds by at most half an ulp of an alpha <= 1 (bounds doubled here).
    double amax_err = 0.0;
    bool miss = false;
    double o[3], sp[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        o[c] = V.origin[c];
        sp[c] = V.spacing[c];
        double hi_plane = o[c] + (double)V.n[c] * sp[c];
        if (d[c] != 0.0) {
            double a0 = (o[c] - s[c]) / d[c];
            double a1 = (hi_plane - s[c]) / d[c];
            double lo = fmin(a0, a1), hi = fmax(a0, a1);
            if (lo > amin) {
                amin = lo;
                amin_ax = c;
            }
            if (hi < amax) {
                amax = hi;
                amax_ax = c;
                const double P = fmax(fmax(fabs(o[c]), fabs(hi_plane)), fabs(s[c]));
                amax_err = (8.0 * P / fabs(d[c]) + (double)(V.n[c] + 4)) * 0x1p-52;
            }
        } else if (!(s[c] >= o[c] && s[c] < hi_plane)) {
            miss = true;
        }
    }
    if (miss || !(amin < amax)) return r;

    // Voxel just past the entry, and each axis's first crossing after it.
    const double ae = amin + (amax - amin) * 0x1p-30;
    // Per-axis state as named scalars (no arrays: a select between array
    // elements in the loop would be lowered to an indexed memory load).
    struct Axis {
        double a, da;
        uint32_t stride;
        uint32_t off;
    };
    auto axis = [&](int c) {
        Axis x;
        const double f = floor((s[c] + ae * d[c] - o[c]) / sp[c]);
        const int32_t i = (int32_t)fmin(fmax(f, 0.0), (double)(V.n[c] - 1));
        x.off = (uint32_t)((i + 1) * pitch[c]);
        if (d[c] > 0.0) {
            x.a = (o[c] + (double)(i + 1) * sp[c] - s[c]) / d[c];
            x.da = sp[c] / d[c];
            x.stride = (uint32_t)pitch[c];
        } else if (d[c] < 0.0) {
            x.a = (o[c] + (double)i * sp[c] - s[c]) / d[c];
            x.da = -sp[c] / d[c];
            x.stride = (uint32_t)(-pitch[c]);
        } else {
            x.a = __builtin_inf();
            x.da = 0.0;
            x.stride = 0u;
        }
        return x;
    };
    const Axis X0 = axis(0), Y0 = axis(1), Z0 = axis(2);
    // The axes by role: e1 < e2 are the two whose Jacobian sums the loop
    // keeps, `derived` the one whose sums follow from the identities.
    constexpr int e1 = derived == 0 ? 1 : 0, e2 = derived == 2 ? 1 : 2;
    const Axis& E1 = e1 == 0 ? X0 : Y0;
    const Axis& E2 = e2 == 2 ? Z0 : Y0;
    const Axis& ED = derived == 0 ? X0 : (derived == 1 ? Y0 : Z0);
    double a1 = E1.a, a2 = E2.a, ad = ED.a;
    // Each axis advances by fma(f, 128 da, a) with the factor f = 2^-7 for
    // the axis that advances and 0 for the others: f * 128 da = da exactly,
    // so this is a + da rounded once.  The high word of f = 2^-7 is
    // 0x3F800000, the bit pattern of 1.0f, so the factor's high word read as
    // a float is the 0/1 weight that files a crossing under its axis in the
    // Jacobian sums (one select per axis serves both).
    // (Steps beyond 2^1000 in alpha, from a direction component of the
    // order of 1e-300, are clamped there so that 128 da stays finite; such
    // an axis is never crossed twice within the ray's [0, 1].)
    const double d1 = fmin(E1.da, 0x1p1000) * 128.0, d2 = fmin(E2.da, 0x1p1000) * 128.0,
                 dd = fmin(ED.da, 0x1p1000) * 128.0;
    const uint32_t s1 = E1.stride, s2 = E2.stride, sd = ED.stride;
    // With the Jacobian, the step factors (2^-7 or 0, low words always 0) of
    // axes e1 and e2 rotate with the in-flight registers (they are the
    // weights the accumulation needs DEPTH steps later); fd is the derived
    // axis's.
    double fd = 0.0;
    uint32_t off = X0.off + Y0.off + Z0.off;
    const uint32_t off_entry = off;
    double acc = 0.0;
    int32_t nseg = 0;
    float vprev = 0.0f;
    // e1 and e2 sums: the running sum A of the jumps at the axis's
    // crossings, and the sum R of A after each of them (B = sum alpha *
    // jump follows from A and R, see below)
    float A1s = 0.f, A2s = 0.f, R1s = 0.f, R2s = 0.f;
    // Where the traversal stops (`clip`: the merge never returns a crossing
    // beyond it).
    //  * Exit through a face of the grid, computed well enough (folded):
    //    the clip lies a margin past alpha_max, below a quarter of every
    //    axis's step and 2^-37 (so below the sliver threshold), and at least
    //    four error bounds away.  The loop then takes the exit face's own
    //    crossing into the zero border (its jump, last voxel minus 0, is the
    //    exit term of the Jacobian sums) and at most one further crossing per
    //    axis, all between border voxels (jump 0, value 0).  Crossings at or
    //    beyond the clip are the derived axis's (weight 0) or, exactly at the
    //    clip, between border voxels: nothing past the clip changes a sum,
    //    so the loop needs no exit mask.
    //  * Otherwise (an end clamped to alpha = 1, or an exit face too close
    //    to parallel to the ray): the double just below alpha_max, as plain
    //    Siddon.  A plane of e1 or e2 that the repeated additions land
    //    exactly on alpha_max is then never taken; one landing on the clip
    //    itself is taken with jump 0 (the masked accumulation below).  The
    //    last segment is one ulp of alpha short (about 1e-16 of the sum).
    // Either way the crossings and sums are the same at every pipeline depth.
    const double amax_m = __longlong_as_double(__double_as_longlong(amax) - 1);
    auto step_or_inf = [](double da) { return da > 0.0 ? da : __builtin_inf(); };
    const double margin =
        fmin(0x1p-37, 0.25 * fmin(fmin(step_or_inf(X0.da), step_or_inf(Y0.da)), step_or_inf(Z0.da)));
    const bool fold = amax_ax >= 0 && 4.0 * amax_err <= margin;
    const double clip = fold ? amax + margin : amax_m;

    // The traversal is split into a merge (pick the next crossing, advance
    // that axis, issue the gather of the voxel beyond it) and an accumulation
    // (add a closed segment's length x value).  The merge runs DEPTH
    // crossings ahead of the accumulation, so every gather has DEPTH merge
    // steps of independent work between its issue and its use.  The
    // in-flight values live in DEPTH + 1 registers (DEPTH + 2 in the folded
    // Jacobian loop) whose roles rotate through a fully unrolled loop
    // (constant indices only): a copy of a loaded value would force an early
    // wait on the load.
    // (Macros rather than lambdas: a by-reference closure makes the compiler
    // keep the strides on the stack and load them every step.)
    //
    // Exactly one axis advances per merge (e1 before e2 before the derived
    // axis).  Tied crossings are therefore taken one per step, the later
    // ones closing zero-length segments; the voxel sequence and the sum are
    // unchanged.  Once the next crossing is the clip, every further merge
    // returns it again (the derived axis "advances" harmlessly, with weight
    // 0) and closes empty segments.
#define DRR_MERGE(vn, a_new, f1_new, f2_new)                                     \
    do {                                                                         \
        const double anext = min_nn(min_nn(a1, a2), min_nn(ad, clip));           \
        const bool b1 = a1 == anext;                                             \
        const bool b2 = !b1 && a2 == anext;                                      \
        const bool bd = (!b1) != b2;      /* = !b1 && !b2, as b2 implies !b1 */ \
        if (JAC) {                                                               \
            /* the factors of axes e1 and e2 are the crossing's weights   */    \
            f1_new = __hiloint2double(b1 ? 0x3F800000 : 0, __double2loint(f1_new)); \
            f2_new = __hiloint2double(b2 ? 0x3F800000 : 0, __double2loint(f2_new)); \
            fd = __hiloint2double(bd ? 0x3F800000 : 0, __double2loint(fd));      \
            a1 = fma(f1_new, d1, a1);                                            \
            a2 = fma(f2_new, d2, a2);                                            \
            ad = fma(fd, dd, ad);                                                \
        } else {                                                                 \
            a1 = fma(b1 ? 0x1p-7 : 0.0, d1, a1);                                 \
            a2 = fma(b2 ? 0x1p-7 : 0.0, d2, a2);                                 \
            ad = fma(bd ? 0x1p-7 : 0.0, dd, ad);                                 \
        }                                                                        \
        off += b1 ? s1 : (b2 ? s2 : sd);                                         \
        vn = ld(rsrc, off);                                                      \
        /* keep the gather where it is: the scheduler would otherwise sink  */ \
        /* it towards its use and shorten the distance the pipeline buys    */ \
        __builtin_amdgcn_sched_barrier(0);                                       \
        a_new = anext;                                                           \
    } while (0)
    // Closes segment [a_start, a_end] in the voxel of value vc; the crossing
    // at a_start (weights w1, w2) has V_before = vprev and V_after = vc.
    // Crossings at or after the clip change nothing (DRR_ACCUM masks their
    // jump to 0; they are the derived axis's, of weight 0, or lie exactly on
    // the clip).
    // Crossing m of an axis lies at alpha = a_first + (m - 1) da, so with the
    // running sums A_m and R = sum_m A_m over its n crossings,
    //   sum_m alpha_m jump_m = a_first A_n + da (n A_n - R),
    // which needs no per-step product with alpha.  (A plane of e1 or e2 that
    // landed exactly on the clip value would be taken with jump 0: it adds
    // 1 to n and A_n to R and leaves n A_n - R unchanged.)
#define DRR_ACCUM(vc, a_start, a_end, f1, f2)                                    \
    do {                                                                         \
        const double seg = (a_end) - (a_start);                                  \
        acc = fma(seg, (double)(vc), acc);                                       \
        if (COUNT) nseg += seg > kSliver ? 1 : 0;                                \
        if (JAC) {                                                               \
            const float w1 = __int_as_float(__double2hiint(f1));                 \
            const float w2 = __int_as_float(__double2hiint(f2));                 \
            const float vnew = (a_start) < clip ? (vc) : vprev;                  \
            const float dl = vprev - vnew;                                       \
            A1s = fmaf(w1, dl, A1s);                                             \
            R1s = fmaf(w1, A1s, R1s);                                            \
            A2s = fmaf(w2, dl, A2s);                                             \
            R2s = fmaf(w2, A2s, R2s);                                            \
            vprev = vnew;                                                        \
        }                                                                        \
    } while (0)

    // The same without the mask, for waves whose rays all fold their exit
    // into the loop: there the jumps at or after the clip are either of
    // weight 0 or between border voxels, and vp is the previous segment's
    // value, still in its in-flight register.
#define DRR_ACCUM_FOLDED(vc, vp, a_start, a_end, f1, f2)                         \
    do {                                                                         \
        const double seg = (a_end) - (a_start);                                  \
        acc = fma(seg, (double)(vc), acc);                                       \
        const float w1 = __int_as_float(__double2hiint(f1));                     \
        const float w2 = __int_as_float(__double2hiint(f2));                     \
        const float dl = (vp) - (vc);                                            \
        A1s = fmaf(w1, dl, A1s);                                                 \
        R1s = fmaf(w1, A1s, R1s);                                                \
        A2s = fmaf(w2, dl, A2s);                                                 \
        R2s = fmaf(w2, A2s, R2s);                                                \
    } while (0)

    // Every crossing either ends the ray or advances an axis by one plane
    // (with a folded exit, at most once more per axis past the exit face),
    // so n_x + n_y + n_z + 8 steps bound the loop for any input.  The loop
    // is wave-uniform; lanes that finished idle under the exec mask.  All
    // steps of an iteration run for a live lane (steps after the exit close
    // empty segments), which keeps each load ahead of its use.
    // Iteration: segment k = [a_k, a_{k+1}] is closed while the merge
    // produces the crossing DEPTH places ahead, into register (k + DEPTH) % NR.
    // (The entry crossing at alpha_min is not one of an axis's loop
    // crossings: it is added after the loop, and has weight 0 here.)
    // After the loop, the pipeline's last DEPTH crossings (registers 0 ..
    // DEPTH - 1, all at the clip, with jump 0) have been merged but not
    // accumulated: their R terms are added in merge order, so that the sums
    // cover every crossing the merge took whatever the depth.
    const int n_all = V.n[0] + V.n[1] + V.n[2];
    bool folded_loop = false;
    if constexpr (JAC && FOLDED_LOOP) folded_loop = __builtin_amdgcn_ballot_w64(!fold) == 0;
    if constexpr (JAC && FOLDED_LOOP) {
        if (folded_loop) {
            // one more in-flight register, so that the previous segment's
            // value is still held when the next segment closes
            constexpr int NR = DEPTH + 2;
            float v[NR];
            double a[NR], p[NR], q[NR];   // p, q: step factors of axes e1, e2
            v[0] = ld(rsrc, off);
            a[0] = amin;
#pragma unroll
            for (int k = 0; k < NR; ++k) {
                if (k > 0) {
                    v[k] = 0.0f;
                    a[k] = amin;
                }
                p[k] = q[k] = 0.0;
            }
#pragma unroll
            for (int k = 1; k < DEPTH; ++k) DRR_MERGE(v[k], a[k], p[k], q[k]);
            const int cap = (n_all + 2 * NR + 8) / NR + 2;
            bool active = true;
            for (int it = 0; it < cap; ++it) {
                if (active) {
#pragma unroll
                    for (int k = 0; k < NR; ++k) {
                        const int m = (k + DEPTH) % NR;
                        DRR_MERGE(v[m], a[m], p[m], q[m]);
                        DRR_ACCUM_FOLDED(v[k], v[(k + NR - 1) % NR], a[k], a[(k + 1) % NR],
                                         p[k], q[k]);
                    }
                    active = a[0] < clip;
                }
                if (__builtin_amdgcn_ballot_w64(active) == 0) break;
            }
#pragma unroll
            for (int k = 0; k < DEPTH; ++k) {
                R1s = fmaf(__int_as_float(__double2hiint(p[k])), A1s, R1s);
                R2s = fmaf(__int_as_float(__double2hiint(q[k])), A2s, R2s);
            }
            // the exit crossing was taken in the loop: the traversal ends in
            // the border, as the masked loop's vprev does for a folded ray
            vprev = 0.0f;
        }
    }
    if (!folded_loop) {
        constexpr int NR = DEPTH + 1;
        float v[NR];
        double a[NR], p[NR], q[NR];
        v[0] = ld(rsrc, off);
        a[0] = amin;
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            if (k > 0) {
                v[k] = 0.0f;
                a[k] = amin;
            }
            p[k] = q[k] = 0.0;
        }
#pragma unroll
        for (int k = 1; k < DEPTH; ++k) DRR_MERGE(v[k], a[k], p[k], q[k]);
        const int cap = (n_all + 2 * NR + 8) / NR + 2;
        bool active = true;
        for (int it = 0; it < cap; ++it) {
            if (active) {
#pragma unroll
                for (int k = 0; k < NR; ++k) {
                    const int m = (k + DEPTH) % NR;
                    DRR_MERGE(v[m], a[m], p[m], q[m]);
                    DRR_ACCUM(v[k], a[k], a[(k + 1) % NR], p[k], q[k]);
                }
                active = a[0] < clip;
            }
            if (__builtin_amdgcn_ballot_w64(active) == 0) break;
        }
        if (JAC) {
#pragma unroll
            for (int k = 0; k < DEPTH; ++k) {
                R1s = fmaf(__int_as_float(__double2hiint(p[k])), A1s, R1s);
                R2s = fmaf(__int_as_float(__double2hiint(q[k])), A2s, R2s);
            }
        }
    }
#undef DRR_MERGE
#undef DRR_ACCUM
#undef DRR_ACCUM_FOLDED
    r.sum = acc;
    r.nseg = nseg;
    if (JAC) {
        // crossings an axis advanced over: its alpha moved by whole steps
        auto advances = [](double a_now, double a_first, double da) {
            return (isfinite(a_first) && da > 0.0) ? rint((a_now - a_first) / da) : 0.0;
        };
        const double n1 = advances(a1, E1.a, d1 * 0x1p-7);
        const double n2 = advances(a2, E2.a, d2 * 0x1p-7);
        // (explicit fma: every instantiation rounds these the same way)
        auto alpha_sum = [](double n, double a_first, double da, float A, float R) {
            return n > 0.0 ? fma(a_first, (double)A, da * fma(n, (double)A, -(double)R)) : 0.0;
        };
        double B1 = alpha_sum(n1, E1.a, d1 * 0x1p-7, A1s, R1s);
        double B2 = alpha_sum(n2, E2.a, d2 * 0x1p-7, A2s, R2s);
        // Ends clamped to alpha = 0 or 1 belong to no axis (sums Ac, Bc); the
        // derived axis takes what the identities leave:
        //   A_d = -(A_e1 + A_e2 + Ac),  B_d = E/|d| - B_e1 - B_e2 - Bc.
        float Ac = 0.0f;
        double Bc = 0.0;
        // entry crossing at alpha_min: V_before = 0, V_after = the first voxel
        const float ventry = ld(rsrc, off_entry);
        if (amin_ax == e1) {
            A1s -= ventry;
            B1 = fma(-amin, (double)ventry, B1);
        } else if (amin_ax == e2) {
            A2s -= ventry;
            B2 = fma(-amin, (double)ventry, B2);
        } else if (amin_ax < 0) {
            Ac -= ventry;          // clamped to alpha = 0 (source inside the grid)
        }
        // exit crossing at alpha_max: V_before = last voxel, V_after = 0 (a
        // folded exit was taken in the loop, and vprev is then the border's 0)
        if (amax_ax == e1) {
            A1s += vprev;
            B1 = fma(amax, (double)vprev, B1);
        } else if (amax_ax == e2) {
            A2s += vprev;
            B2 = fma(amax, (double)vprev, B2);
        } else if (amax_ax < 0) {
            Ac += vprev;
            Bc = amax * (double)vprev;
        }
        const float Ad = -(A1s + A2s + Ac);
        const float Bd = (float)(acc - B1 - B2 - Bc);
        r.a0 = derived == 0 ? Ad : A1s;
        r.b0 = derived == 0 ? Bd : (float)B1;
        r.a1 = derived == 0 ? A1s : (derived == 1 ? Ad : A2s);
        r.b1 = derived == 0 ? (float)B1 : (derived == 1 ? Bd : (float)B2);
        r.a2 = derived == 2 ? Ad : A2s;
        r.b2 = derived == 2 ? Bd : (float)B2;
    }
    return r;
}

// d E / d pose for one ray from its traversal sums (frozen voxel indices).
//   E = L * sum_k alpha_k (V_{k-1} - V_k),  alpha_k = (q_k - s_c) / d_c,
//   d alpha_k = -(s'_c + alpha_k d'_c) / d_c,  d L = dhat . d'
//   => dE = g_d . d' + g_s . s'  with  g_s = -L A / d,
//      g_d = sum * d / L - L B / d   (per axis c; axes with d_c = 0 drop out)
// The pose enters through s' and d' = p' - s', with R = Z Y X (the three
// elementary rotations), c = (-2 rho, u, v) and e_x fixed by X:
//   theta:  g_d . Z'Y X c + rho g_s . Z'Y e_x
//   phi:    g_d . Z Y'X c + rho g_s . Z Y'e_x
//   gamma:  g_d . Z Y X'c           (X' e_x = 0)
//   t_c:    g_s[c]
//   sdd:    (g_s / 2 - g_d) . Z Y e_x
// evaluated as row-vector x matrix products so that no 3 x 3 matrix is
// held in registers.
//
// With `Jp`, also the derivatives with respect to the detector's pitch and
// principal-point offset: the pixel moves by R e_y (w + 1/2 - W/2) per unit
// delta_x, R e_z (h + 1/2 - H/2) per unit delta_y, R e_y per unit offset_u
// and R e_z per unit offset_v, the source not at all, so dE = g_d . d' with
// R e_y = Z Y (0, cg, sg), R e_z = Z Y (0, -sg, cg); ku, kv are the factors.
__device__ inline void ray_jacobian(const RayAcc& r, const PoseTrig& q, double u, double v,
                                    float J[7], float* Jp = nullptr, double ku = 0.0,
                                    double kv = 0.0)
{
    const double ct = q.ct, st = q.st, cp = q.cp, sp = q.sp, cg = q.cg, sg = q.sg;
    // X c with c = (-2 rho, u, v); X' c
    const double c0 = -2.0 * q.rho;
    const double xc1 = cg * u - sg * v, xc2 = sg * u + cg * v;
    const double dxc1 = -sg * u - cg * v, dxc2 = cg * u - sg * v;
    // Y (X c), Y' (X c), Y e_x, Y' e_x, Y (X' c)
    const double yx0 = cp * c0 + sp * xc2, yx1 = xc1, yx2 = -sp * c0 + cp * xc2;
    const double dyx0 = -sp * c0 + cp * xc2, dyx2 = -cp * c0 - sp * xc2;
    const double ye0 = cp, ye2 = -sp;
    const double dye0 = -sp, dye2 = -cp;
    const double ydx0 = sp * dxc2, ydx1 = dxc1, ydx2 = cp * dxc2;
    // ray direction d = Z Y X c
    double d[3];
    d[0] = ct * yx0 - st * yx1;
    d[1] = st * yx0 + ct * yx1;
    d[2] = yx2;
    const double L = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double A[3], B[3];
    A[0] = r.a0;
    A[1] = r.a1;
    A[2] = r.a2;
    B[0] = r.b0;
    B[1] = r.b1;
    B[2] = r.b2;
    double gs[3], gd[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double Bc = B[c];
        if (d[c] != 0.0) {
            gs[c] = -L * A[c] / d[c];
            gd[c] = r.sum * d[c] / L - L * Bc / d[c];
        } else {
            gs[c] = 0.0;
            gd[c] = 0.0;
        }
    }
    // row vectors g Z and g Z' (for g_s only the first components: it meets
    // only Y e_x and Y' e_x, whose second component is zero)
    const double gdz0 = gd[0] * ct + gd[1] * st, gdz1 = -gd[0] * st + gd[1] * ct;
    const double gsz0 = gs[0] * ct + gs[1] * st;
    const double gdzd0 = -gd[0] * st + gd[1] * ct, gdzd1 = -gd[0] * ct - gd[1] * st;
    const double gszd0 = -gs[0] * st + gs[1] * ct;
    // (Z' has a zero third row, Z keeps the third component)
    J[0] = (float)(gdzd0 * yx0 + gdzd1 * yx1 + q.rho * (gszd0 * ye0));
    J[1] = (float)(gdz0 * dyx0 + gd[2] * dyx2 + q.rho * (gsz0 * dye0 + gs[2] * dye2));
    J[2] = (float)(gdz0 * ydx0 + gdz1 * ydx1 + gd[2] * ydx2);
    J[3] = (float)gs[0];
    J[4] = (float)gs[1];
    J[5] = (float)gs[2];
    J[6] = (float)((0.5 * gsz0 - gdz0) * ye0 + (0.5 * gs[2] - gd[2]) * ye2);
    if (Jp) {
        const double gu = gdz0 * sp * sg + gdz1 * cg + gd[2] * cp * sg;   // g_d . R e_y
        const double gv = gdz0 * sp * cg - gdz1 * sg + gd[2] * cp * cg;   // g_d . R e_z
        Jp[0] = (float)(ku * gu);
        Jp[1] = (float)(kv * gv);
        Jp[2] = (float)gu;
        Jp[3] = (float)gv;
    }
}

// Hides a pointer's provenance from the optimiser, so that values loaded
// through it are recomputed rather than kept alive from earlier loads.
template <typename T>
__device__ inline T* launder(T* p)
{
    asm volatile("" : "+v"(p));
    return p;
}

// The descriptor must live in scalar registers.  Where the volume arguments
// were read from memory (plan item tables) the compiler cannot prove them
// wave-uniform and would wrap every gather in a loop over distinct
// descriptors; reading the fields through readfirstlane states that they are.
__device__ inline __amdgpu_buffer_rsrc_t make_rsrc(const VolArgs& V, int copy)
{
    const uint64_t addr = (uint64_t)V.packed + (uint64_t)copy * V.copy_bytes;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)addr);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(addr >> 32));
    const int nrec = __builtin_amdgcn_readfirstlane((int)V.copy_bytes);
    const char* base = (const char*)(((uint64_t)hi << 32) | lo);
    return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, nrec, (int)kBufferDword3);
}

// Maps the hardware workgroup id to a logical one so that the workgroups
// that land on one XCD (dispatch is round-robin over the 8 XCDs) take a
// contiguous range of logical ids, i.e. neighbouring tiles of one pose.
__device__ inline uint32_t xcd_logical(uint32_t bid, uint32_t total)
{
    const uint32_t per = total / 8u, rem = total % 8u;
    const uint32_t xcd = bid % 8u, local = bid / 8u;
    return xcd < rem ? xcd * (per + 1u) + local : rem * (per + 1u) + (xcd - rem) * per + local;
}

// ------------------------------------------------------------------ reductions

__device__ inline double wave_sum(double x)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

}  // namespace drr
