// Host-side helpers shared by the C-ABI entry points: argument validation,
// the thread-local error message, and conversion of public descriptors into
// kernel argument blocks.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>

#include "../../include/drr.h"
#include "launch_budget.hpp"
#include "siddon.hpp"

namespace drr {

int32_t fail(int32_t code, const char* fmt, ...);
int32_t check_launch(const char* what);

inline bool finite_pos(double x) { return isfinite(x) && x > 0.0; }

// Largest packed volume the 32-bit buffer offsets can address.
constexpr uint64_t kMaxPackedBytes = 0xFFFFFF00ull;

// Elements of one zero-bordered copy of the grid.
inline uint64_t copy_elems(const drr_volume_desc& v)
{
    return (uint64_t)(v.nx + 2) * (uint64_t)(v.ny + 2) * (uint64_t)(v.nz + 2);
}

inline int num_copies(const drr_volume_desc& v)
{
    return v.layout == DRR_LAYOUT_PER_AXIS ? 3 : 1;
}

inline uint64_t packed_elems(const drr_volume_desc& v) { return copy_elems(v) * num_copies(v); }

// Memory order of copy q (slowest axis first).  DRR_LAYOUT_INPUT keeps the
// caller's (x, y, z).  DRR_LAYOUT_PER_AXIS: copy q serves rays running
// mostly along axis q; q is the slowest axis and, of the other two, the one
// with the finer spacing varies fastest.
struct CopyOrder {
    int axis[3];
};

inline CopyOrder copy_order(const drr_volume_desc& v, int q)
{
    CopyOrder o;
    if (v.layout != DRR_LAYOUT_PER_AXIS) {
        o.axis[0] = 0;
        o.axis[1] = 1;
        o.axis[2] = 2;
        return o;
    }
    const int a = (q + 1) % 3, b = (q + 2) % 3;
    const bool a_finer = v.spacing[a] < v.spacing[b] || (v.spacing[a] == v.spacing[b] && a > b);
    o.axis[0] = q;
    o.axis[1] = a_finer ? b : a;
    o.axis[2] = a_finer ? a : b;
    return o;
}

// Element pitch of each logical axis in copy q.
inline void copy_pitch(const drr_volume_desc& v, int q, int64_t pitch[3])
{
    const int64_t P[3] = {v.nx + 2, v.ny + 2, v.nz + 2};
    const CopyOrder o = copy_order(v, q);
    pitch[o.axis[2]] = 1;
    pitch[o.axis[1]] = P[o.axis[2]];
    pitch[o.axis[0]] = P[o.axis[2]] * P[o.axis[1]];
}

inline int32_t validate_volume(const drr_volume_desc* v)
{
    if (!v) return fail(DRR_EINVAL, "volume descriptor is NULL");
    if (v->nx < 1 || v->ny < 1 || v->nz < 1)
        return fail(DRR_EINVAL, "volume dims must be >= 1 (got %d x %d x %d)", v->nx, v->ny,
                    v->nz);
    for (int c = 0; c < 3; ++c) {
        if (!finite_pos(v->spacing[c]))
            return fail(DRR_EINVAL, "volume spacing[%d] must be finite and > 0", c);
        if (!isfinite(v->origin[c])) return fail(DRR_EINVAL, "volume origin[%d] is not finite", c);
    }
    if (v->layout != DRR_LAYOUT_INPUT && v->layout != DRR_LAYOUT_PER_AXIS)
        return fail(DRR_EINVAL, "unknown volume layout %d", v->layout);
    if (copy_elems(*v) * 4ull > kMaxPackedBytes)
        return fail(DRR_ENOTSUP, "packed volume copy of %llu bytes exceeds the 4 GiB buffer limit",
                    (unsigned long long)(copy_elems(*v) * 4ull));
    return DRR_OK;
}

inline int32_t validate_detector(const drr_detector_desc* d)
{
    if (!d) return fail(DRR_EINVAL, "detector descriptor is NULL");
    if (d->height < 1 || d->width < 1)
        return fail(DRR_EINVAL, "detector size must be >= 1 (got %d x %d)", d->height, d->width);
    if ((int64_t)d->height * d->width > (int64_t)1 << 30)
        return fail(DRR_ENOTSUP, "detector of %d x %d pixels is too large", d->height, d->width);
    if (!finite_pos(d->delta_x) || !finite_pos(d->delta_y))
        return fail(DRR_EINVAL, "detector pitch must be finite and > 0");
    if (!isfinite(d->offset_u) || !isfinite(d->offset_v))
        return fail(DRR_EINVAL, "detector offsets must be finite");
    return DRR_OK;
}

inline VolArgs vol_args(const void* packed, const drr_volume_desc& v)
{
    VolArgs a;
    a.packed = (const float*)packed;
    a.n[0] = v.nx;
    a.n[1] = v.ny;
    a.n[2] = v.nz;
    for (int c = 0; c < 3; ++c) {
        a.spacing[c] = v.spacing[c];
        a.origin[c] = v.origin[c];
    }
    a.copy_bytes = (uint32_t)(copy_elems(v) * 4ull);
    const int nc = num_copies(v);
    for (int q = 0; q < 3; ++q) {
        int64_t p[3];
        copy_pitch(v, q < nc ? q : 0, p);
        for (int c = 0; c < 3; ++c) a.pitch[q][c] = (int32_t)(p[c] * 4);
        a.copy_for[q] = q < nc ? q : 0;
    }
    return a;
}

inline DetArgs det_args(const drr_detector_desc& d)
{
    DetArgs a;
    a.H = d.height;
    a.W = d.width;
    a.dx = d.delta_x;
    a.dy = d.delta_y;
    a.ou = d.offset_u;
    a.ov = d.offset_v;
    return a;
}

inline hipStream_t as_stream(void* s) { return (hipStream_t)s; }

// Compute units of the device current at the first launch (queried once).
inline int num_cus()
{
    static const int n = [] {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) != hipSuccess) dev = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            v <= 0)
            v = 256;
        return v;
    }();
    return n;
}

// LDS per CU and per workgroup, queried once (thread-safe initialisation of
// a function-local static) on the device current at the first launch.
inline LdsLimits lds_limits()
{
    static const LdsLimits lim = [] {
        int dev = 0, v = 0, b = 0;
        if (hipGetDevice(&dev) != hipSuccess) dev = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) !=
                hipSuccess || v <= 0)
            v = 160 * 1024;
        if (hipDeviceGetAttribute(&b, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
                hipSuccess || b <= 0)
            b = 64 * 1024;
        return LdsLimits{(size_t)v, (size_t)(b < v ? b : v)};
    }();
    return lim;
}

// Dynamic LDS that caps residency at `wg_per_cu` workgroups per CU on this
// device (see occupancy_lds_bytes).
inline size_t occupancy_lds(int wg_per_cu, size_t static_bytes)
{
    return occupancy_lds_bytes(lds_limits(), wg_per_cu, static_bytes);
}

}  // namespace drr
