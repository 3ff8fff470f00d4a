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
#include "siddon.hpp"

namespace drr {

int32_t fail(int32_t code, const char* fmt, ...);
int32_t check_launch(const char* what);

inline bool finite_pos(double x) { return isfinite(x) && x > 0.0; }

// Largest packed volume the 32-bit buffer offsets can address.
constexpr uint64_t kMaxPackedBytes = 0xFFFFFF00ull;

inline uint64_t packed_elems(const drr_volume_desc& v)
{
    return (uint64_t)(v.nx + 2) * (uint64_t)(v.ny + 2) * (uint64_t)(v.nz + 2);
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
    if (packed_elems(*v) * 4ull > kMaxPackedBytes)
        return fail(DRR_ENOTSUP, "packed volume of %llu bytes exceeds the 4 GiB buffer limit",
                    (unsigned long long)(packed_elems(*v) * 4ull));
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
    a.bytes = (uint32_t)(packed_elems(v) * 4ull);
    return a;
}

inline DetArgs det_args(const drr_detector_desc& d)
{
    DetArgs a;
    a.H = d.height;
    a.W = d.width;
    a.dx = d.delta_x;
    a.dy = d.delta_y;
    return a;
}

inline hipStream_t as_stream(void* s) { return (hipStream_t)s; }

}  // namespace drr
