// Device helpers shared by the reduction kernels of the direct entry points
// and of plans: the fixed-order sum of per-tile moment rows and the -ZNCC
// loss and pose gradient computed from the summed moments.
#pragma once

#include "render_kernels.hpp"

namespace drr {

constexpr int kReduceThreads = 256;

// Sums base[0..n)[0..NS) over the first index into lds row 0, in a fixed
// order.
template <int NS>
__device__ inline void sum_tile_partials(const double* __restrict__ base, int n, double* lds)
{
    const int i = threadIdx.x;
    double acc[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) acc[k] = 0.0;
    for (int t = i; t < n; t += kReduceThreads)
#pragma unroll
        for (int k = 0; k < NS; ++k) acc[k] += base[(int64_t)t * NS + k];
#pragma unroll
    for (int k = 0; k < NS; ++k) lds[i * NS + k] = acc[k];
    __syncthreads();
    for (int stride = kReduceThreads / 2; stride >= 1; stride >>= 1) {
        if (i < stride)
#pragma unroll
            for (int k = 0; k < NS; ++k) lds[i * NS + k] += lds[(i + stride) * NS + k];
        __syncthreads();
    }
}

// -ZNCC and its pose gradient from the 26 summed tile moments S (threads
// 0..6 write grad[0..6], thread 0 the loss).
__device__ inline void ncc_from_sums(const double* S, double npix, float* loss, float* grad)
{
    if ((int)threadIdx.x < 7) {
        const double mi = S[0] / npix, mt = S[2] / npix;
        const double si = sqrt(fmax(S[1] / npix - mi * mi, 0.0));
        const double st = sqrt(fmax(S[3] / npix - mt * mt, 0.0));
        const double z = (S[4] / npix - mi * mt) / (si * st);
        const int j = threadIdx.x;
        const double tj = (S[12 + j] - mt * S[5 + j]) / st;
        const double ij = (S[19 + j] - mi * S[5 + j]) / si;
        grad[j] = (float)(-(tj - z * ij) / (npix * si));
        if (j == 0) *loss = (float)(-z);
    }
}

}  // namespace drr
