// Streaming reductions and elementwise kernels around the renderer:
// per-pose sums of tile partials, the stored-Jacobian pose gradient, the
// ZNCC moments / loss / image gradient, and the momentum pose update.
// Every reduction has a fixed summation order (no atomics), so results are
// bitwise reproducible and independent of what else is in the batch.
#pragma once

#include "reduce_common.hpp"

namespace drr {

constexpr int kChunkPixels = 1024;   // pixels per workgroup in streaming kernels

// Sums partials[b][0..n)[0..NS) over the middle index for pose b = blockIdx.x
// into lds row 0, in a fixed order.
template <int NS>
__device__ inline void sum_partials(const double* __restrict__ partials, int n, double* lds)
{
    sum_tile_partials<NS>(partials + (int64_t)blockIdx.x * n * NS, n, lds);
}

// grad_pose[b][j] = sum of partials (7 values per tile).
__global__ __launch_bounds__(kReduceThreads) void k_grad_finalize(const double* partials, int n,
                                                                  float* grad_pose)
{
    __shared__ double lds[kReduceThreads * 7];
    sum_partials<7>(partials, n, lds);
    if ((int)threadIdx.x < 7) grad_pose[blockIdx.x * 7 + threadIdx.x] = (float)lds[threadIdx.x];
}

// Loss and pose gradient of -ZNCC from the fused tile sums.
//   Z = cov(I, T) / (std I std T), loss = -Z
//   d loss / d pose = -1/(N std I) [ (S_TJ - mean T S_J) / std T
//                                    - Z (S_IJ - mean I S_J) / std I ]
__global__ __launch_bounds__(kReduceThreads) void k_ncc_grad_finalize(const double* partials,
                                                                      int n, double npix,
                                                                      float* loss,
                                                                      float* grad_pose)
{
    __shared__ double lds[kReduceThreads * kNccSums];
    sum_partials<kNccSums>(partials, n, lds);
    ncc_from_sums(lds, npix, loss + blockIdx.x, grad_pose + blockIdx.x * 7);
}

// Loss only, from fused tile sums (I, I^2, T, T^2, IT): loss[b] = -Z.
__global__ __launch_bounds__(kReduceThreads) void k_ncc_loss_finalize(const double* partials,
                                                                      int n, double npix,
                                                                      float* loss)
{
    __shared__ double lds[kReduceThreads * 5];
    sum_partials<5>(partials, n, lds);
    if (threadIdx.x == 0) {
        const double* S = lds;
        const double mi = S[0] / npix, mt = S[2] / npix;
        const double si = sqrt(fmax(S[1] / npix - mi * mi, 0.0));
        const double st = sqrt(fmax(S[3] / npix - mt * mt, 0.0));
        loss[blockIdx.x] = (float)(-(S[4] / npix - mi * mt) / (si * st));
    }
}

// Mean squared difference and its pose gradient from the fused tile sums
// ((I-T)^2 and, with NS = 8, (I-T) J[7]):
//   loss = S_0 / N,  d loss / d pose_j = 2 S_{1+j} / N.
template <int NS>
__global__ __launch_bounds__(kReduceThreads) void k_l2_finalize(const double* partials, int n,
                                                                double npix, float* loss,
                                                                float* grad_pose)
{
    __shared__ double lds[kReduceThreads * NS];
    sum_partials<NS>(partials, n, lds);
    const int j = threadIdx.x;
    if (j == 0) loss[blockIdx.x] = (float)(lds[0] / npix);
    if (NS == 8 && j < 7) grad_pose[blockIdx.x * 7 + j] = (float)(2.0 * lds[1 + j] / npix);
}

// Stored-Jacobian contraction: partial[b][chunk][j] = sum g * jac over the chunk.
__global__ __launch_bounds__(kReduceThreads) void k_jac_dot(const float* __restrict__ jac,
                                                            const float* __restrict__ g,
                                                            int64_t hw, int chunks,
                                                            double* partials)
{
    __shared__ double lds[7 * (kReduceThreads / 64)];
    const int b = blockIdx.y, c = blockIdx.x;
    const int64_t p0 = (int64_t)c * kChunkPixels;
    double vals[7];
#pragma unroll
    for (int j = 0; j < 7; ++j) vals[j] = 0.0;
    for (int k = 0; k < kChunkPixels / kReduceThreads; ++k) {
        const int64_t p = p0 + k * kReduceThreads + threadIdx.x;
        if (p < hw) {
            const double gv = g[(int64_t)b * hw + p];
            const float* jp = jac + ((int64_t)b * hw + p) * 7;
#pragma unroll
            for (int j = 0; j < 7; ++j) vals[j] += gv * (double)jp[j];
        }
    }
    block_sums<7, kReduceThreads / 64>(vals, lds, partials + ((int64_t)b * chunks + c) * 7);
}

// ZNCC moments per chunk: sum I, I^2, T, T^2, I T.
__global__ __launch_bounds__(kReduceThreads) void k_ncc_moments(const float* __restrict__ img,
                                                                const float* __restrict__ tgt,
                                                                int64_t tstride, int64_t hw,
                                                                int chunks, double* partials)
{
    __shared__ double lds[5 * (kReduceThreads / 64)];
    const int b = blockIdx.y, c = blockIdx.x;
    const int64_t p0 = (int64_t)c * kChunkPixels;
    double vals[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < kChunkPixels / kReduceThreads; ++k) {
        const int64_t p = p0 + k * kReduceThreads + threadIdx.x;
        if (p < hw) {
            const double I = img[(int64_t)b * hw + p];
            const double T = tgt[(int64_t)b * tstride + p];
            vals[0] += I;
            vals[1] += I * I;
            vals[2] += T;
            vals[3] += T * T;
            vals[4] += I * T;
        }
    }
    block_sums<5, kReduceThreads / 64>(vals, lds, partials + ((int64_t)b * chunks + c) * 5);
}

// stats[b] = (mean I, std I, mean T, std T, Z); loss[b] = -Z.
__global__ __launch_bounds__(kReduceThreads) void k_ncc_stats(const double* partials, int n,
                                                              double npix, double* stats,
                                                              float* loss)
{
    __shared__ double lds[kReduceThreads * 5];
    sum_partials<5>(partials, n, lds);
    if (threadIdx.x == 0) {
        const double* S = lds;
        const double mi = S[0] / npix, mt = S[2] / npix;
        const double si = sqrt(fmax(S[1] / npix - mi * mi, 0.0));
        const double st = sqrt(fmax(S[3] / npix - mt * mt, 0.0));
        const double z = (S[4] / npix - mi * mt) / (si * st);
        double* o = stats + (int64_t)blockIdx.x * 5;
        o[0] = mi;
        o[1] = si;
        o[2] = mt;
        o[3] = st;
        o[4] = z;
        loss[blockIdx.x] = (float)(-z);
    }
}

// grad_image = grad_loss * d(-Z)/dI = -grad_loss (That - Z Ihat) / (N std I).
__global__ __launch_bounds__(kReduceThreads) void k_ncc_backward(
    const float* __restrict__ img, const float* __restrict__ tgt, int64_t tstride,
    const double* __restrict__ stats, const float* __restrict__ gl, int64_t hw, double npix,
    float* __restrict__ out)
{
    const int b = blockIdx.y;
    const int64_t p = (int64_t)blockIdx.x * kReduceThreads + threadIdx.x;
    if (p >= hw) return;
    const double* st = stats + (int64_t)b * 5;
    const double ih = ((double)img[(int64_t)b * hw + p] - st[0]) / st[1];
    const double th = ((double)tgt[(int64_t)b * tstride + p] - st[2]) / st[3];
    out[(int64_t)b * hw + p] = (float)(-(double)gl[b] * (th - st[4] * ih) / (npix * st[1]));
}

// Heavy-ball step: v <- m v + g; pose <- pose - rate .* v.
__global__ void k_momentum(float* __restrict__ poses, float* __restrict__ vel,
                           const float* __restrict__ grad, const float* __restrict__ rate,
                           float m, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float v = m * vel[i] + grad[i];
    vel[i] = v;
    poses[i] = poses[i] - rate[i] * v;
}

// Copies a C-order volume into one zero-bordered copy whose memory order is
// (o0 slowest, o1, o2 fastest) over the padded dims P.
__global__ void k_pack(const float* __restrict__ src, float* __restrict__ dst, int nx, int ny,
                       int nz, int o0, int o1, int o2, uint64_t total)
{
    const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    const uint64_t P[3] = {(uint64_t)nx + 2, (uint64_t)ny + 2, (uint64_t)nz + 2};
    uint64_t idx[3];
    idx[o2] = e % P[o2];
    idx[o1] = (e / P[o2]) % P[o1];
    idx[o0] = e / (P[o2] * P[o1]);
    const int i = (int)idx[0], j = (int)idx[1], k = (int)idx[2];
    float v = 0.0f;
    if (i >= 1 && i <= nx && j >= 1 && j <= ny && k >= 1 && k <= nz)
        v = src[((uint64_t)(i - 1) * ny + (j - 1)) * nz + (k - 1)];
    dst[e] = v;
}

}  // namespace drr
