// Gather-rate calibration for the voxel loads of the renderer.
//
// One 64-lane dword gather through a raw buffer descriptor, repeated: lane l
// reads word (l / k) % 32 of line (l % k) of a per-wave window, so that one
// load instruction touches exactly k distinct 128-byte lines.  The window
// advances by one line per instruction over `window_lines` lines (1: the same
// k lines every time, L1-resident; larger: L2 / Infinity Cache / HBM).  The
// time per instruction and CU against k is the ceiling that scattered 4-byte
// gathers can reach, whatever HBM bandwidth allows.
//
// Measurement tool only: not part of the rendering library.
#include <hip/hip_runtime.h>
#include <cstdint>

namespace {

__device__ inline float ldb(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}

__global__ __launch_bounds__(256) void gather_lines(const float* buf, uint32_t nbytes, int k,
                                                    int iters, int window_lines, float* out)
{
    const __amdgpu_buffer_rsrc_t r =
        __builtin_amdgcn_make_buffer_rsrc((void*)buf, (short)0, (int)nbytes, 0x00020000);
    const int lane = threadIdx.x & 63;
    const uint32_t wave = blockIdx.x * 4u + (threadIdx.x >> 6);
    const uint32_t lines = nbytes / 128u;
    // every line read below is < lines: base + 63 + window < lines
    const uint32_t base = (wave * 64u) % (lines - 64u - (uint32_t)window_lines);
    const uint32_t line0 = base + (uint32_t)(lane % k);
    const uint32_t word = (uint32_t)((lane / k) % 32);
    const uint32_t shift = window_lines > 1 ? 1u : 0u;
    float acc = 0.0f;
    uint32_t cur = 0;
    for (int it = 0; it < iters; it += 8) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            v[u] = ldb(r, (line0 + cur) * 128u + word * 4u);
            cur += shift;
            if (cur >= (uint32_t)window_lines) cur = 0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += v[u];
    }
    if (acc == 12345.0f) out[0] = acc;  // keeps the loads live; never true
}

}  // namespace

extern "C" {

// Times `reps` launches of `blocks` x 256 threads, each wave issuing `iters`
// (a multiple of 8) gathers that touch k lines each; writes the mean launch
// time in ms.  Allocates and frees its own 64 MiB buffer.  Returns 0, or a
// negative value on a HIP error or invalid argument.
int32_t gathercal_run(int32_t k, int32_t window_lines, int32_t iters, int32_t blocks,
                      int32_t reps, float* ms_out)
{
    if (k < 1 || k > 64 || window_lines < 1 || window_lines > 65536 || iters < 8 ||
        iters % 8 != 0 || blocks < 1 || reps < 1 || !ms_out)
        return -1;
    const uint32_t nbytes = 64u << 20;
    float* buf = nullptr;
    float* out = nullptr;
    if (hipMalloc(&buf, nbytes) != hipSuccess) return -2;
    if (hipMalloc(&out, sizeof(float)) != hipSuccess) {
        (void)hipFree(buf);
        return -2;
    }
    int32_t st = 0;
    hipEvent_t a = nullptr, b = nullptr;
    if (hipMemset(buf, 0, nbytes) != hipSuccess || hipEventCreate(&a) != hipSuccess ||
        hipEventCreate(&b) != hipSuccess)
        st = -3;
    if (st == 0) {
        hipLaunchKernelGGL(gather_lines, dim3(blocks), dim3(256), 0, 0, buf, nbytes, k, iters,
                           window_lines, out);
        (void)hipEventRecord(a, 0);
        for (int i = 0; i < reps; ++i)
            hipLaunchKernelGGL(gather_lines, dim3(blocks), dim3(256), 0, 0, buf, nbytes, k,
                               iters, window_lines, out);
        (void)hipEventRecord(b, 0);
        float ms = 0.0f;
        if (hipGetLastError() != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
            hipEventElapsedTime(&ms, a, b) != hipSuccess)
            st = -4;
        *ms_out = ms / (float)reps;
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    (void)hipFree(out);
    (void)hipFree(buf);
    return st;
}

// Peak shader clock of the current device in kHz (0 on error).
int32_t gathercal_clock_khz(void)
{
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeClockRate, dev) != hipSuccess) return 0;
    return khz;
}

}  // extern "C"
