// C-ABI entry points of libdrr.so (declared in include/drr.h): volume
// packing, forward render, Jacobian / retrace pose gradients, ZNCC loss and
// the fused registration objective.  Host code here validates arguments and
// enqueues kernels; it never allocates device memory.
#include <string.h>

#include <atomic>
#include <mutex>

#include "common.hpp"
#include "reduce_kernels.hpp"

namespace drr {

static thread_local char g_err[512] = "";

int32_t fail(int32_t code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

int32_t check_launch(const char* what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(DRR_EHIP, "%s: %s", what, hipGetErrorString(e));
    return DRR_OK;
}

// Launch shape of the direct (non-plan) entry points (kDirectShape).  Fewer
// resident workgroups per CU than the register file allows keep the gather
// working set inside the L1/L2 caches; the limit is imposed by reserving LDS
// per workgroup (default 4 workgroups = 4 waves per SIMD).
constexpr int kTW = kDirectShape.tw, kWX = kDirectShape.wx, kWY = kDirectShape.wy;
using DefaultShape = TileShape<kTW, kWX, kWY>;

// -1: the default, 4 resident workgroups per CU: with 4 x 16-pixel waves in
// 16 x 16-pixel tiles it was the fastest setting for the image and the fused
// gradient modes on the 512 x 512 x 133 CT workload (fewer resident rays keep
// their gathers' lines in the 32 KB L1)
// set by drr_set_launch_occupancy, read by every direct launch (any thread)
static std::atomic<int> g_wg_per_cu{-1};

static int wg_per_cu_for(const drr_volume_desc& vol)
{
    (void)vol;
    const int w = g_wg_per_cu.load(std::memory_order_relaxed);
    return w >= 0 ? w : 4;
}

struct FlatGrid {
    int tiles_x, tiles_y, wg_per_pose;
};

static FlatGrid flat_grid(const drr_detector_desc& d)
{
    FlatGrid g;
    g.tiles_x = (d.width + DefaultShape::px_w - 1) / DefaultShape::px_w;
    g.tiles_y = (d.height + DefaultShape::px_h - 1) / DefaultShape::px_h;
    g.wg_per_pose = g.tiles_x * g.tiles_y;
    return g;
}

// Static LDS of render_flat<kTW, kWX, kWY, MODE> (its block-sum buffer).
template <int MODE>
static constexpr size_t flat_static_lds()
{
    return tile_sum_lds_bytes(ModeTraits<MODE>::nsum, kWX * kWY);
}

template <int MODE>
static int32_t launch_flat(const void* packed, const drr_volume_desc& vol,
                           const drr_detector_desc& det, const float* poses, int32_t n_poses,
                           float* image, float* jac, int32_t* counts, const float* aux,
                           int64_t aux_stride, double* partials, hipStream_t stream)
{
    const FlatGrid g = flat_grid(det);
    const uint64_t blocks = (uint64_t)g.wg_per_pose * (uint64_t)n_poses;
    if (blocks > 0x7FFFFFFFull) return fail(DRR_ENOTSUP, "too many tiles in one launch");
    // launches of up to 16 workgroups per CU (16 poses of 256 x 256 pixels)
    // take the deep pipeline in every mode: measured faster down to a lone
    // wave per SIMD, where it cuts a single DRR's time by a third; launches
    // of at most one workgroup per CU (a single DRR of up to 256 x 256
    // pixels) leave each SIMD one wave and take the deepest pipeline
    const uint64_t cus = (uint64_t)num_cus();
    if constexpr (MODE == kImage || MODE == kCount) {
        // per-pixel results that do not depend on the launch shape: a launch
        // of at most one workgroup per CU uses 8 x 8-pixel waves (16 x 16
        // pixels per workgroup), whose rays gather from fewer cache lines per
        // step than 4 x 16-pixel waves; it left a lone wave per SIMD either way
        using TS = TileShape<8, 2, 2>;
        const int tx = (det.width + TS::px_w - 1) / TS::px_w;
        const uint64_t tb = (uint64_t)tx * (uint64_t)((det.height + TS::px_h - 1) / TS::px_h) *
                            (uint64_t)n_poses;
        if (tb <= cus) {
            hipLaunchKernelGGL((render_flat<8, 2, 2, MODE, kTinyDepth>), dim3((unsigned)tb),
                               dim3(TS::threads), 0, stream, vol_args(packed, vol), det_args(det),
                               poses, tx, (int)(tb / (uint64_t)n_poses), image, jac, counts, aux,
                               aux_stride, partials);
            return check_launch("render kernel launch");
        }
    }
    auto kernel = blocks <= cus ? render_flat<kTW, kWX, kWY, MODE, kTinyDepth>
                  : blocks <= 16ull * cus ? render_flat<kTW, kWX, kWY, MODE, kDeepDepth>
                                          : render_flat<kTW, kWX, kWY, MODE, full_depth<MODE>()>;
    hipLaunchKernelGGL(kernel, dim3((unsigned)blocks),
                       dim3(DefaultShape::threads),
                       occupancy_lds(wg_per_cu_for(vol), flat_static_lds<MODE>()), stream,
                       vol_args(packed, vol),
                       det_args(det), poses, g.tiles_x, g.wg_per_pose, image, jac, counts, aux,
                       aux_stride, partials);
    return check_launch("render kernel launch");
}

static size_t chunks_of(int64_t hw) { return (size_t)((hw + kChunkPixels - 1) / kChunkPixels); }

// Scratch of drr_render_ncc_grad_noalloc: file-scope device memory, one copy
// on each GPU the library runs on, held until the process ends.  Host code
// must not pass `scratch` itself to a kernel (on the host it names a
// stand-in, not a device address): its device address is looked up once per
// device with hipGetSymbolAddress and kept in g_scratch_ptr.
static_assert(DRR_NOALLOC_SCRATCH_BYTES % sizeof(double) == 0, "scratch holds doubles");
static __device__ __align__(256) double scratch[DRR_NOALLOC_SCRATCH_BYTES / sizeof(double)];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];   // device address of `scratch`, per device

// Device address of `scratch` on the current device (looked up on the first
// call on that device, with the device current).
static int32_t scratch_on_current_device(void** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(DRR_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(DRR_ENOTSUP, "device %d: at most %d devices", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(DRR_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                        hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return DRR_OK;
}

}  // namespace drr

using namespace drr;

extern "C" {

const char* drr_last_error(void) { return g_err; }

int32_t drr_version(void) { return 10000; }

int32_t drr_set_launch_occupancy(int32_t wg_per_cu)
{
    if (wg_per_cu < -1 || wg_per_cu > 64)
        return fail(DRR_EINVAL, "set_launch_occupancy: %d outside [-1, 64]", wg_per_cu);
    g_wg_per_cu.store(wg_per_cu, std::memory_order_relaxed);
    return DRR_OK;
}

const char* drr_status_string(int32_t s)
{
    switch (s) {
    case DRR_OK: return "ok";
    case DRR_EINVAL: return "invalid argument";
    case DRR_ENOMEM: return "workspace too small or allocation failed";
    case DRR_EHIP: return "HIP runtime error";
    case DRR_ENOTSUP: return "unsupported size";
    default: return "unknown status";
    }
}

size_t drr_volume_packed_bytes(const drr_volume_desc* vol)
{
    if (validate_volume(vol) != DRR_OK) return 0;
    return (size_t)(packed_elems(*vol) * 4ull);
}

int32_t drr_volume_pack(const float* src, void* packed, const drr_volume_desc* vol, void* stream)
{
    int32_t st = validate_volume(vol);
    if (st) return st;
    if (!src || !packed) return fail(DRR_EINVAL, "volume_pack: NULL pointer");
    const uint64_t total = copy_elems(*vol);
    const unsigned blocks = (unsigned)((total + 255) / 256);
    for (int q = 0; q < num_copies(*vol); ++q) {
        const CopyOrder o = copy_order(*vol, q);
        hipLaunchKernelGGL(k_pack, dim3(blocks), dim3(256), 0, as_stream(stream), src,
                           (float*)packed + q * total, vol->nx, vol->ny, vol->nz, o.axis[0],
                           o.axis[1], o.axis[2], total);
        st = check_launch("volume_pack");
        if (st) return st;
    }
    return DRR_OK;
}

static int32_t common_render_checks(const void* packed, const drr_volume_desc* vol,
                                    const drr_detector_desc* det, const float* poses,
                                    int32_t n_poses)
{
    int32_t st = validate_volume(vol);
    if (st) return st;
    st = validate_detector(det);
    if (st) return st;
    if (n_poses < 0) return fail(DRR_EINVAL, "n_poses must be >= 0 (got %d)", n_poses);
    if (n_poses > 0 && (!packed || !poses)) return fail(DRR_EINVAL, "NULL volume or poses");
    return DRR_OK;
}

int32_t drr_render(const void* packed, const drr_volume_desc* vol, const drr_detector_desc* det,
                   const float* poses, int32_t n_poses, float* image, float* jac, void* stream)
{
    int32_t st = common_render_checks(packed, vol, det, poses, n_poses);
    if (st) return st;
    if (n_poses == 0) return DRR_OK;
    if (!image) return fail(DRR_EINVAL, "render: image is NULL");
    if (jac)
        return launch_flat<kJac>(packed, *vol, *det, poses, n_poses, image, jac, nullptr, nullptr,
                                 0, nullptr, as_stream(stream));
    return launch_flat<kImage>(packed, *vol, *det, poses, n_poses, image, nullptr, nullptr,
                               nullptr, 0, nullptr, as_stream(stream));
}

int32_t drr_render_detector_jacobian(const void* packed, const drr_volume_desc* vol,
                                     const drr_detector_desc* det, const float* poses,
                                     int32_t n_poses, float* image, float* jac_det,
                                     void* stream)
{
    int32_t st = common_render_checks(packed, vol, det, poses, n_poses);
    if (st) return st;
    if (n_poses == 0) return DRR_OK;
    if (!image || !jac_det) return fail(DRR_EINVAL, "render_detector_jacobian: NULL output");
    return launch_flat<kJacDet>(packed, *vol, *det, poses, n_poses, image, jac_det, nullptr,
                                nullptr, 0, nullptr, as_stream(stream));
}

int32_t drr_render_count(const void* packed, const drr_volume_desc* vol,
                         const drr_detector_desc* det, const float* poses, int32_t n_poses,
                         float* image, int32_t* counts, void* stream)
{
    int32_t st = common_render_checks(packed, vol, det, poses, n_poses);
    if (st) return st;
    if (n_poses == 0) return DRR_OK;
    if (!image || !counts) return fail(DRR_EINVAL, "render_count: NULL output");
    return launch_flat<kCount>(packed, *vol, *det, poses, n_poses, image, nullptr, counts,
                               nullptr, 0, nullptr, as_stream(stream));
}

size_t drr_backward_workspace_bytes(const drr_detector_desc* det, int32_t n_poses)
{
    if (validate_detector(det) != DRR_OK || n_poses < 0) return 0;
    const int64_t hw = (int64_t)det->height * det->width;
    size_t per = chunks_of(hw);
    size_t tiles = (size_t)flat_grid(*det).wg_per_pose;
    if (tiles > per) per = tiles;
    return per * (size_t)n_poses * 7 * sizeof(double);
}

int32_t drr_render_backward(const drr_detector_desc* det, int32_t n_poses, const float* jac,
                            const float* grad_image, float* grad_pose, void* workspace,
                            size_t workspace_bytes, void* stream)
{
    int32_t st = validate_detector(det);
    if (st) return st;
    if (n_poses < 0) return fail(DRR_EINVAL, "n_poses must be >= 0");
    if (n_poses == 0) return DRR_OK;
    if (!jac || !grad_image || !grad_pose || !workspace)
        return fail(DRR_EINVAL, "render_backward: NULL pointer");
    if (workspace_bytes < drr_backward_workspace_bytes(det, n_poses))
        return fail(DRR_ENOMEM, "render_backward: workspace of %zu bytes, need %zu",
                    workspace_bytes, drr_backward_workspace_bytes(det, n_poses));
    const int64_t hw = (int64_t)det->height * det->width;
    const int chunks = (int)chunks_of(hw);
    hipStream_t s = as_stream(stream);
    hipLaunchKernelGGL(k_jac_dot, dim3(chunks, n_poses), dim3(kReduceThreads), 0, s, jac,
                       grad_image, hw, chunks, (double*)workspace);
    if ((st = check_launch("jac_dot"))) return st;
    hipLaunchKernelGGL(k_grad_finalize, dim3(n_poses), dim3(kReduceThreads), 0, s,
                       (const double*)workspace, chunks, grad_pose);
    return check_launch("grad_finalize");
}

int32_t drr_render_backward_retrace(const void* packed, const drr_volume_desc* vol,
                                    const drr_detector_desc* det, const float* poses,
                                    int32_t n_poses, const float* grad_image, float* grad_pose,
                                    void* workspace, size_t workspace_bytes, void* stream)
{
    int32_t st = common_render_checks(packed, vol, det, poses, n_poses);
    if (st) return st;
    if (n_poses == 0) return DRR_OK;
    if (!grad_image || !grad_pose || !workspace)
        return fail(DRR_EINVAL, "render_backward_retrace: NULL pointer");
    if (workspace_bytes < drr_backward_workspace_bytes(det, n_poses))
        return fail(DRR_ENOMEM, "render_backward_retrace: workspace too small");
    const int64_t hw = (int64_t)det->height * det->width;
    hipStream_t s = as_stream(stream);
    st = launch_flat<kRetrace>(packed, *vol, *det, poses, n_poses, nullptr, nullptr, nullptr,
                               grad_image, hw, (double*)workspace, s);
    if (st) return st;
    hipLaunchKernelGGL(k_grad_finalize, dim3(n_poses), dim3(kReduceThreads), 0, s,
                       (const double*)workspace, flat_grid(*det).wg_per_pose, grad_pose);
    return check_launch("grad_finalize");
}

size_t drr_ncc_workspace_bytes(int32_t n_poses, int64_t hw)
{
    if (n_poses < 0 || hw < 1) return 0;
    return chunks_of(hw) * (size_t)n_poses * 5 * sizeof(double);
}

int32_t drr_ncc_forward(const float* image, const float* target, int64_t target_stride,
                        int32_t n_poses, int64_t hw, double* stats, float* loss,
                        void* workspace, size_t workspace_bytes, void* stream)
{
    if (n_poses < 0 || hw < 2) return fail(DRR_EINVAL, "ncc_forward: n_poses >= 0, hw >= 2");
    if (target_stride != 0 && target_stride != hw)
        return fail(DRR_EINVAL, "ncc_forward: target_stride must be 0 or hw");
    if (n_poses == 0) return DRR_OK;
    if (!image || !target || !stats || !loss || !workspace)
        return fail(DRR_EINVAL, "ncc_forward: NULL pointer");
    if (workspace_bytes < drr_ncc_workspace_bytes(n_poses, hw))
        return fail(DRR_ENOMEM, "ncc_forward: workspace too small");
    const int chunks = (int)chunks_of(hw);
    hipStream_t s = as_stream(stream);
    hipLaunchKernelGGL(k_ncc_moments, dim3(chunks, n_poses), dim3(kReduceThreads), 0, s, image,
                       target, target_stride, hw, chunks, (double*)workspace);
    int32_t st = check_launch("ncc_moments");
    if (st) return st;
    hipLaunchKernelGGL(k_ncc_stats, dim3(n_poses), dim3(kReduceThreads), 0, s,
                       (const double*)workspace, chunks, (double)hw, stats, loss);
    return check_launch("ncc_stats");
}

int32_t drr_ncc_backward(const float* image, const float* target, int64_t target_stride,
                         const double* stats, const float* grad_loss, int32_t n_poses,
                         int64_t hw, float* grad_image, void* stream)
{
    if (n_poses < 0 || hw < 2) return fail(DRR_EINVAL, "ncc_backward: n_poses >= 0, hw >= 2");
    if (target_stride != 0 && target_stride != hw)
        return fail(DRR_EINVAL, "ncc_backward: target_stride must be 0 or hw");
    if (n_poses == 0) return DRR_OK;
    if (!image || !target || !stats || !grad_loss || !grad_image)
        return fail(DRR_EINVAL, "ncc_backward: NULL pointer");
    const unsigned bx = (unsigned)((hw + kReduceThreads - 1) / kReduceThreads);
    hipLaunchKernelGGL(k_ncc_backward, dim3(bx, n_poses), dim3(kReduceThreads), 0,
                       as_stream(stream), image, target, target_stride, stats, grad_loss, hw,
                       (double)hw, grad_image);
    return check_launch("ncc_backward");
}

size_t drr_ncc_grad_workspace_bytes(const drr_detector_desc* det, int32_t n_poses)
{
    if (validate_detector(det) != DRR_OK || n_poses < 0) return 0;
    return (size_t)flat_grid(*det).wg_per_pose * (size_t)n_poses * kNccSums * sizeof(double);
}

int32_t drr_render_ncc_grad(const void* packed, const drr_volume_desc* vol,
                            const drr_detector_desc* det, const float* poses, int32_t n_poses,
                            const float* target, int64_t target_stride, float* image,
                            float* loss, float* grad_pose, void* workspace,
                            size_t workspace_bytes, void* stream)
{
    int32_t st = common_render_checks(packed, vol, det, poses, n_poses);
    if (st) return st;
    const int64_t hw = (int64_t)det->height * det->width;
    if (target_stride != 0 && target_stride != hw)
        return fail(DRR_EINVAL, "render_ncc_grad: target_stride must be 0 or H*W");
    if (hw < 2) return fail(DRR_EINVAL, "render_ncc_grad: need at least 2 pixels");
    if (n_poses == 0) return DRR_OK;
    if (!target || !loss || !grad_pose || !workspace)
        return fail(DRR_EINVAL, "render_ncc_grad: NULL pointer");
    if (workspace_bytes < drr_ncc_grad_workspace_bytes(det, n_poses))
        return fail(DRR_ENOMEM, "render_ncc_grad: workspace too small");
    hipStream_t s = as_stream(stream);
    st = launch_flat<kNcc>(packed, *vol, *det, poses, n_poses, image, nullptr, nullptr, target,
                           target_stride, (double*)workspace, s);
    if (st) return st;
    hipLaunchKernelGGL(k_ncc_grad_finalize, dim3(n_poses), dim3(kReduceThreads), 0, s,
                       (const double*)workspace, flat_grid(*det).wg_per_pose, (double)hw, loss,
                       grad_pose);
    return check_launch("ncc_grad_finalize");
}

int32_t drr_render_ncc_grad_noalloc(const void* packed, const drr_volume_desc* vol,
                                    const drr_detector_desc* det, const float* poses,
                                    int32_t n_poses, const float* target, int64_t target_stride,
                                    float* image, float* loss, float* grad_pose, void* stream)
{
    int32_t st = common_render_checks(packed, vol, det, poses, n_poses);
    if (st) return st;
    if (n_poses == 0) return DRR_OK;
    const size_t need = drr_ncc_grad_workspace_bytes(det, n_poses);
    if (need > (size_t)DRR_NOALLOC_SCRATCH_BYTES)
        return fail(DRR_ENOMEM,
                    "render_ncc_grad_noalloc: %d poses of %d x %d pixels need %zu bytes of "
                    "scratch, more than the fixed %zu; split the batch",
                    n_poses, det->height, det->width, need, (size_t)DRR_NOALLOC_SCRATCH_BYTES);
    void* ws = nullptr;
    if ((st = scratch_on_current_device(&ws))) return st;
    return drr_render_ncc_grad(packed, vol, det, poses, n_poses, target, target_stride, image,
                               loss, grad_pose, ws, DRR_NOALLOC_SCRATCH_BYTES, stream);
}

size_t drr_ncc_loss_workspace_bytes(const drr_detector_desc* det, int32_t n_poses)
{
    if (validate_detector(det) != DRR_OK || n_poses < 0) return 0;
    return (size_t)flat_grid(*det).wg_per_pose * (size_t)n_poses * 5 * sizeof(double);
}

int32_t drr_render_ncc_loss(const void* packed, const drr_volume_desc* vol,
                            const drr_detector_desc* det, const float* poses, int32_t n_poses,
                            const float* target, int64_t target_stride, float* image,
                            float* loss, void* workspace, size_t workspace_bytes, void* stream)
{
    int32_t st = common_render_checks(packed, vol, det, poses, n_poses);
    if (st) return st;
    const int64_t hw = (int64_t)det->height * det->width;
    if (target_stride != 0 && target_stride != hw)
        return fail(DRR_EINVAL, "render_ncc_loss: target_stride must be 0 or H*W");
    if (hw < 2) return fail(DRR_EINVAL, "render_ncc_loss: need at least 2 pixels");
    if (n_poses == 0) return DRR_OK;
    if (!target || !loss || !workspace) return fail(DRR_EINVAL, "render_ncc_loss: NULL pointer");
    if (workspace_bytes < drr_ncc_loss_workspace_bytes(det, n_poses))
        return fail(DRR_ENOMEM, "render_ncc_loss: workspace too small");
    hipStream_t s = as_stream(stream);
    st = launch_flat<kNccLoss>(packed, *vol, *det, poses, n_poses, image, nullptr, nullptr,
                               target, target_stride, (double*)workspace, s);
    if (st) return st;
    hipLaunchKernelGGL(k_ncc_loss_finalize, dim3(n_poses), dim3(kReduceThreads), 0, s,
                       (const double*)workspace, flat_grid(*det).wg_per_pose, (double)hw, loss);
    return check_launch("ncc_loss_finalize");
}

size_t drr_l2_workspace_bytes(const drr_detector_desc* det, int32_t n_poses)
{
    if (validate_detector(det) != DRR_OK || n_poses < 0) return 0;
    return (size_t)flat_grid(*det).wg_per_pose * (size_t)n_poses * 8 * sizeof(double);
}

int32_t drr_render_l2(const void* packed, const drr_volume_desc* vol,
                      const drr_detector_desc* det, const float* poses, int32_t n_poses,
                      const float* target, int64_t target_stride, float* image, float* loss,
                      float* grad_pose, void* workspace, size_t workspace_bytes, void* stream)
{
    int32_t st = common_render_checks(packed, vol, det, poses, n_poses);
    if (st) return st;
    const int64_t hw = (int64_t)det->height * det->width;
    if (target_stride != 0 && target_stride != hw)
        return fail(DRR_EINVAL, "render_l2: target_stride must be 0 or H*W");
    if (n_poses == 0) return DRR_OK;
    if (!target || !loss || !workspace) return fail(DRR_EINVAL, "render_l2: NULL pointer");
    if (workspace_bytes < drr_l2_workspace_bytes(det, n_poses))
        return fail(DRR_ENOMEM, "render_l2: workspace too small");
    hipStream_t s = as_stream(stream);
    const int tiles = flat_grid(*det).wg_per_pose;
    if (grad_pose) {
        st = launch_flat<kL2>(packed, *vol, *det, poses, n_poses, image, nullptr, nullptr, target,
                              target_stride, (double*)workspace, s);
        if (st) return st;
        hipLaunchKernelGGL(k_l2_finalize<8>, dim3(n_poses), dim3(kReduceThreads), 0, s,
                           (const double*)workspace, tiles, (double)hw, loss, grad_pose);
    } else {
        st = launch_flat<kL2Loss>(packed, *vol, *det, poses, n_poses, image, nullptr, nullptr,
                                  target, target_stride, (double*)workspace, s);
        if (st) return st;
        hipLaunchKernelGGL(k_l2_finalize<1>, dim3(n_poses), dim3(kReduceThreads), 0, s,
                           (const double*)workspace, tiles, (double)hw, loss, nullptr);
    }
    return check_launch("l2_finalize");
}

int32_t drr_pose_momentum_step(float* poses, float* velocity, const float* grad_pose,
                               const float* rate, float momentum, int32_t n_poses, void* stream)
{
    if (n_poses < 0) return fail(DRR_EINVAL, "n_poses must be >= 0");
    if (!isfinite(momentum)) return fail(DRR_EINVAL, "momentum must be finite");
    if (n_poses == 0) return DRR_OK;
    if (!poses || !velocity || !grad_pose || !rate)
        return fail(DRR_EINVAL, "pose_momentum_step: NULL pointer");
    const int n = n_poses * 7;
    hipLaunchKernelGGL(k_momentum, dim3((n + 255) / 256), dim3(256), 0, as_stream(stream), poses,
                       velocity, grad_pose, rate, momentum, n);
    return check_launch("pose_momentum_step");
}

}  // extern "C"
