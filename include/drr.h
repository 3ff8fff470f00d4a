/*
 * drr.h -- C ABI of the MI355X (gfx950) Siddon DRR library, libdrr.so.
 *
 * Method: Gopalakrishnan & Golland, "Fast Auto-Differentiable Digitally
 * Reconstructed Radiographs for Solving Inverse Problems in Intraoperative
 * Imaging" (arXiv:2208.12737).  A digitally reconstructed radiograph (DRR)
 * pixel is the radiological path of Eq. 2: the length-weighted sum of the
 * CT voxel attenuations along the ray from the X-ray source s to the pixel p,
 * with the segment boundaries given by the ray's crossings of the CT grid
 * planes (Eq. 3) taken in increasing order (Eq. 4; Siddon-Jacobs order,
 * Sec. 2.2).  Poses are the rotation/translation/distance parameters of
 * Sec. 2.4; gradients are those of Sec. 2.4 (voxel indices held fixed).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Pointers named as device pointers must point to device memory of the
 *    current HIP device; host pointers (descriptors, item tables) are read
 *    during the call only.  The caller owns every buffer it passes.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Calls only enqueue work on it and return; a device fault surfaces as a
 *    HIP error at the caller's next synchronisation.
 *  - Return value: DRR_OK (0) or a negative DRR_E* code; nothing throws across
 *    the ABI.  drr_last_error() returns a thread-local message for the last
 *    failing call of the calling thread.
 *  - No call allocates device memory except drr_plan_create.  Calls that need
 *    scratch memory take a caller-provided device workspace and report its
 *    required size through a *_workspace_bytes query; too small a workspace
 *    gives DRR_ENOMEM and enqueues nothing.  drr_render_ncc_grad_noalloc
 *    uses a fixed device array of the library instead.
 *  - Results are deterministic: per-pose reductions use a fixed order, so the
 *    same inputs give bitwise the same outputs, independent of batch size,
 *    batch composition and of which other work shares the GPU.
 *  - Pose contents are not validated: a non-finite pose yields NaN pixels.  A
 *    ray that misses the volume yields 0.  Voxel values must be finite: the
 *    traversal reads a few voxels past each ray's exit and weights them by
 *    zero, so an infinite voxel can turn unrelated pixels into NaN.
 *
 * Geometry (Sec. 2.4; reading of the paper's spherical parameterisation):
 *   pose = float[7] = {theta, phi, gamma, tx, ty, tz, sdd} (radians, mm).
 *   R = Rz(theta) * Ry(phi) * Rx(gamma), rho = sdd / 2.
 *   source       s      = R * ( rho, 0,   0  ) + t
 *   pixel (h, w) p(h,w) = R * (-rho, u_w, v_h) + t
 *   u_w = (w + 1/2 - W/2) * delta_x + offset_u,
 *   v_h = (h + 1/2 - H/2) * delta_y + offset_v.
 *   Images are row-major [pose][h][w] float32.
 *
 * Volume (Sec. 2.2): nx * ny * nz voxels of size spacing[0..2] (mm), plane 0
 * of axis c at origin[c] (the paper's b_x, b_y, b_z); the caller's array is
 * C-order float32 V[(i * ny + j) * nz + k].
 */
#ifndef DRR_H
#define DRR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DRR_OK 0
#define DRR_EINVAL (-1)   /* bad argument: NULL pointer, size <= 0, non-finite descriptor */
#define DRR_ENOMEM (-2)   /* caller workspace too small, or plan allocation failed */
#define DRR_EHIP (-3)     /* HIP runtime error (launch, copy, graph) */
#define DRR_ENOTSUP (-4)  /* unsupported size: a packed volume copy of 4 GiB or more (the
                             gathers use 32-bit byte offsets), a detector of more than
                             2^30 pixels, or more than 2^31 - 1 tiles in one launch */

/* Memory layouts of the packed volume.  Both hold the voxels surrounded by a
 * one-voxel border of zeros and give bitwise identical renders; they differ
 * in speed only.
 *   DRR_LAYOUT_INPUT     one copy in the caller's order (z fastest).
 *   DRR_LAYOUT_PER_AXIS  three copies, one per principal ray axis: a pose
 *                        whose central ray runs mostly along axis c reads the
 *                        copy whose fastest-varying memory axis is the
 *                        finer-spaced of the two other axes, so that the
 *                        rays of neighbouring detector pixels gather from
 *                        shared cache lines.  Three times the memory. */
#define DRR_LAYOUT_INPUT 0
#define DRR_LAYOUT_PER_AXIS 1

typedef struct drr_volume_desc {
    int32_t nx, ny, nz;   /* voxels per axis, each >= 1 */
    double spacing[3];    /* voxel size per axis, mm, > 0 */
    double origin[3];     /* position of plane 0 per axis, mm (centred grid: -n*spacing/2) */
    int32_t layout;       /* DRR_LAYOUT_* of the packed copy */
} drr_volume_desc;

typedef struct drr_detector_desc {
    int32_t height, width; /* H rows, W columns, each >= 1 */
    double delta_x;        /* column pitch (along w), mm, > 0 */
    double delta_y;        /* row pitch (along h), mm, > 0 */
    double offset_u;       /* principal-point offset along w, mm, finite (usually 0) */
    double offset_v;       /* principal-point offset along h, mm, finite (usually 0) */
} drr_detector_desc;

/* ---------------------------------------------------------------- volume */

/* Bytes of the packed, render-ready copy of a volume in the descriptor's
 * layout.  Returns 0 for an invalid or unsupported descriptor. */
size_t drr_volume_packed_bytes(const drr_volume_desc* vol);

/* Packs the caller's C-order float32 volume `src` (device, nx*ny*nz floats)
 * into `packed` (device, drr_volume_packed_bytes bytes).  The packed copy is
 * what every render call reads; it is immutable afterwards and may be shared
 * by concurrent calls. */
int32_t drr_volume_pack(const float* src, void* packed, const drr_volume_desc* vol,
                        void* stream);

/* ---------------------------------------------------------------- render */

/* Forward DRRs (Eq. 2-4) for n_poses poses.
 *   packed   device, from drr_volume_pack
 *   poses    device float[n_poses][7]
 *   image    device float[n_poses][H][W]            (output)
 *   jac      device float[n_poses][H][W][7] or NULL (output): d image / d pose,
 *            the frozen-voxel-index derivative of Sec. 2.4.
 * n_poses == 0 is a no-op. */
int32_t drr_render(const void* packed, const drr_volume_desc* vol, const drr_detector_desc* det,
                   const float* poses, int32_t n_poses, float* image, float* jac,
                   void* stream);

/* Forward DRRs plus the derivative of every pixel with respect to the
 * detector's intrinsic parameters (the paper notes gradients with respect to
 * the pixel spacing exist, Sec. 3.2):
 *   jac_det  device float[n_poses][H][W][4]
 *            = d image / d (delta_x, delta_y, offset_u, offset_v)
 * (frozen voxel indices, as for the pose Jacobian).  These parameters move
 * the pixel, not the source. */
int32_t drr_render_detector_jacobian(const void* packed, const drr_volume_desc* vol,
                                     const drr_detector_desc* det, const float* poses,
                                     int32_t n_poses, float* image, float* jac_det,
                                     void* stream);

/* Forward DRRs plus, per pixel, the number of positive-length segments
 * (= voxel gathers) the ray made: counts device int32[n_poses][H][W]. */
int32_t drr_render_count(const void* packed, const drr_volume_desc* vol,
                         const drr_detector_desc* det, const float* poses, int32_t n_poses,
                         float* image, int32_t* counts, void* stream);

/* Workspace (bytes) needed by the pose-gradient reductions below. */
size_t drr_backward_workspace_bytes(const drr_detector_desc* det, int32_t n_poses);

/* Pose gradient from a stored Jacobian (Sec. 2.4, chain rule):
 *   grad_pose[b][j] = sum_{h,w} grad_image[b][h][w] * jac[b][h][w][j]
 *   jac         device float[n_poses][H][W][7] (from drr_render)
 *   grad_image  device float[n_poses][H][W]
 *   grad_pose   device float[n_poses][7] (output, overwritten)
 *   workspace   device, drr_backward_workspace_bytes(det, n_poses) bytes */
int32_t drr_render_backward(const drr_detector_desc* det, int32_t n_poses, const float* jac,
                            const float* grad_image, float* grad_pose, void* workspace,
                            size_t workspace_bytes, void* stream);

/* Same gradient without a stored Jacobian: the rays are traced again and
 * each pixel's Jacobian row is contracted with grad_image on the fly. */
int32_t drr_render_backward_retrace(const void* packed, const drr_volume_desc* vol,
                                    const drr_detector_desc* det, const float* poses,
                                    int32_t n_poses, const float* grad_image, float* grad_pose,
                                    void* workspace, size_t workspace_bytes, void* stream);

/* ---------------------------------------------------------------- NCC loss */

/* Negative zero-normalised cross-correlation (Sec. 3.2) per pose, over all
 * H*W pixels, with population standard deviations:
 *   Z_b = (1/N) sum_i (I_i - mean I)(T_i - mean T) / (std I * std T),
 *   loss[b] = -Z_b.
 *   image, target  device float[n_poses][hw] (target may be shared by passing
 *                  target_stride = 0, else target_stride = hw)
 *   stats          device double[n_poses][5] (output): mean I, std I, mean T,
 *                  std T, Z -- consumed by drr_ncc_backward
 *   loss           device float[n_poses] (output)
 * A constant image or target gives NaN. */
size_t drr_ncc_workspace_bytes(int32_t n_poses, int64_t hw);
int32_t drr_ncc_forward(const float* image, const float* target, int64_t target_stride,
                        int32_t n_poses, int64_t hw, double* stats, float* loss,
                        void* workspace, size_t workspace_bytes, void* stream);

/* grad_image[b][i] = grad_loss[b] * d loss_b / d image[b][i]
 *                  = -grad_loss[b] * (That_i - Z_b Ihat_i) / (N std I). */
int32_t drr_ncc_backward(const float* image, const float* target, int64_t target_stride,
                         const double* stats, const float* grad_loss, int32_t n_poses,
                         int64_t hw, float* grad_image, void* stream);

/* Fused registration objective: one tracing pass renders each pose, forms
 * the negative ZNCC against its target and returns the loss and its pose
 * gradient, without storing the image Jacobian.
 *   target   device float[n_poses][H][W] (target_stride = H*W) or one shared
 *            image (target_stride = 0)
 *   image    device float[n_poses][H][W] or NULL (output)
 *   loss     device float[n_poses] (output), grad_pose device float[n_poses][7]
 *   workspace device, drr_ncc_grad_workspace_bytes(det, n_poses) bytes */
size_t drr_ncc_grad_workspace_bytes(const drr_detector_desc* det, int32_t n_poses);
int32_t drr_render_ncc_grad(const void* packed, const drr_volume_desc* vol,
                            const drr_detector_desc* det, const float* poses, int32_t n_poses,
                            const float* target, int64_t target_stride, float* image,
                            float* loss, float* grad_pose, void* workspace,
                            size_t workspace_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * fused objective as drr_render_ncc_grad, with the same arguments and
 * results (bitwise), except that its scratch is a fixed device array of
 * DRR_NOALLOC_SCRATCH_BYTES inside the library, one per GPU, kept until the
 * process ends.  The call allocates nothing (no hipMalloc, no library
 * allocation); its first call on a device only looks up that array's
 * address.  Batches whose drr_ncc_grad_workspace_bytes(det, n_poses) exceeds
 * DRR_NOALLOC_SCRATCH_BYTES return DRR_ENOMEM and enqueue nothing (at the
 * direct launch shape, 256 x 256-pixel poses take 53 248 bytes each, so up
 * to 157 of them fit).  Every call on one GPU shares that GPU's array: calls
 * whose work overlaps on the device (other streams, other threads) race and
 * must be serialized by the caller; a call on one stream after another is
 * safe.  Nothing in the array needs clearing between calls. */
#define DRR_NOALLOC_SCRATCH_BYTES (8u << 20)
int32_t drr_render_ncc_grad_noalloc(const void* packed, const drr_volume_desc* vol,
                                    const drr_detector_desc* det, const float* poses,
                                    int32_t n_poses, const float* target, int64_t target_stride,
                                    float* image, float* loss, float* grad_pose, void* stream);

/* Loss only (no gradient), e.g. for sweeps of the loss landscape (Sec. 3.2):
 * one tracing pass renders each pose and reduces the five ZNCC moments per
 * tile; loss[b] = -ZNCC(image_b, target_b).  Arguments as for
 * drr_render_ncc_grad; workspace: drr_ncc_loss_workspace_bytes bytes. */
size_t drr_ncc_loss_workspace_bytes(const drr_detector_desc* det, int32_t n_poses);
int32_t drr_render_ncc_loss(const void* packed, const drr_volume_desc* vol,
                            const drr_detector_desc* det, const float* poses, int32_t n_poses,
                            const float* target, int64_t target_stride, float* image,
                            float* loss, void* workspace, size_t workspace_bytes, void* stream);

/* Fused L2 objective, the alternative image loss of Sec. 3.2 (the paper
 * reports loss landscapes like those of the negative ZNCC for it): one
 * tracing pass renders each pose and returns
 *   loss[b]        = (1/N) sum_i (image_b[i] - target_b[i])^2,  N = H*W
 *   grad_pose[b][j] = (2/N) sum_i (image_b[i] - target_b[i]) d image_b[i] / d pose_j
 * without storing the image Jacobian.  grad_pose may be NULL: then only the
 * loss is formed, in a pass that computes no Jacobian.  Other arguments as
 * for drr_render_ncc_grad; workspace: drr_l2_workspace_bytes bytes (enough
 * for either form).  NaN poses give NaN losses. */
size_t drr_l2_workspace_bytes(const drr_detector_desc* det, int32_t n_poses);
int32_t drr_render_l2(const void* packed, const drr_volume_desc* vol,
                      const drr_detector_desc* det, const float* poses, int32_t n_poses,
                      const float* target, int64_t target_stride, float* image, float* loss,
                      float* grad_pose, void* workspace, size_t workspace_bytes, void* stream);

/* Gradient descent with momentum on the poses (Sec. 3.2, registration):
 *   velocity <- momentum * velocity + grad_pose
 *   poses    <- poses - rate .* velocity
 * poses, velocity, grad_pose, rate: device float[n_poses][7] (rate holds the
 * per-problem, per-parameter step sizes; a zero rate freezes a parameter). */
int32_t drr_pose_momentum_step(float* poses, float* velocity, const float* grad_pose,
                               const float* rate, float momentum, int32_t n_poses,
                               void* stream);

/* ---------------------------------------------------------------- plans */

/* A plan batches heterogeneous render work -- any mix of resident volumes,
 * detector sizes and poses, rendering images, Jacobians, gather counts or
 * the fused -ZNCC objective -- into one execute: per output group, a
 * persistent launch whose workgroups pull ray tiles from device queues, or
 * one workgroup per tile (DRR_PLAN_* below).  With use_graph the launches
 * are captured into HIP graphs and replayed; the tile shape and occupancy
 * are fixed or chosen by an autotuner (timed candidates, cached on disk when
 * a cache path is given). */

#define DRR_ITEM_JAC 1      /* also write the Jacobian to item.jac */
#define DRR_ITEM_COUNT 2    /* also write per-pixel gather counts to item.counts */
#define DRR_ITEM_NCC 4      /* fused objective: -ZNCC against item.target and its pose
                               gradient, as drr_render_ncc_grad (no Jacobian stored) */

typedef struct drr_work_item {
    int32_t volume;          /* index into the plan's volume table */
    int32_t flags;           /* DRR_ITEM_*; at most one of JAC, COUNT, NCC */
    drr_detector_desc det;
    const float* pose;       /* device float[7] */
    float* image;            /* device float[H][W]; may be NULL for DRR_ITEM_NCC */
    float* jac;              /* device float[H][W][7] when DRR_ITEM_JAC */
    int32_t* counts;         /* device int32[H][W] when DRR_ITEM_COUNT */
    const float* target;     /* device float[H][W] when DRR_ITEM_NCC */
    float* loss;             /* device float[1] when DRR_ITEM_NCC: -ZNCC */
    float* grad;             /* device float[7] when DRR_ITEM_NCC: d loss / d pose */
    double* partials;        /* device scratch of drr_plan_item_workspace_bytes(&det)
                                bytes when DRR_ITEM_NCC, private to the item until
                                the execute completes */
} drr_work_item;

/* Scratch bytes a DRR_ITEM_NCC item needs for its detector (enough for any
 * launch shape the plan may use); 0 for an invalid detector. */
size_t drr_plan_item_workspace_bytes(const drr_detector_desc* det);

typedef struct drr_plan_desc {
    int32_t max_items;                   /* capacity of one execute call */
    int32_t n_volumes;
    const drr_volume_desc* volumes;      /* host array [n_volumes] */
    const void* const* packed;           /* host array of device pointers [n_volumes] */
    int32_t use_graph;                   /* 1: capture the launch in a HIP graph */
    int32_t autotune;                    /* 1: time candidate launch shapes at create */
    const char* tune_cache_path;         /* NULL or a file for autotune results */
    int32_t strategy;                    /* without autotune: DRR_PLAN_* (-1 = default:
                                            DRR_PLAN_AUTO) */
    int32_t tile_code;                   /* without autotune: launch shape (-1 = default: 4,
                                            16 x 16-pixel tiles of 4 x 16-pixel waves) */
    int32_t wg_per_cu;                   /* without autotune: resident workgroups per CU
                                            (-1 = default: 4; 0 = as many as registers
                                            allow) */
} drr_plan_desc;

/* Plan strategies: a persistent grid sized to the GPU whose workgroups pull
 * tiles from per-XCD device queues (one graph serves any batch), or one
 * workgroup per tile (the graph is re-captured when the tile count of a
 * batch changes), or, per output group of each execute, the flat grid when
 * the group has no more tiles than the persistent grid has workgroups and
 * the queues otherwise (small batches start sooner; large ones keep the
 * queues' balance under concurrent executes). */
#define DRR_PLAN_PERSISTENT 0
#define DRR_PLAN_FLAT 1
#define DRR_PLAN_AUTO 2

typedef struct drr_plan drr_plan;

/* Creates a plan (allocates its device item tables and, when autotuning,
 * runs timed candidates of the persistent and flat strategies on `stream`
 * using tune_items, at least one item, as the sample work; without
 * autotuning tune_items is ignored and may be NULL). */
int32_t drr_plan_create(const drr_plan_desc* desc, const drr_work_item* tune_items,
                        int32_t n_tune_items, void* stream, drr_plan** out);

/* Enqueues the items on `stream`.  Items are independent; their results are
 * identical to rendering each alone.  The host table is copied before the
 * call returns.  Calls on one plan are serialized by a lock inside it. */
int32_t drr_plan_execute(drr_plan* plan, const drr_work_item* items, int32_t n_items,
                         void* stream);

/* Chosen launch: strategy, tile code and workgroups per CU (for reports). */
int32_t drr_plan_config(const drr_plan* plan, int32_t* strategy, int32_t* tile_code,
                        int32_t* wg_per_cu, int32_t* use_graph);

void drr_plan_destroy(drr_plan* plan);

/* ---------------------------------------------------------------- misc */

/* Resident workgroups per CU for the direct render entry points (those not
 * going through a plan); 0 = as many as registers allow; -1 (default) = 4,
 * which trades occupancy for cache locality of the voxel gathers.
 * Process-wide; affects launches enqueued after the call. */
int32_t drr_set_launch_occupancy(int32_t wg_per_cu);

const char* drr_status_string(int32_t status);
const char* drr_last_error(void);
int32_t drr_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DRR_H */
