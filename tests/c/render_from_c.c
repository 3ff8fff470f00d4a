/* A plain C consumer of libdrr (no Python, no torch): reads a volume, poses
 * and a detector from files, renders through the C ABI and writes the
 * images, the fused -ZNCC losses and pose gradients.  Used by
 * tests/test_gpu_c_consumer.py.
 *
 * usage: render_from_c <dir>   with, in <dir>:
 *   meta.txt    nx ny nz sx sy sz ox oy oz H W dx dy n_poses
 *   volume.f32  nx*ny*nz float32 (C order)
 *   poses.f32   n_poses*7 float32
 *   target.f32  H*W float32 (one shared target)
 * writes image.f32 (n*H*W), loss.f32 (n), grad.f32 (n*7). */
#define __HIP_PLATFORM_AMD__ 1
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "drr.h"

#define CHECK_HIP(x)                                                     \
    do {                                                                 \
        hipError_t e_ = (x);                                             \
        if (e_ != hipSuccess) {                                          \
            fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));      \
            return 2;                                                    \
        }                                                                \
    } while (0)
#define CHECK_DRR(x)                                                     \
    do {                                                                 \
        int32_t s_ = (x);                                                \
        if (s_ != DRR_OK) {                                              \
            fprintf(stderr, "%s: %s\n", #x, drr_last_error());          \
            return 3;                                                    \
        }                                                                \
    } while (0)

static void* read_file(const char* dir, const char* name, size_t bytes)
{
    char path[1024];
    snprintf(path, sizeof path, "%s/%s", dir, name);
    FILE* f = fopen(path, "rb");
    if (!f) return NULL;
    void* buf = malloc(bytes);
    if (buf && fread(buf, 1, bytes, f) != bytes) {
        free(buf);
        buf = NULL;
    }
    fclose(f);
    return buf;
}

static int write_file(const char* dir, const char* name, const void* buf, size_t bytes)
{
    char path[1024];
    snprintf(path, sizeof path, "%s/%s", dir, name);
    FILE* f = fopen(path, "wb");
    if (!f) return 1;
    size_t w = fwrite(buf, 1, bytes, f);
    fclose(f);
    return w == bytes ? 0 : 1;
}

int main(int argc, char** argv)
{
    if (argc != 2) return 1;
    const char* dir = argv[1];
    char path[1024];
    snprintf(path, sizeof path, "%s/meta.txt", dir);
    FILE* m = fopen(path, "r");
    if (!m) return 1;
    drr_volume_desc vol;
    drr_detector_desc det;
    int n = 0;
    memset(&vol, 0, sizeof vol);
    memset(&det, 0, sizeof det);
    if (fscanf(m, "%d %d %d %lf %lf %lf %lf %lf %lf %d %d %lf %lf %d", &vol.nx, &vol.ny,
               &vol.nz, &vol.spacing[0], &vol.spacing[1], &vol.spacing[2], &vol.origin[0],
               &vol.origin[1], &vol.origin[2], &det.height, &det.width, &det.delta_x,
               &det.delta_y, &n) != 14) {
        fclose(m);
        return 1;
    }
    fclose(m);
    vol.layout = DRR_LAYOUT_PER_AXIS;
    const size_t nvox = (size_t)vol.nx * vol.ny * vol.nz, hw = (size_t)det.height * det.width;
    float* h_vol = (float*)read_file(dir, "volume.f32", nvox * 4);
    float* h_pose = (float*)read_file(dir, "poses.f32", (size_t)n * 7 * 4);
    float* h_tgt = (float*)read_file(dir, "target.f32", hw * 4);
    if (!h_vol || !h_pose || !h_tgt) return 1;

    hipStream_t st;
    CHECK_HIP(hipStreamCreate(&st));
    const size_t packed_bytes = drr_volume_packed_bytes(&vol);
    const size_t ws_bytes = drr_ncc_grad_workspace_bytes(&det, n);
    if (packed_bytes == 0 || ws_bytes == 0) return 3;
    float *d_src, *d_pose, *d_img, *d_tgt, *d_loss, *d_grad;
    void *d_packed, *d_ws;
    CHECK_HIP(hipMalloc((void**)&d_src, nvox * 4));
    CHECK_HIP(hipMalloc(&d_packed, packed_bytes));
    CHECK_HIP(hipMalloc((void**)&d_pose, (size_t)n * 7 * 4));
    CHECK_HIP(hipMalloc((void**)&d_img, (size_t)n * hw * 4));
    CHECK_HIP(hipMalloc((void**)&d_tgt, hw * 4));
    CHECK_HIP(hipMalloc((void**)&d_loss, (size_t)n * 4));
    CHECK_HIP(hipMalloc((void**)&d_grad, (size_t)n * 7 * 4));
    CHECK_HIP(hipMalloc(&d_ws, ws_bytes));
    CHECK_HIP(hipMemcpy(d_src, h_vol, nvox * 4, hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(d_pose, h_pose, (size_t)n * 7 * 4, hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(d_tgt, h_tgt, hw * 4, hipMemcpyHostToDevice));

    CHECK_DRR(drr_volume_pack(d_src, d_packed, &vol, st));
    CHECK_DRR(drr_render(d_packed, &vol, &det, d_pose, n, d_img, NULL, st));
    CHECK_DRR(drr_render_ncc_grad(d_packed, &vol, &det, d_pose, n, d_tgt, 0, NULL, d_loss,
                                  d_grad, d_ws, ws_bytes, st));
    CHECK_HIP(hipStreamSynchronize(st));

    float* h_img = (float*)malloc((size_t)n * hw * 4);
    float h_loss[4096], h_grad[4096 * 7];
    if (!h_img || n > 4096) return 1;
    CHECK_HIP(hipMemcpy(h_img, d_img, (size_t)n * hw * 4, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(h_loss, d_loss, (size_t)n * 4, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(h_grad, d_grad, (size_t)n * 7 * 4, hipMemcpyDeviceToHost));
    if (write_file(dir, "image.f32", h_img, (size_t)n * hw * 4) ||
        write_file(dir, "loss.f32", h_loss, (size_t)n * 4) ||
        write_file(dir, "grad.f32", h_grad, (size_t)n * 7 * 4))
        return 1;
    hipFree(d_src);
    hipFree(d_packed);
    hipFree(d_pose);
    hipFree(d_img);
    hipFree(d_tgt);
    hipFree(d_loss);
    hipFree(d_grad);
    hipFree(d_ws);
    hipStreamDestroy(st);
    free(h_vol);
    free(h_pose);
    free(h_tgt);
    free(h_img);
    return 0;
}
