/*
 * FP64 reference implementation of Siddon's digitally reconstructed
 * radiograph (DRR) and of its pose derivatives.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU path is
 * checked against.  It is plain and slow on purpose: every ray builds the
 * complete list of its plane crossings and sorts it, exactly as the
 * vectorised formulation of Siddon's method describes, with no blocking,
 * no incremental traversal and no reuse between rays.  It shares no code,
 * header or constant with the HIP library, and only the test suite, the
 * package's smoke check and the CPU-baseline leg of the benchmark load it.
 *
 * What is followed (Gopalakrishnan & Golland, "Fast Auto-Differentiable
 * Digitally Reconstructed Radiographs ...", arXiv:2208.12737):
 *   - ray model R(alpha) = s + alpha (p - s), alpha in [0, 1]   (Sec. 2.1)
 *   - radiological path: E = |p - s| * sum_m (a_{m+1} - a_m) V[voxel at the
 *     segment midpoint]                                          (Eq. 2)
 *   - plane crossings alpha_x(i) = (b_x + i dX - s_x)/(p_x - s_x),
 *     i = 0..n_x, and likewise for y and z                      (Eq. 3)
 *   - alpha_min = max_c min(alpha_c(0), alpha_c(n_c)),
 *     alpha_max = min_c max(alpha_c(0), alpha_c(n_c))          (Sec. 2.3)
 *   - keep the crossings inside [alpha_min, alpha_max] and sort them
 *                                                        (Eq. 4, Sec. 2.3)
 *   - seven pose parameters: half source-to-detector distance, three
 *     rotations, three translations                              (Sec. 2.4)
 *   - derivatives of the DRR with the voxel indices held fixed, which is
 *     what automatic differentiation of the tensor pipeline yields, since
 *     floor/integer indexing carries no gradient                 (Sec. 2.4)
 *   - negative zero-normalised cross-correlation as the loss     (Sec. 3.2)
 *
 * Readings where the paper is silent (each listed in the design notes):
 *   - n_c + 1 planes per axis (i = 0..n_c); the bounds use alpha_c(n_c).
 *   - alpha_min / alpha_max are clamped to [0, 1] (the integral runs over
 *     [0, 1]); a ray with alpha_min >= alpha_max misses and gives E = 0.
 *   - p_c == s_c: the axis adds no crossings; the ray misses when s_c lies
 *     outside the half-open slab [b_c, b_c + n_c dC).
 *   - voxel of a segment: floor((x_c - b_c)/dC) at the segment midpoint,
 *     clamped to [0, n_c - 1]; cells are half-open.
 *   - the image stores E itself (no exponential, no normalisation).
 *   - geometry: with R = Rz(theta) Ry(phi) Rx(gamma) and rho = sdd/2, the
 *     source is R (rho, 0, 0) + t and detector pixel (h, w) is
 *     R (-rho, u_w, v_h) + t, u_w = (w + 1/2 - W/2) delta_x + offset_u,
 *     v_h = (h + 1/2 - H/2) delta_y + offset_v (offsets: the detector's
 *     principal point, 0 by default); the image is row-major [h][w].
 *   - pose vector order: (theta, phi, gamma, tx, ty, tz, sdd).
 *
 * Volume layout: C-order double array V[(i * ny + j) * nz + k], plane 0 of
 * axis c at origin[c].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MISS_NONE (-1)

/* ------------------------------------------------------------------ */
/* Geometry (Sec. 2.4)                                                 */
/* ------------------------------------------------------------------ */

static void mat_mul3(const double a[9], const double b[9], double c[9])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += a[3 * i + k] * b[3 * k + j];
            c[3 * i + j] = acc;
        }
}

static void rot_z(double t, double m[9], int deriv)
{
    double c = cos(t), s = sin(t);
    if (!deriv) {
        double r[9] = {c, -s, 0, s, c, 0, 0, 0, 1};
        memcpy(m, r, sizeof r);
    } else {
        double r[9] = {-s, -c, 0, c, -s, 0, 0, 0, 0};
        memcpy(m, r, sizeof r);
    }
}

static void rot_y(double t, double m[9], int deriv)
{
    double c = cos(t), s = sin(t);
    if (!deriv) {
        double r[9] = {c, 0, s, 0, 1, 0, -s, 0, c};
        memcpy(m, r, sizeof r);
    } else {
        double r[9] = {-s, 0, c, 0, 0, 0, -c, 0, -s};
        memcpy(m, r, sizeof r);
    }
}

static void rot_x(double t, double m[9], int deriv)
{
    double c = cos(t), s = sin(t);
    if (!deriv) {
        double r[9] = {1, 0, 0, 0, c, -s, 0, s, c};
        memcpy(m, r, sizeof r);
    } else {
        double r[9] = {0, 0, 0, 0, -s, -c, 0, c, -s};
        memcpy(m, r, sizeof r);
    }
}

/* R = Rz(theta) Ry(phi) Rx(gamma); which = -1 gives R, which = 0/1/2 gives
 * the derivative of R with respect to theta / phi / gamma. */
void orc_rotation(double theta, double phi, double gamma, int which, double R[9])
{
    double a[9], b[9], c[9], ab[9];
    rot_z(theta, a, which == 0);
    rot_y(phi, b, which == 1);
    rot_x(gamma, c, which == 2);
    mat_mul3(a, b, ab);
    mat_mul3(ab, c, R);
}

static void mat_vec3(const double m[9], const double v[3], double out[3])
{
    for (int i = 0; i < 3; ++i)
        out[i] = m[3 * i] * v[0] + m[3 * i + 1] * v[1] + m[3 * i + 2] * v[2];
}

/* Source position and the position of detector pixel (h, w). */
void orc_ray_endpoints(const double pose[7], int H, int W, double delta_x, double delta_y,
                       double off_u, double off_v, int h, int w, double s[3], double p[3])
{
    double R[9];
    orc_rotation(pose[0], pose[1], pose[2], -1, R);
    double rho = 0.5 * pose[6];
    double cs[3] = {rho, 0.0, 0.0};
    double cp[3] = {-rho, (w + 0.5 - 0.5 * W) * delta_x + off_u,
                    (h + 0.5 - 0.5 * H) * delta_y + off_v};
    double rs[3], rp[3];
    mat_vec3(R, cs, rs);
    mat_vec3(R, cp, rp);
    for (int c = 0; c < 3; ++c) {
        s[c] = rs[c] + pose[3 + c];
        p[c] = rp[c] + pose[3 + c];
    }
}

/* Analytic derivatives of s and p(h, w) with respect to the seven pose
 * parameters: ds[c * 7 + j] = d s_c / d pose_j, likewise dp. */
void orc_ray_endpoint_derivs(const double pose[7], int H, int W, double delta_x,
                             double delta_y, double off_u, double off_v, int h, int w,
                             double ds[21], double dp[21])
{
    double rho = 0.5 * pose[6];
    double cs[3] = {rho, 0.0, 0.0};
    double cp[3] = {-rho, (w + 0.5 - 0.5 * W) * delta_x + off_u,
                    (h + 0.5 - 0.5 * H) * delta_y + off_v};
    memset(ds, 0, 21 * sizeof(double));
    memset(dp, 0, 21 * sizeof(double));
    for (int a = 0; a < 3; ++a) {
        double dR[9], vs[3], vp[3];
        orc_rotation(pose[0], pose[1], pose[2], a, dR);
        mat_vec3(dR, cs, vs);
        mat_vec3(dR, cp, vp);
        for (int c = 0; c < 3; ++c) {
            ds[c * 7 + a] = vs[c];
            dp[c * 7 + a] = vp[c];
        }
    }
    for (int c = 0; c < 3; ++c) {
        ds[c * 7 + 3 + c] = 1.0;
        dp[c * 7 + 3 + c] = 1.0;
    }
    /* rho = sdd / 2 scales the canonical source (+rho) and detector (-rho) */
    double R[9], ex[3] = {1.0, 0.0, 0.0}, rx[3];
    orc_rotation(pose[0], pose[1], pose[2], -1, R);
    mat_vec3(R, ex, rx);
    for (int c = 0; c < 3; ++c) {
        ds[c * 7 + 6] = 0.5 * rx[c];
        dp[c * 7 + 6] = -0.5 * rx[c];
    }
}

/* ------------------------------------------------------------------ */
/* One ray: Eq. 2-4 with the crossing list built in full and sorted     */
/* ------------------------------------------------------------------ */

typedef struct {
    double alpha;
    int axis; /* 0, 1, 2 for a plane of that axis; -1 for a clamped end */
} crossing;

static int cmp_crossing(const void *a, const void *b)
{
    double x = ((const crossing *)a)->alpha, y = ((const crossing *)b)->alpha;
    return (x > y) - (x < y);
}

typedef struct {
    int n[3];
    double spacing[3];
    double origin[3];
    const double *vol;
} orc_grid;

/* Builds the sorted crossing list of the ray s -> p.  Returns the number of
 * entries (0 when the ray misses).  `list` must hold nx+ny+nz+5 entries. */
static int build_crossings(const orc_grid *g, const double s[3], const double p[3],
                           crossing *list)
{
    double d[3];
    for (int c = 0; c < 3; ++c) d[c] = p[c] - s[c];

    /* Bounds of Sec. 2.3, with the clamp to the ray's own [0, 1]. */
    double amin = 0.0, amax = 1.0;
    int amin_axis = -1, amax_axis = -1;
    for (int c = 0; c < 3; ++c) {
        if (d[c] == 0.0) {
            double lo = g->origin[c], hi = g->origin[c] + g->n[c] * g->spacing[c];
            if (!(s[c] >= lo && s[c] < hi)) return 0;
            continue;
        }
        double a0 = (g->origin[c] - s[c]) / d[c];
        double an = (g->origin[c] + g->n[c] * g->spacing[c] - s[c]) / d[c];
        double lo = a0 < an ? a0 : an;
        double hi = a0 < an ? an : a0;
        if (lo > amin) {
            amin = lo;
            amin_axis = c;
        }
        if (hi < amax) {
            amax = hi;
            amax_axis = c;
        }
    }
    if (!(amin < amax)) return 0;

    int m = 0;
    list[m].alpha = amin;
    list[m++].axis = amin_axis;
    list[m].alpha = amax;
    list[m++].axis = amax_axis;
    for (int c = 0; c < 3; ++c) {
        if (d[c] == 0.0) continue;
        for (int i = 0; i <= g->n[c]; ++i) {
            double a = (g->origin[c] + i * g->spacing[c] - s[c]) / d[c];
            if (a > amin && a < amax) {
                list[m].alpha = a;
                list[m++].axis = c;
            }
        }
    }
    qsort(list, (size_t)m, sizeof(crossing), cmp_crossing);
    return m;
}

/* Flat index of the voxel containing the midpoint of [a, b]. */
static int64_t midpoint_voxel(const orc_grid *g, const double s[3], const double d[3],
                              double a, double b)
{
    double mid = 0.5 * (a + b);
    int64_t idx[3];
    for (int c = 0; c < 3; ++c) {
        double x = s[c] + mid * d[c];
        double f = floor((x - g->origin[c]) / g->spacing[c]);
        int64_t i = (int64_t)f;
        if (f < 0.0) i = 0;
        if (f > g->n[c] - 1) i = g->n[c] - 1;
        idx[c] = i;
    }
    return (idx[0] * g->n[1] + idx[1]) * g->n[2] + idx[2];
}

/* E for one ray, plus the number of positive-length segments and a hash of
 * their voxel sequence (FNV-1a over the flat indices). */
static double trace_ray(const orc_grid *g, const double s[3], const double p[3],
                        crossing *list, int64_t *nseg, uint64_t *hash)
{
    double d[3];
    for (int c = 0; c < 3; ++c) d[c] = p[c] - s[c];
    double L = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    int m = build_crossings(g, s, p, list);
    double sum = 0.0;
    int64_t cnt = 0;
    uint64_t hsh = 1469598103934665603ULL;
    for (int k = 0; k + 1 < m; ++k) {
        double a = list[k].alpha, b = list[k + 1].alpha;
        if (!(b > a)) continue;
        int64_t v = midpoint_voxel(g, s, d, a, b);
        sum += (b - a) * g->vol[v];
        ++cnt;
        hsh = (hsh ^ (uint64_t)v) * 1099511628211ULL;
    }
    if (nseg) *nseg = cnt;
    if (hash) *hash = hsh;
    return L * sum;
}

/* Derivatives of E with respect to the endpoints s and p, with every voxel
 * index and the plane identity of every crossing held fixed.
 *
 * Writing E = L * sum_m (a_{m+1} - a_m) V_m as L * sum_k a_k (V_{k-1} - V_k)
 * (V before the first and after the last crossing is zero), and using
 * a_k = (q_k - s_c) / d_c for a crossing of a plane at q_k on axis c:
 *   d a_k / d s_c = -(1 - a_k) / d_c,   d a_k / d p_c = -a_k / d_c,
 *   d L / d s = -d / L,                 d L / d p = d / L.
 * A clamped end (alpha = 0 or 1) does not move. */
static void trace_ray_grad(const orc_grid *g, const double s[3], const double p[3],
                           crossing *list, double *E, double dEds[3], double dEdp[3])
{
    double d[3];
    for (int c = 0; c < 3; ++c) d[c] = p[c] - s[c];
    double L = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    for (int c = 0; c < 3; ++c) dEds[c] = dEdp[c] = 0.0;
    int m = build_crossings(g, s, p, list);
    if (m == 0) {
        *E = 0.0;
        return;
    }
    /* voxel value of every segment, zero-length ones included */
    double sum = 0.0;
    double per_s[3] = {0, 0, 0}, per_p[3] = {0, 0, 0};
    double v_prev = 0.0;
    for (int k = 0; k < m; ++k) {
        double v_next = 0.0;
        if (k + 1 < m) {
            int64_t v = midpoint_voxel(g, s, d, list[k].alpha, list[k + 1].alpha);
            v_next = g->vol[v];
            sum += (list[k + 1].alpha - list[k].alpha) * v_next;
        }
        double delta = v_prev - v_next;
        int c = list[k].axis;
        if (c >= 0) {
            double a = list[k].alpha;
            per_s[c] += delta * (-(1.0 - a) / d[c]);
            per_p[c] += delta * (-a / d[c]);
        }
        v_prev = v_next;
    }
    *E = L * sum;
    for (int c = 0; c < 3; ++c) {
        dEds[c] = -d[c] / L * sum + L * per_s[c];
        dEdp[c] = d[c] / L * sum + L * per_p[c];
    }
}

static void grid_from(orc_grid *g, const double *vol, const int32_t dims[3],
                      const double spacing[3], const double origin[3])
{
    for (int c = 0; c < 3; ++c) {
        g->n[c] = dims[c];
        g->spacing[c] = spacing[c];
        g->origin[c] = origin[c];
    }
    g->vol = vol;
}

/* ------------------------------------------------------------------ */
/* Exported entry points                                               */
/* ------------------------------------------------------------------ */

/* E, segment count and voxel-sequence hash for n arbitrary rays. */
void orc_trace_rays(const double *vol, const int32_t dims[3], const double spacing[3],
                    const double origin[3], const double *src /*[n][3]*/,
                    const double *dst /*[n][3]*/, int64_t n, double *E, int64_t *nseg,
                    uint64_t *hash, int nthreads)
{
    orc_grid g;
    grid_from(&g, vol, dims, spacing, origin);
    int cap = dims[0] + dims[1] + dims[2] + 5;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
    {
        crossing *list = (crossing *)malloc(sizeof(crossing) * (size_t)cap);
#pragma omp for schedule(dynamic, 64)
        for (int64_t r = 0; r < n; ++r) {
            int64_t c = 0;
            uint64_t h = 0;
            E[r] = trace_ray(&g, src + 3 * r, dst + 3 * r, list, &c, &h);
            if (nseg) nseg[r] = c;
            if (hash) hash[r] = h;
        }
        free(list);
    }
}

/* DRR images for n_poses poses: image[b][h][w] (double), optional segment
 * counts and voxel-sequence hashes of the same shape.  Rows are processed
 * in [row_begin, row_end) only (the rest of the image is left untouched),
 * so callers can evaluate a bounded sample of a large detector. */
void orc_render(const double *vol, const int32_t dims[3], const double spacing[3],
                const double origin[3], const double *poses /*[n][7]*/, int32_t n_poses,
                int32_t H, int32_t W, double delta_x, double delta_y, double off_u,
                double off_v, int32_t row_begin, int32_t row_end, double *image,
                int64_t *nseg, uint64_t *hash, int nthreads)
{
    orc_grid g;
    grid_from(&g, vol, dims, spacing, origin);
    int cap = dims[0] + dims[1] + dims[2] + 5;
    if (row_begin < 0) row_begin = 0;
    if (row_end > H) row_end = H;
    int64_t rows = row_end > row_begin ? row_end - row_begin : 0;
    int64_t total = (int64_t)n_poses * rows * W;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
    {
        crossing *list = (crossing *)malloc(sizeof(crossing) * (size_t)cap);
#pragma omp for schedule(dynamic, 64)
        for (int64_t r = 0; r < total; ++r) {
            int64_t b = r / (rows * W);
            int64_t rem = r % (rows * W);
            int h = (int)(row_begin + rem / W), w = (int)(rem % W);
            double s[3], p[3];
            orc_ray_endpoints(poses + 7 * b, H, W, delta_x, delta_y, off_u, off_v, h, w, s, p);
            int64_t o = (b * H + h) * (int64_t)W + w;
            int64_t c = 0;
            uint64_t hh = 0;
            image[o] = trace_ray(&g, s, p, list, &c, &hh);
            if (nseg) nseg[o] = c;
            if (hash) hash[o] = hh;
        }
        free(list);
    }
}

/* Endpoint derivatives for n arbitrary rays: dEds, dEdp are [n][3]. */
void orc_trace_rays_grad(const double *vol, const int32_t dims[3], const double spacing[3],
                         const double origin[3], const double *src, const double *dst,
                         int64_t n, double *E, double *dEds, double *dEdp, int nthreads)
{
    orc_grid g;
    grid_from(&g, vol, dims, spacing, origin);
    int cap = dims[0] + dims[1] + dims[2] + 5;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
    {
        crossing *list = (crossing *)malloc(sizeof(crossing) * (size_t)cap);
#pragma omp for schedule(dynamic, 64)
        for (int64_t r = 0; r < n; ++r)
            trace_ray_grad(&g, src + 3 * r, dst + 3 * r, list, E + r, dEds + 3 * r,
                           dEdp + 3 * r);
        free(list);
    }
}

/* Per-pixel Jacobian of the image with respect to the pose,
 * jac[b][h][w][j] = d image[b][h][w] / d pose[b][j], j = 0..6, by the chain
 * rule through the endpoint derivatives above. */
void orc_render_jacobian(const double *vol, const int32_t dims[3], const double spacing[3],
                         const double origin[3], const double *poses, int32_t n_poses,
                         int32_t H, int32_t W, double delta_x, double delta_y, double off_u,
                         double off_v, double *image, double *jac, int nthreads)
{
    orc_grid g;
    grid_from(&g, vol, dims, spacing, origin);
    int cap = dims[0] + dims[1] + dims[2] + 5;
    int64_t total = (int64_t)n_poses * H * W;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
    {
        crossing *list = (crossing *)malloc(sizeof(crossing) * (size_t)cap);
#pragma omp for schedule(dynamic, 64)
        for (int64_t r = 0; r < total; ++r) {
            int64_t b = r / ((int64_t)H * W);
            int h = (int)((r / W) % H), w = (int)(r % W);
            const double *pose = poses + 7 * b;
            double s[3], p[3], ds[21], dp[21], gs[3], gp[3], E;
            orc_ray_endpoints(pose, H, W, delta_x, delta_y, off_u, off_v, h, w, s, p);
            orc_ray_endpoint_derivs(pose, H, W, delta_x, delta_y, off_u, off_v, h, w, ds, dp);
            trace_ray_grad(&g, s, p, list, &E, gs, gp);
            image[r] = E;
            for (int j = 0; j < 7; ++j) {
                double acc = 0.0;
                for (int c = 0; c < 3; ++c) acc += gs[c] * ds[c * 7 + j] + gp[c] * dp[c * 7 + j];
                jac[r * 7 + j] = acc;
            }
        }
        free(list);
    }
}

/* Per-pixel derivative of the image with respect to the detector's
 * intrinsic parameters: jac[b][h][w][0..3] = d image / d (delta_x, delta_y,
 * offset_u, offset_v).  They move only the pixel, not the source:
 * d p / d delta_x = R e_y (w + 1/2 - W/2), d p / d delta_y = R e_z
 * (h + 1/2 - H/2), d p / d offset_u = R e_y, d p / d offset_v = R e_z. */
void orc_render_detector_jacobian(const double *vol, const int32_t dims[3],
                                  const double spacing[3], const double origin[3],
                                  const double *poses, int32_t n_poses, int32_t H, int32_t W,
                                  double delta_x, double delta_y, double off_u, double off_v,
                                  double *image, double *jac, int nthreads)
{
    orc_grid g;
    grid_from(&g, vol, dims, spacing, origin);
    int cap = dims[0] + dims[1] + dims[2] + 5;
    int64_t total = (int64_t)n_poses * H * W;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
    {
        crossing *list = (crossing *)malloc(sizeof(crossing) * (size_t)cap);
#pragma omp for schedule(dynamic, 64)
        for (int64_t r = 0; r < total; ++r) {
            int64_t b = r / ((int64_t)H * W);
            int h = (int)((r / W) % H), w = (int)(r % W);
            const double *pose = poses + 7 * b;
            double s[3], p[3], gs[3], gp[3], E, R[9];
            orc_ray_endpoints(pose, H, W, delta_x, delta_y, off_u, off_v, h, w, s, p);
            trace_ray_grad(&g, s, p, list, &E, gs, gp);
            orc_rotation(pose[0], pose[1], pose[2], -1, R);
            double ku = w + 0.5 - 0.5 * W, kv = h + 0.5 - 0.5 * H;
            double gu = 0.0, gv = 0.0;   /* gp . R e_y, gp . R e_z */
            for (int c = 0; c < 3; ++c) {
                gu += gp[c] * R[3 * c + 1];
                gv += gp[c] * R[3 * c + 2];
            }
            image[r] = E;
            jac[4 * r] = gu * ku;
            jac[4 * r + 1] = gv * kv;
            jac[4 * r + 2] = gu;
            jac[4 * r + 3] = gv;
        }
        free(list);
    }
}

/* Zero-normalised cross-correlation of two images of n pixels (population
 * standard deviations), and its gradient with respect to the first image. */
double orc_zncc(const double *I, const double *T, int64_t n, double *grad /*nullable*/)
{
    double mi = 0.0, mt = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        mi += I[i];
        mt += T[i];
    }
    mi /= (double)n;
    mt /= (double)n;
    double vi = 0.0, vt = 0.0, cov = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        vi += (I[i] - mi) * (I[i] - mi);
        vt += (T[i] - mt) * (T[i] - mt);
        cov += (I[i] - mi) * (T[i] - mt);
    }
    double si = sqrt(vi / (double)n), st = sqrt(vt / (double)n);
    double z = cov / (double)n / (si * st);
    if (grad) {
        /* dZ/dI_i = (That_i - Z Ihat_i) / (n sigma_I) */
        for (int64_t i = 0; i < n; ++i) {
            double ih = (I[i] - mi) / si, th = (T[i] - mt) / st;
            grad[i] = (th - z * ih) / ((double)n * si);
        }
    }
    return z;
}

/* Mean squared difference of two images of n pixels, the L2 image loss that
 * Sec. 3.2 compares with the negative ZNCC: loss = (1/n) sum (I - T)^2, and
 * its gradient with respect to the first image, 2 (I - T) / n. */
double orc_l2(const double *I, const double *T, int64_t n, double *grad /*nullable*/)
{
    double acc = 0.0;
    for (int64_t i = 0; i < n; ++i) acc += (I[i] - T[i]) * (I[i] - T[i]);
    if (grad)
        for (int64_t i = 0; i < n; ++i) grad[i] = 2.0 * (I[i] - T[i]) / (double)n;
    return acc / (double)n;
}

int orc_openmp_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
