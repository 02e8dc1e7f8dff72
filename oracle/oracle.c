/*
 * oracle.c -- plain, slow, FP64 CPU oracle for the deskew of an oblique-plane
 * light-sheet stack and its projections.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file or the library built from it; only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg use it.  It shares no
 * source with the HIP library: every formula below is written out from the
 * paper's text (Lamb, Ward & Kaminski, arXiv 2211.00645).
 *
 * Notation (all indices are pixel centres, zero-based):
 *   S[n][r][c]   raw stack, n = image (scan position), r = row, c = column;
 *                the column axis is the one the sheet angle shears.
 *   o[n]         lateral offset of image n in pixels ("Physical principles",
 *                Eq. 1: l = z cos(alpha), divided by the sample-space pixel
 *                size so the remap happens in image pixels).
 *   b, W         origin and width of the larger image each raw image is
 *                remapped into ("Physical principles", remap paragraph;
 *                Fig. 2c).
 *   D[n][r][x']  deskewed volume: image n placed at its accumulated lateral
 *                shift, sampled with linear interpolation, zero outside the
 *                raw image.
 *   Psum, Pmax   sum and maximum over n of D (the maximum projection is the
 *                mimicked widefield view, Fig. 2d; the sum is its linear
 *                counterpart).
 *
 * Every value is computed in FP64 and rounded once to FP32 on output.
 * Parallelism is one OpenMP loop over independent output rows; no blocking,
 * fusion or reordering beyond that.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

/* Threads the parallel loops below use. */
int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Set the threads the parallel loops use (n >= 1); for timing only. */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Eq. 1: the lateral shift between consecutive images is l = z cos(alpha),
 * z being the scan distance between images.  Expressed in image pixels of
 * sample-space size p: s = (z * cos(alpha)) / p, alpha given in degrees. */
double orc_shift_px(double angle_deg, double step_um, double pixel_um)
{
    double alpha = angle_deg * ORC_PI / 180.0;
    return (step_um * cos(alpha)) / pixel_um;
}

/* Uniform scan: image n sits n scan steps away from image 0, so its
 * accumulated offset is n times the per-step shift (Eq. 1 applied n times). */
void orc_offsets_uniform(int64_t n_planes, double shift_px, double *offsets)
{
    for (int64_t n = 0; n < n_planes; ++n)
        offsets[n] = (double)n * shift_px;
}

/* The larger image of the remap: it must hold every image at its offset.
 * b is the leftmost integer column any image touches, W the number of
 * columns from there to the rightmost column any image touches.  A column
 * x' of the larger image corresponds to raw column x' + b - o[n]. */
void orc_frame(int64_t n_planes, const double *offsets, int64_t cols,
               int64_t *origin, int64_t *width)
{
    double lo = offsets[0], hi = offsets[0];
    for (int64_t n = 1; n < n_planes; ++n) {
        if (offsets[n] < lo) lo = offsets[n];
        if (offsets[n] > hi) hi = offsets[n];
    }
    *origin = (int64_t)floor(lo);
    *width = cols + (int64_t)ceil(hi) - *origin;
}

/* Raw sample with zero outside the image. */
static double raw_at(const void *row, int is_f32, int64_t cols, int64_t i)
{
    if (i < 0 || i >= cols) return 0.0;
    if (is_f32) return (double)((const float *)row)[i];
    return (double)((const uint16_t *)row)[i];
}

/* Deskew by remapping (Physical principles, remap paragraph) plus the
 * projections over the image axis (Fig. 2d).
 *
 * For every output column x' of image n the raw coordinate is
 *     u = x' + b - o[n],  i = floor(u),  f = u - i,
 * and the remapped value is the linear interpolation
 *     D = (1 - f) * S~[i] + f * S~[i + 1],   S~ = 0 outside [0, cols).
 * Psum = sum_n D and Pmax = max_n D over the dense D (padding included).
 *
 * Rows r in [r0, r1) are computed; outputs are laid out for that row range:
 * vol/vol64 as [n_planes][r1 - r0][width], psum/pmax as [r1 - r0][width].
 * Any output pointer may be NULL. */
void orc_deskew(const void *stack, int is_f32, int64_t n_planes, int64_t rows,
                int64_t cols, const double *offsets, int64_t origin,
                int64_t width, int64_t r0, int64_t r1, float *vol,
                double *vol64, float *psum, float *pmax)
{
    const int64_t nr = r1 - r0;
    const size_t esz = is_f32 ? sizeof(float) : sizeof(uint16_t);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t rr = 0; rr < nr; ++rr) {
        const int64_t r = r0 + rr;
        double *sum = (double *)calloc((size_t)width, sizeof(double));
        double *mx = (double *)malloc((size_t)width * sizeof(double));
        for (int64_t x = 0; x < width; ++x) mx[x] = -INFINITY;
        for (int64_t n = 0; n < n_planes; ++n) {
            const char *row =
                (const char *)stack + (size_t)((n * rows + r) * cols) * esz;
            for (int64_t x = 0; x < width; ++x) {
                double u = (double)x + (double)origin - offsets[n];
                double fi = floor(u);
                double f = u - fi;
                int64_t i = (int64_t)fi;
                double d = (1.0 - f) * raw_at(row, is_f32, cols, i) +
                           f * raw_at(row, is_f32, cols, i + 1);
                size_t o = (size_t)((n * nr + rr) * width + x);
                if (vol) vol[o] = (float)d;
                if (vol64) vol64[o] = d;
                sum[x] += d;
                if (d > mx[x]) mx[x] = d;
            }
        }
        for (int64_t x = 0; x < width; ++x) {
            if (psum) psum[rr * width + x] = (float)sum[x];
            if (pmax) pmax[rr * width + x] = (float)mx[x];
        }
        free(sum);
        free(mx);
    }
}

/* Transpose of the remap, assembled explicitly as a scatter: every output
 * voxel hands its gradient back to the two raw pixels it was interpolated
 * from, with the same weights (1 - f) and f.  grad_in is [n_planes][rows]
 * [cols]; grad_vol is the full [n_planes][rows][width] volume. */
void orc_adjoint(const float *grad_vol, int64_t n_planes, int64_t rows,
                 int64_t cols, const double *offsets, int64_t origin,
                 int64_t width, float *grad_in, double *grad_in64)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t nr = 0; nr < n_planes * rows; ++nr) {
        const int64_t n = nr / rows;
        double *acc = (double *)calloc((size_t)cols, sizeof(double));
        const float *g = grad_vol + (size_t)nr * (size_t)width;
        for (int64_t x = 0; x < width; ++x) {
            double u = (double)x + (double)origin - offsets[n];
            double fi = floor(u);
            double f = u - fi;
            int64_t i = (int64_t)fi;
            if (i >= 0 && i < cols) acc[i] += (1.0 - f) * (double)g[x];
            if (i + 1 >= 0 && i + 1 < cols) acc[i + 1] += f * (double)g[x];
        }
        for (int64_t c = 0; c < cols; ++c) {
            if (grad_in) grad_in[(size_t)nr * cols + c] = (float)acc[c];
            if (grad_in64) grad_in64[(size_t)nr * cols + c] = acc[c];
        }
        free(acc);
    }
}

/* Derivative of the loss with respect to each image's offset o[n].
 * Inside a cell D = (1 - f) S~[i] + f S~[i + 1] with u = x' + b - o[n], so
 * dD/do[n] = S~[j] - S~[j + 1].  The cell is taken as j = ceil(u) - 1, which
 * is floor(u) away from integer u and, at integer u, the cell entered when
 * o[n] grows: the right derivative in o[n].  grad_off[n] is the FP64 sum of
 * grad_vol * dD/do[n] over all rows and output columns of image n. */
void orc_shear_grad(const float *stack, const float *grad_vol,
                    int64_t n_planes, int64_t rows, int64_t cols,
                    const double *offsets, int64_t origin, int64_t width,
                    double *grad_off)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t n = 0; n < n_planes; ++n) {
        double acc = 0.0;
        for (int64_t r = 0; r < rows; ++r) {
            const float *row = stack + (size_t)((n * rows + r) * cols);
            const float *g = grad_vol + (size_t)((n * rows + r) * width);
            for (int64_t x = 0; x < width; ++x) {
                double u = (double)x + (double)origin - offsets[n];
                int64_t j = (int64_t)ceil(u) - 1;
                double dd = raw_at(row, 1, cols, j) - raw_at(row, 1, cols, j + 1);
                acc += (double)g[x] * dd;
            }
        }
        grad_off[n] = acc;
    }
}

/* Shear-warp rotated view (Fig. 3 and the shear-warp paragraph of
 * "Physical principles"): remapping with a different shift per image and
 * then stretching the projection along the column axis renders the
 * projection of the sample seen from another direction.
 *
 * Geometry, in the plane spanned by the scan axis (coordinate Y) and the
 * optical axis (height Z): a point (Y, Z) is recorded in image
 * n = (Y - Z cot(alpha)) / z at raw column c = Z / (p sin(alpha)).  Remapped
 * with a shift of s' pixels per image it lands at
 *     x' = c + n s' - b = Y s' / z + Z (1 / (p sin(alpha)) - s' cot(alpha) / z) - b.
 * Projecting along the image axis collapses every point with the same x',
 * so the projection is the view along the direction in which x' is
 * constant.  Its image coordinate for a view that makes angle theta with
 * the optical axis is u = Y cos(theta) + Z sin(theta); x' is proportional
 * to u exactly when
 *     s' = z cos(theta) / (p cos(theta - alpha)),
 * and then x' + b = u / (p cos(theta - alpha)): the warp that turns x' into
 * view pixels u / p is a stretch by cos(theta - alpha).  theta = alpha gives
 * back Eq. 1 with no stretch; theta = 0 looks down the optical axis. */
void orc_view_geometry(double theta_deg, double angle_deg, double step_um,
                       double pixel_um, double *shear_px, double *warp)
{
    double theta = theta_deg * ORC_PI / 180.0;
    double alpha = angle_deg * ORC_PI / 180.0;
    *shear_px = step_um * cos(theta) / (pixel_um * cos(theta - alpha));
    *warp = cos(theta - alpha);
}

/* Number of view columns j = 0, 1, ... whose source coordinate j / warp
 * stays inside the projection's width_in columns. */
int64_t orc_view_width(int64_t width_in, double warp)
{
    return (int64_t)floor((double)(width_in - 1) * warp) + 1;
}

/* The warp: view column j samples the projection row at x' = j / warp with
 * linear interpolation, zero outside [0, width_in).  proj is
 * [rows][width_in], out is [rows][width_out], both FP64. */
void orc_warp(const double *proj, int64_t rows, int64_t width_in,
              double warp, int64_t width_out, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < rows; ++r) {
        const double *p = proj + (size_t)(r * width_in);
        for (int64_t j = 0; j < width_out; ++j) {
            double u = (double)j / warp;
            double fi = floor(u);
            double f = u - fi;
            int64_t i = (int64_t)fi;
            double a = (i >= 0 && i < width_in) ? p[i] : 0.0;
            double c = (i + 1 >= 0 && i + 1 < width_in) ? p[i + 1] : 0.0;
            out[(size_t)(r * width_out + j)] = (1.0 - f) * a + f * c;
        }
    }
}

/* Real-space (affine) deskew, the alternative to the remap that the paper
 * contrasts it with ("Physical principles", remap paragraph: an affine
 * transformation of the whole stack, possible only once the stack is
 * complete).  The stack is resampled onto a Cartesian grid of the sample:
 *   X = r p            (rows are already lateral sample coordinates),
 *   Z = c p sin(alpha)  (height above the coverslip of raw column c),
 *   Y = Y0 + y dy       (scan axis, step dy chosen by the caller),
 * where raw image n, column c images the scan coordinate
 * Y = n z + c p cos(alpha) (the sheet is tilted by alpha from the scan axis).
 * With Z on the raw column grid, every output voxel (y, x, z) lies on the
 * line of raw column z between two images: its image coordinate is
 *   u = (Y0 + y dy - z p cos(alpha)) / z_step
 * and the value is the linear interpolation between images floor(u) and
 * floor(u) + 1 (zero outside the stack).  Y0 is the smallest scan
 * coordinate of the stack's corners and ny covers the largest.
 * Output vol [ny][rows][cols]. */
void orc_affine_frame(int64_t n_planes, int64_t cols, double angle_deg,
                      double step_um, double pixel_um, double dy_um,
                      double *y0, int64_t *ny)
{
    double alpha = angle_deg * ORC_PI / 180.0;
    double pc = pixel_um * cos(alpha);
    double lo = 0.0, hi = 0.0;
    double corners[4] = {0.0, (double)(n_planes - 1) * step_um,
                         (double)(cols - 1) * pc,
                         (double)(n_planes - 1) * step_um + (double)(cols - 1) * pc};
    for (int k = 0; k < 4; ++k) {
        if (k == 0 || corners[k] < lo) lo = corners[k];
        if (k == 0 || corners[k] > hi) hi = corners[k];
    }
    *y0 = lo;
    *ny = (int64_t)floor((hi - lo) / dy_um) + 1;
}

void orc_affine(const void *stack, int is_f32, int64_t n_planes, int64_t rows,
                int64_t cols, double angle_deg, double step_um,
                double pixel_um, double dy_um, double y0, int64_t ny,
                float *vol, double *vol64)
{
    double alpha = angle_deg * ORC_PI / 180.0;
    double pc = pixel_um * cos(alpha);
    const size_t esz = is_f32 ? sizeof(float) : sizeof(uint16_t);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t y = 0; y < ny; ++y) {
        double yy = y0 + (double)y * dy_um;
        for (int64_t x = 0; x < rows; ++x) {
            for (int64_t z = 0; z < cols; ++z) {
                double u = (yy - (double)z * pc) / step_um;
                double fi = floor(u);
                double f = u - fi;
                int64_t n0 = (int64_t)fi;
                double a = 0.0, b = 0.0;
                if (n0 >= 0 && n0 < n_planes) {
                    const char *row = (const char *)stack +
                                      (size_t)((n0 * rows + x) * cols) * esz;
                    a = raw_at(row, is_f32, cols, z);
                }
                if (n0 + 1 >= 0 && n0 + 1 < n_planes) {
                    const char *row = (const char *)stack +
                                      (size_t)(((n0 + 1) * rows + x) * cols) * esz;
                    b = raw_at(row, is_f32, cols, z);
                }
                double d = (1.0 - f) * a + f * b;
                size_t o = (size_t)((y * rows + x) * cols + z);
                if (vol) vol[o] = (float)d;
                if (vol64) vol64[o] = d;
            }
        }
    }
}
