// Shear-warp rotated view (Fig. 3; shear-warp paragraph of "Physical
// principles"): the stack is remapped with a changed per-image shift and
// projected by the forward kernel, then each projection row is stretched
// along the column axis by a 1-D linear resample.
//
// Geometry (rotation in the plane of the scan axis Y and the optical axis
// Z): a point (Y, Z) sits in image n = (Y - Z cot a) / z at raw column
// c = Z / (p sin a).  With a shift s' per image it lands at
// x' + b = Y s' / z + Z (1 / (p sin a) - s' cot a / z).  The view at angle t
// to the optical axis has image coordinate u = Y cos t + Z sin t; x' + b is
// proportional to u exactly for s' = z cos t / (p cos(t - a)), and then
// u / p = cos(t - a) (x' + b).  So the stretch is cos(t - a).
#include <cmath>
#include <cstdint>

#include <hip/hip_runtime.h>

#include "common.hpp"
#include "deskew.h"

using namespace dsk;

namespace {

constexpr int kStretchBlock = 256;

// out[r][j] = (1 - f) proj[r][i] + f proj[r][i + 1] with j / stretch = i + f,
// zero outside [0, win).  The coordinate is FP64; the two weights are
// rounded once to FP32 like the remap's.
__global__ __launch_bounds__(kStretchBlock) void k_stretch(const float *__restrict__ proj,
                                                           float *__restrict__ out, int64_t win,
                                                           int64_t wout, int64_t total,
                                                           double stretch) {
    const int64_t t = (int64_t)blockIdx.x * kStretchBlock + threadIdx.x;
    if (t >= total) return;
    const int64_t r = t / wout, j = t - r * wout;
    const double u = (double)j / stretch;
    const double fi = floor(u);
    const double f = __dsub_rn(u, fi);
    const int64_t i = (int64_t)fi;
    const float *p = proj + r * win;
    const float a = (i >= 0 && i < win) ? p[i] : 0.0f;
    const float c = (i + 1 >= 0 && i + 1 < win) ? p[i + 1] : 0.0f;
    const float whi = (float)__dsub_rn(1.0, f), wlo = (float)f;
    out[t] = fmaf(wlo, c, whi * a);
}

bool stretch_args_ok(int64_t rows, int64_t win, double stretch, int64_t wout) {
    if (rows <= 0 || win <= 0 || wout <= 0) return false;
    if (!std::isfinite(stretch) || !(stretch >= 1e-6) || !(stretch <= 1e6)) return false;
    return true;
}

int stretch_shape_ok(int64_t rows, int64_t win, int64_t wout) {
    if (win >= (int64_t(1) << 30) || wout >= (int64_t(1) << 30)) return DSK_ESHAPE;
    if (rows * wout / kStretchBlock >= kMaxI32) return DSK_ESHAPE;
    return DSK_OK;
}

void launch_stretch(const float *proj, int64_t rows, int64_t win, double stretch, float *out,
                    int64_t wout, hipStream_t stream) {
    const int64_t total = rows * wout;
    const dim3 grid((unsigned)((total + kStretchBlock - 1) / kStretchBlock));
    hipLaunchKernelGGL(k_stretch, grid, dim3(kStretchBlock), 0, stream, proj, out, win, wout,
                       total, stretch);
}

}  // namespace

// Columns of a stretched row: the last input column (width_in - 1) lands at
// (width_in - 1) * stretch, and the output keeps every column up to it.
extern "C" int dsk_stretch_width(int64_t width_in, double stretch, int64_t *width_out) {
    if (!width_out || width_in <= 0 || !std::isfinite(stretch) || !(stretch > 0.0))
        return DSK_EINVAL;
    const double last = std::floor((double)(width_in - 1) * stretch);
    if (!(last < 1.0e15)) return DSK_ESHAPE;
    *width_out = (int64_t)last + 1;
    return DSK_OK;
}

extern "C" int dsk_view_plan(dsk_dims d, dsk_geom g, double theta_deg, double *shear_px,
                             double *stretch, int64_t *proj_width, int64_t *origin,
                             int64_t *view_width) {
    if (!dims_ok(d) || !std::isfinite(theta_deg) || !std::isfinite(g.angle_deg) ||
        !std::isfinite(g.step_um) || !std::isfinite(g.pixel_um) || !(g.pixel_um > 0.0))
        return DSK_EINVAL;
    const double pi = 3.14159265358979323846;
    const double theta = theta_deg * pi / 180.0;
    const double alpha = g.angle_deg * pi / 180.0;
    const double c = std::cos(theta - alpha);
    if (!(c > 1e-6)) return DSK_EINVAL;  // the view must face the sheet side
    const double s = g.step_um * std::cos(theta) / (g.pixel_um * c);
    int64_t w = 0, b = 0;
    const int st = dsk_plan(d, nullptr, s, &w, &b);
    if (st != DSK_OK) return st;
    int64_t vw = 0;
    const int sw = dsk_stretch_width(w, c, &vw);
    if (sw != DSK_OK) return sw;
    if (shear_px) *shear_px = s;
    if (stretch) *stretch = c;
    if (proj_width) *proj_width = w;
    if (origin) *origin = b;
    if (view_width) *view_width = vw;
    return DSK_OK;
}

extern "C" size_t dsk_view_workspace_bytes(dsk_dims d, int64_t proj_width) {
    if (!dims_ok(d) || proj_width <= 0) return 0;
    return 2 * sizeof(float) * (size_t)d.rows * (size_t)proj_width;
}

extern "C" int dsk_view_u16(const uint16_t *in, dsk_dims d, double shear_px, double stretch,
                            int64_t origin, int64_t proj_width, float *vsum, float *vmax,
                            int64_t view_width, void *workspace, size_t workspace_bytes,
                            hipStream_t stream) {
    if (!in || !dims_ok(d) || (!vsum && !vmax) || !workspace) return DSK_EINVAL;
    if (!std::isfinite(shear_px) || !stretch_args_ok(d.rows, proj_width, stretch, view_width))
        return DSK_EINVAL;
    if ((uintptr_t)workspace & 15) return DSK_EINVAL;
    int st = check_frame(d, origin, proj_width);
    if (st != DSK_OK) return st;
    st = stretch_shape_ok(d.rows, proj_width, view_width);
    if (st != DSK_OK) return st;
    if (workspace_bytes < dsk_view_workspace_bytes(d, proj_width)) return DSK_ESHAPE;
    float *ps = (float *)workspace;
    float *pm = ps + (size_t)d.rows * (size_t)proj_width;
    st = launch_forward(in, 0, d, nullptr, shear_px, origin, nullptr, vsum ? ps : nullptr,
                        vmax ? pm : nullptr, proj_width, kDefaultProjTune, stream);
    if (st != DSK_OK) return st;
    if (vsum) launch_stretch(ps, d.rows, proj_width, stretch, vsum, view_width, stream);
    if (vmax) launch_stretch(pm, d.rows, proj_width, stretch, vmax, view_width, stream);
    return hip_status(hipGetLastError());
}

extern "C" int dsk_stretch_f32(const float *proj, int64_t rows, int64_t width_in, double stretch,
                               float *out, int64_t width_out, hipStream_t stream) {
    if (!proj || !out || !stretch_args_ok(rows, width_in, stretch, width_out)) return DSK_EINVAL;
    const int st = stretch_shape_ok(rows, width_in, width_out);
    if (st != DSK_OK) return st;
    launch_stretch(proj, rows, width_in, stretch, out, width_out, stream);
    return hip_status(hipGetLastError());
}
