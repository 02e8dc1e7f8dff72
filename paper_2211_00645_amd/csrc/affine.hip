// Real-space (affine) deskew: the stack resampled onto a Cartesian grid of
// the sample, the alternative the paper contrasts the remap with
// ("Physical principles", remap paragraph).  Raw image n, row x, column z
// images the point X = x p, Z = z p sin(a), Y = n s_z + z p cos(a)
// (s_z the scan step).  With the output's Z on the raw column grid, voxel
// (y, x, z) at Y = Y0 + y dy lies on raw column z between images
// floor(u) and floor(u) + 1, u = (Y - z p cos(a)) / s_z, and is their linear
// interpolation (zero outside the stack).
//
// The output is several times the remap's volume, so the kernel is a
// one-shot grid in output order: consecutive workgroups write consecutive
// memory (the write stream stays on one front), each lane writes 4
// consecutive z with one 16-byte store, and the interpolation reads come
// from the two or three images the lane's 4 columns cross.  Consecutive y
// of one (x, z range) re-read nearly the same input lines; they are
// R*C/1024 workgroups apart (1024 for a 512 x 2048 image: a multiple of the
// 8 XCDs, so the same XCD), and those reads hit its L2 or the MALL.
#include <cmath>
#include <cstdint>

#include <hip/hip_runtime.h>

#include "common.hpp"
#include "deskew.h"
#include "kernels.hpp"

using namespace dsk;

namespace {

constexpr int kAffBlock = 256;

template <typename TIn>
struct AffArgs {
    const TIn *in;
    float *vol;
    int64_t ny, zgroups;  // output y count; 4-column groups per row
    int32_t N, R, C;
    double u0, uy, uz;    // u = u0 + y uy - z uz
};

// Value of image n at (x, z); zero outside the stack's images.
template <typename TIn>
__device__ __forceinline__ float img_px(const AffArgs<TIn> &a, int64_t n, int64_t x, int64_t z) {
    if (n < 0 || n >= a.N) return 0.0f;
    return (float)a.in[(n * a.R + x) * a.C + z];
}

template <typename TIn>
__device__ __forceinline__ float aff_voxel(const AffArgs<TIn> &a, double uy_part, int64_t x,
                                           int64_t z) {
    double u = __dsub_rn(uy_part, __dmul_rn((double)z, a.uz));
    // far outside the stack either way: keep the image index in range
    u = u < -1.0e15 ? -1.0e15 : (u > 1.0e15 ? 1.0e15 : u);
    const double fi = floor(u);
    const double f = __dsub_rn(u, fi);
    const int64_t n0 = (int64_t)fi;
    const float whi = (float)__dsub_rn(1.0, f), wlo = (float)f;
    const float lo = img_px(a, n0, x, z), hi = img_px(a, n0 + 1, x, z);
    return fmaf(wlo, hi, whi * lo);
}

// One lane per (y, x, 4-column group), flat in output order.  VEC: C is a
// multiple of 4 and the volume 16-byte aligned (one aligned store per
// lane); otherwise each column is stored on its own, with a bound check.
template <typename TIn, bool VEC>
__global__ __launch_bounds__(kAffBlock) void k_affine(AffArgs<TIn> a) {
    const int64_t t = (int64_t)blockIdx.x * kAffBlock + threadIdx.x;
    const int64_t per_y = (int64_t)a.R * a.zgroups;
    const int64_t y = t / per_y;
    if (y >= a.ny) return;
    const int64_t rem = t - y * per_y;
    const int64_t x = rem / a.zgroups;
    const int64_t z0 = 4 * (rem - x * a.zgroups);
    const double uy_part = __dadd_rn(a.u0, __dmul_rn((double)y, a.uy));
    float *o = a.vol + (y * a.R + x) * a.C + z0;
    if constexpr (VEC) {
        f32x4 v;
        v.x = aff_voxel(a, uy_part, x, z0);
        v.y = aff_voxel(a, uy_part, x, z0 + 1);
        v.z = aff_voxel(a, uy_part, x, z0 + 2);
        v.w = aff_voxel(a, uy_part, x, z0 + 3);
        store_f32x4<true>(o, v);
    } else {
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (z0 + i < a.C) store_f32<true>(o + i, aff_voxel(a, uy_part, x, z0 + i));
    }
}

bool geom_ok(dsk_geom g) {
    return std::isfinite(g.angle_deg) && std::isfinite(g.step_um) && std::isfinite(g.pixel_um) &&
           g.pixel_um > 0.0 && g.step_um != 0.0;
}

}  // namespace

extern "C" int dsk_affine_plan(dsk_dims d, dsk_geom g, double dy_um, double *y0_um,
                               int64_t *ny) {
    if (!dims_ok(d) || !geom_ok(g) || !std::isfinite(dy_um) || !(dy_um > 0.0)) return DSK_EINVAL;
    const double pi = 3.14159265358979323846;
    const double pc = g.pixel_um * std::cos(g.angle_deg * pi / 180.0);
    const double c[4] = {0.0, (double)(d.planes - 1) * g.step_um, (double)(d.cols - 1) * pc,
                         (double)(d.planes - 1) * g.step_um + (double)(d.cols - 1) * pc};
    double lo = c[0], hi = c[0];
    for (int k = 1; k < 4; ++k) {
        lo = c[k] < lo ? c[k] : lo;
        hi = c[k] > hi ? c[k] : hi;
    }
    const double n = std::floor((hi - lo) / dy_um) + 1.0;
    if (!(n >= 1.0) || n >= 1.0e15) return DSK_ESHAPE;
    if (y0_um) *y0_um = lo;
    if (ny) *ny = (int64_t)n;
    return DSK_OK;
}

extern "C" int dsk_affine_u16(const uint16_t *in, dsk_dims d, dsk_geom g, double dy_um,
                              double y0_um, int64_t ny, float *vol, hipStream_t stream) {
    if (!in || !vol || !dims_ok(d) || !geom_ok(g) || !std::isfinite(dy_um) || !(dy_um > 0.0) ||
        !std::isfinite(y0_um) || ny <= 0)
        return DSK_EINVAL;
    const double pi = 3.14159265358979323846;
    const double pc = g.pixel_um * std::cos(g.angle_deg * pi / 180.0);
    AffArgs<uint16_t> a{in, vol, ny, (d.cols + 3) / 4, d.planes, d.rows, d.cols,
                        y0_um / g.step_um, dy_um / g.step_um, pc / g.step_um};
    const int64_t threads = ny * (int64_t)d.rows * a.zgroups;
    if (threads / kAffBlock >= kMaxI32) return DSK_ESHAPE;
    const dim3 grid((unsigned)((threads + kAffBlock - 1) / kAffBlock));
    const bool vec = d.cols % 4 == 0 && ((uintptr_t)vol & 15) == 0;
    if (vec)
        hipLaunchKernelGGL((k_affine<uint16_t, true>), grid, dim3(kAffBlock), 0, stream, a);
    else
        hipLaunchKernelGGL((k_affine<uint16_t, false>), grid, dim3(kAffBlock), 0, stream, a);
    return hip_status(hipGetLastError());
}
