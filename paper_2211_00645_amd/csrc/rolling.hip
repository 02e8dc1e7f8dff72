// rolling.hip -- rolling display mode: projections refreshed after every
// camera image (methods section, rolling update; Fig. 4a).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "common.hpp"
#include "deskew.h"
#include "kernels.hpp"

using namespace dsk;

namespace {

// Levels of the max-tree above the N leaves (0 for a single image).
int tree_levels(int32_t n) {
    int l = 0;
    for (int64_t c = n; c > 1; c = (c + 1) / 2) ++l;
    return l;
}

int64_t tree_nodes(int32_t n) {
    int64_t tot = 0;
    for (int64_t c = n; c > 1;) {
        c = (c + 1) / 2;
        tot += c;
    }
    return tot;
}

template <typename T>
hipError_t zero(T *p, int64_t n, hipStream_t s) {
    if (!p || n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_zero<T>, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace

extern "C" size_t dsk_rolling_tree_bytes(dsk_dims d, int64_t out_width) {
    if (!dims_ok(d) || out_width <= 0) return 0;
    return (size_t)tree_nodes(d.planes) * (size_t)d.rows * (size_t)out_width * sizeof(float);
}

extern "C" int dsk_rolling_reset(dsk_dims d, int64_t out_width, float *vol, float *tree,
                                 double *sum64, float *psum, float *pmax, hipStream_t stream) {
    if (!dims_ok(d) || !vol || !sum64 || !psum || !pmax) return DSK_EINVAL;
    if (tree_levels(d.planes) > 0 && !tree) return DSK_EINVAL;
    const int st = check_frame(d, 0, out_width);
    if (st != DSK_OK) return st;
    const int64_t rw = (int64_t)d.rows * out_width;
    hipError_t e = zero(vol, rw * d.planes, stream);
    if (e == hipSuccess) e = zero(tree, rw * tree_nodes(d.planes), stream);
    if (e == hipSuccess) e = zero(sum64, rw, stream);
    if (e == hipSuccess) e = zero(psum, rw, stream);
    if (e == hipSuccess) e = zero(pmax, rw, stream);
    return hip_status(e);
}

extern "C" int dsk_rolling_update_u16(const uint16_t *plane, int32_t n, dsk_dims d,
                                      const double *offsets_dev, double shift_px,
                                      int64_t origin, int64_t out_width, float *vol, float *tree,
                                      double *sum64, float *psum, float *pmax,
                                      hipStream_t stream) {
    if (!plane || !dims_ok(d) || !vol || !sum64 || !psum || !pmax) return DSK_EINVAL;
    if (n < 0 || n >= d.planes) return DSK_EINVAL;
    if (!offsets_dev && !std::isfinite(shift_px)) return DSK_EINVAL;
    const int levels = tree_levels(d.planes);
    if (levels > 0 && !tree) return DSK_EINVAL;
    const int st = check_frame(d, origin, out_width);
    if (st != DSK_OK) return st;
    const int64_t rw = (int64_t)d.rows * out_width;
    RollArgs a{plane, vol, tree, sum64, psum, pmax, offsets_dev, shift_px, (double)origin,
               out_width, d.planes, d.rows, d.cols, n, levels};
    // 4 pixels per thread when every array is 16-byte aligned and the
    // plane's pixel count is a multiple of 4
    const bool vec = rw % 4 == 0 && ((uintptr_t)vol & 15) == 0 && ((uintptr_t)sum64 & 15) == 0 &&
                     ((uintptr_t)psum & 15) == 0 && ((uintptr_t)pmax & 15) == 0 &&
                     (levels == 0 || ((uintptr_t)tree & 15) == 0);
    const int64_t per = vec ? 4 : 1;
    const int64_t blocks = (rw / per + 255) / 256;
    if (blocks > kMaxI32) return DSK_ESHAPE;
    if (vec)
        hipLaunchKernelGGL(k_rolling_update4<uint16_t>, dim3((unsigned)blocks), dim3(256), 0,
                           stream, a);
    else
        hipLaunchKernelGGL(k_rolling_update<uint16_t>, dim3((unsigned)blocks), dim3(256), 0,
                           stream, a);
    return hip_status(hipGetLastError());
}
