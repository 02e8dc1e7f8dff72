// deskew.hip -- C ABI of the single-stack path: geometry plan (Eq. 1 and the
// remap frame), forward deskew with fused projections, adjoint and shear
// gradient.  Host code validates everything before enqueueing a kernel.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>
#include <type_traits>

#include "common.hpp"
#include "deskew.h"
#include "kernels.hpp"

using namespace dsk;

extern "C" int dsk_debug_bounds_violations(unsigned long long *count, int reset) {
    if (!count) return DSK_EINVAL;
    *count = 0;
#if DSK_CHECK_BOUNDS
    unsigned long long a = 0, b = 0;
    if (dsk::read_bounds_violations(&a, reset != 0) != 0 ||
        dsk::batch_bounds_violations(&b, reset != 0) != 0)
        return DSK_EHIP;
    *count = a + b;
    return 1;
#else
    (void)reset;
    return 0;
#endif
}

extern "C" const char *dsk_status_string(int status) {
    switch (status) {
    case DSK_OK: return "ok";
    case DSK_EINVAL: return "invalid argument";
    case DSK_ESHAPE: return "size out of range";
    case DSK_EHIP: return "HIP runtime error";
    case DSK_ENOMEM: return "out of memory";
    case DSK_EBUDGET: return "over the memory budget";
    default: return "unknown status";
    }
}

// Eq. 1: l = z cos(alpha); in pixels of sample-space size p.
extern "C" int dsk_shift_px(dsk_geom g, double *shift_px) {
    if (!shift_px) return DSK_EINVAL;
    if (!std::isfinite(g.angle_deg) || !std::isfinite(g.step_um) ||
        !std::isfinite(g.pixel_um) || !(g.pixel_um > 0.0))
        return DSK_EINVAL;
    const double pi = 3.14159265358979323846;
    const double alpha = g.angle_deg * pi / 180.0;
    *shift_px = (g.step_um * std::cos(alpha)) / g.pixel_um;
    return DSK_OK;
}

// The larger image of the remap: origin b = floor(min o), width
// W = C + ceil(max o) - b, with o[n] = n * s unless offsets are given.
extern "C" int dsk_plan(dsk_dims d, const double *offsets_px, double shift_px,
                        int64_t *out_width, int64_t *origin) {
    if (!out_width || !origin || !dims_ok(d)) return DSK_EINVAL;
    if (!offsets_px && !std::isfinite(shift_px)) return DSK_EINVAL;
    double lo = 0.0, hi = 0.0;
    for (int32_t n = 0; n < d.planes; ++n) {
        const double o = offsets_px ? offsets_px[n] : (double)n * shift_px;
        if (!std::isfinite(o)) return DSK_EINVAL;
        if (n == 0 || o < lo) lo = o;
        if (n == 0 || o > hi) hi = o;
    }
    const double fb = std::floor(lo), fh = std::ceil(hi);
    if (std::fabs(fb) > 4.0e15 || std::fabs(fh) > 4.0e15) return DSK_ESHAPE;
    const int64_t b = (int64_t)fb;
    const int64_t w = (int64_t)d.cols + (int64_t)fh - b;
    if (w <= 0 || w >= (int64_t(1) << 30)) return DSK_ESHAPE;
    *origin = b;
    *out_width = w;
    return DSK_OK;
}

namespace dsk {

int device_cus() {
    static int cache[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (dev < 0 || dev >= 64) dev = 0;
    if (cache[dev] <= 0) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus <= 0)
            cus = 256;
        cache[dev] = cus;
    }
    return cache[dev];
}

// Workgroups of the vector kernel one compute unit holds at once (cached
// per kernel instance).
template <typename TIn, int B, int G, int U, bool NT, bool VOL>
static int vec_resident_per_cu() {
    static int occ = 0;
    if (occ <= 0) {
        int o = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, k_forward_vec<TIn, B, G, U, NT, VOL>, B,
                                                         0) != hipSuccess ||
            o <= 0)
            o = 1;
        occ = o;
    }
    return occ;
}

template <typename TIn, int B, int PT, int U, bool NT>
static hipError_t fwd_launch(FwdArgs<TIn> a, bool vec, int64_t tiles, int64_t edge, int pace_gbs,
                             hipStream_t s) {
    const dim3 block(B);
    if constexpr (PT >= 4) {
        if (vec) {
            // launches without a volume only read: no store kind to choose
            auto kern = a.vol ? k_forward_vec<TIn, B, PT / 4, U, NT, true>
                              : k_forward_vec<TIn, B, PT / 4, U, false, false>;
            // Pacing holds every wavefront to one plane schedule: with a
            // volume it keeps the write stream local; without one, wavefronts
            // whose plane ranges start late wait for their turn.
            int64_t cap = 0;
            if (pace_gbs > 0)
                cap = (int64_t)(a.vol ? vec_resident_per_cu<TIn, B, PT / 4, U, NT, true>()
                                      : vec_resident_per_cu<TIn, B, PT / 4, U, false, false>()) *
                      device_cus();
            // without a volume a frame whose tiles do not all fit at once is
            // not paced: its later tiles would wait out a schedule that began
            // before they started
            if (!a.vol && pace_gbs > 0 && tiles * a.R > cap) pace_gbs = 0;
            auto launch_rows = [&](FwdArgs<TIn> f, int64_t f_edge) {
                if (pace_gbs > 0) {
                    // one tile's share of a plane's bytes, timed at pace_gbs
                    // (the edge columns' workgroups are not paced)
                    const double plane_bytes = (double)f.R * f.C * sizeof(TIn) +
                                               (f.vol ? 4.0 * (double)f.R * (double)f.W : 0.0);
                    const double t = plane_bytes / (double)(tiles * f.R) /
                                     ((double)pace_gbs * 1e9) * 1e8 * 65536.0;
                    f.tau_wg = t >= 4.0e9 ? 4000000000u : (uint32_t)t;
                    f.pace_cap = (int32_t)(cap < 1 ? 1 : (cap > kMaxI32 ? kMaxI32 : cap));
                }
                f.edge_wg = (int32_t)f_edge;
                hipLaunchKernelGGL(kern, dim3((unsigned)(tiles * f.R + f_edge)), block, 0, s, f,
                                   (int)tiles);
                return hipGetLastError();
            };
            // A paced frame with a volume and more tiles than resident
            // workgroups goes out as bands of rows that each fit, one launch
            // after another: a second round of tiles starting as the first
            // ones end would fall behind their schedule and spread the write
            // stream over the volume.  Bands start at multiples of 4 rows, so
            // every row keeps its residues mod 4 (r W and r in_row) and with
            // them the kernel's alignment.
            const int64_t band = cap / tiles / 4 * 4;
            if (a.vol && pace_gbs > 0 && tiles * a.R > cap && band >= 4) {
                const int64_t nb = (a.R + band - 1) / band;
                const int64_t rows = ((a.R + nb - 1) / nb + 3) / 4 * 4;
                const int64_t per = B;   // edge lanes per workgroup with a volume
                for (int64_t r0 = 0; r0 < a.R; r0 += rows) {
                    FwdArgs<TIn> f = a;
                    const int64_t nr = a.R - r0 < rows ? a.R - r0 : rows;
                    const int64_t in_off = r0 * a.in_row;
                    f.in = a.in + in_off;
                    f.in_lo = a.in_lo + in_off;
                    f.in_hi = a.in_hi - in_off;
                    f.R = (int32_t)nr;
                    f.vol = a.vol + r0 * a.W;
                    f.psum = a.psum ? a.psum + r0 * a.W : nullptr;
                    f.pmax = a.pmax ? a.pmax + r0 * a.W : nullptr;
                    const hipError_t e = launch_rows(f, edge > 0 ? (6 * nr + per - 1) / per : 0);
                    if (e != hipSuccess) return e;
                }
                return hipSuccess;
            }
            return launch_rows(a, edge);
        }
    }
    hipLaunchKernelGGL((k_forward_scalar<TIn, B, PT, NT>), dim3((unsigned)(tiles * a.R)), block,
                       0, s, a, (int)tiles);
    return hipGetLastError();
}

template <typename TIn>
static hipError_t fwd_dispatch(const FwdArgs<TIn> &a, const dsk_tune &t, bool vec, int64_t tiles,
                               int64_t edge, hipStream_t stream) {
    return dispatch_tune(t, [&](auto B, auto P, auto U, auto NT) {
        return fwd_launch<TIn, decltype(B)::value, decltype(P)::value, decltype(U)::value,
                          decltype(NT)::value>(a, vec, tiles, edge, t.pace_gbs, stream);
    });
}

// Tiles per row of the vector kernel's 128-byte-aligned grids (groups of
// per groups): each row's grid starts shift groups before its first group,
// shift being the groups between the previous 128-byte boundary of the
// volume and that group (the kernel's rule).  With rows*W a multiple of 32
// the shifts repeat every 32 rows.  The grids are used only when they need
// no more tiles than the plain ones: a tile that holds only the few groups a
// shift pushes past the row's last full tile walks every plane for them (on
// 512 rows of 1793 columns in float32, 0.28 -> 0.36 ms), while widths whose
// shifted grids fit (8 mod 16 columns, say) keep the gain.
static int64_t aligned_tiles(const float *vol, int64_t rows, int64_t width, int64_t per) {
    int64_t need = 1;
    for (int64_t r = 0; r < rows && r < 32; ++r) {
        const int64_t ca = (4 - ((r * width) & 3)) & 3;
        const int64_t ng = width > ca ? (width - ca) / 4 : 0;
        const int64_t shift = (int64_t)((((uintptr_t)(vol + r * width + ca)) >> 2) & 31) >> 2;
        const int64_t n = (ng + shift + per - 1) / per;
        if (n > need) need = n;
    }
    return need;
}

int launch_forward_layout(const void *in, int in_is_f32, dsk_dims d, const InLayout &lay,
                          const double *offs, double shift, int64_t origin, float *vol,
                          float *psum, float *pmax, int64_t width, const dsk_tune &t,
                          hipStream_t stream) {
    if (!in || !dims_ok(d) || (!vol && !psum && !pmax)) return DSK_EINVAL;
    if (!offs && !std::isfinite(shift)) return DSK_EINVAL;
    if (!tune_ok(t)) return DSK_EINVAL;
    int st = check_frame(d, origin, width);
    if (st != DSK_OK) return st;
    // every row must lie inside the readable extent
    const int64_t last = (int64_t)(d.planes - 1) * lay.plane + (int64_t)(d.rows - 1) * lay.row;
    if (lay.row < d.cols || lay.plane < (int64_t)(d.rows - 1) * lay.row + d.cols || lay.lo < 0 ||
        lay.hi < last + d.cols)
        return DSK_ESHAPE;
    const bool vec = vec_ok(t, d, width, in, in_is_f32, vol, lay.plane);
    // volume rows' tiles on 128-byte boundaries when the plane pitch keeps
    // them there in every plane and the shifted grids need no more tiles
    const int64_t tiles_plain = tiles_x(width, t, vec);
    const bool align = vec && vol && ((int64_t)d.rows * width) % 32 == 0 &&
                       aligned_tiles(vol, d.rows, width, (int64_t)t.block * t.per_thread / 4) <=
                           tiles_plain;
    const int64_t tiles = tiles_plain;
    const int64_t edge = edge_blocks(d, width, t, vec, vol != nullptr);
    if (tiles * (int64_t)d.rows + edge > kMaxI32) return DSK_ESHAPE;
    hipError_t e;
    if (in_is_f32) {
        FwdArgs<float> a{(const float *)in, vol, psum, pmax, offs, shift, (double)origin,
                         width, d.planes, d.rows, d.cols, lay.row, lay.plane, lay.lo, lay.hi,
                         0u, 0u, 0, (int32_t)edge, (int64_t)d.rows * width, align ? 1 : 0};
        e = fwd_dispatch<float>(a, t, vec, tiles, edge, stream);
    } else {
        FwdArgs<uint16_t> a{(const uint16_t *)in, vol, psum, pmax, offs, shift, (double)origin,
                            width, d.planes, d.rows, d.cols, lay.row, lay.plane, lay.lo, lay.hi,
                            0u, 0u, 0, (int32_t)edge, (int64_t)d.rows * width, align ? 1 : 0};
        e = fwd_dispatch<uint16_t>(a, t, vec, tiles, edge, stream);
    }
    return hip_status(e);
}

int launch_forward(const void *in, int in_is_f32, dsk_dims d, const double *offs, double shift,
                   int64_t origin, float *vol, float *psum, float *pmax, int64_t width,
                   const dsk_tune &t, hipStream_t stream) {
    if (!dims_ok(d)) return DSK_EINVAL;
    return launch_forward_layout(in, in_is_f32, d, dense_layout(d), offs, shift, origin, vol,
                                 psum, pmax, width, t, stream);
}

}  // namespace dsk

extern "C" int dsk_deskew_u16(const uint16_t *in, dsk_dims d, dsk_geom g, float *vol,
                              float *psum, float *pmax, int64_t out_width,
                              hipStream_t stream) {
    if (!dims_ok(d) || out_width < 0) return DSK_EINVAL;
    double s = 0.0;
    int st = dsk_shift_px(g, &s);
    if (st != DSK_OK) return st;
    int64_t w = 0, b = 0;
    st = dsk_plan(d, nullptr, s, &w, &b);
    if (st != DSK_OK) return st;
    if (out_width > 0) w = out_width;
    return launch_forward(in, 0, d, nullptr, s, b, vol, psum, pmax, w, default_tune(vol), stream);
}

extern "C" int dsk_deskew_channel_u16(const uint16_t *frames, int64_t frame_cols, int64_t col0,
                                      dsk_dims d, dsk_geom g, float *vol, float *psum,
                                      float *pmax, int64_t out_width, hipStream_t stream) {
    if (!frames || !dims_ok(d) || out_width < 0 || col0 < 0 || frame_cols < col0 + d.cols)
        return DSK_EINVAL;
    if (frame_cols >= (int64_t(1) << 30)) return DSK_ESHAPE;
    double s = 0.0;
    int st = dsk_shift_px(g, &s);
    if (st != DSK_OK) return st;
    int64_t w = 0, b = 0;
    st = dsk_plan(d, nullptr, s, &w, &b);
    if (st != DSK_OK) return st;
    if (out_width > 0) w = out_width;
    const int64_t plane = (int64_t)d.rows * frame_cols;
    const InLayout lay{frame_cols, plane, col0, (int64_t)d.planes * plane - col0};
    return launch_forward_layout(frames + col0, 0, d, lay, nullptr, s, b, vol, psum, pmax, w,
                                 default_tune(vol), stream);
}

extern "C" int dsk_deskew_offsets_u16(const uint16_t *in, dsk_dims d, const double *offsets_dev,
                                      int64_t origin, float *vol, float *psum, float *pmax,
                                      int64_t out_width, hipStream_t stream) {
    if (!offsets_dev || out_width <= 0) return DSK_EINVAL;
    return launch_forward(in, 0, d, offsets_dev, 0.0, origin, vol, psum, pmax, out_width,
                          default_tune(vol), stream);
}

extern "C" int dsk_deskew_offsets_f32(const float *in, dsk_dims d, const double *offsets_dev,
                                      int64_t origin, float *vol, float *psum, float *pmax,
                                      int64_t out_width, hipStream_t stream) {
    if (!offsets_dev || out_width <= 0) return DSK_EINVAL;
    return launch_forward(in, 1, d, offsets_dev, 0.0, origin, vol, psum, pmax, out_width,
                          default_tune(vol), stream);
}

extern "C" int dsk_deskew_offsets_tuned(const void *in, int in_is_f32, dsk_dims d,
                                        const double *offsets_dev, double shift_px,
                                        int64_t origin, float *vol, float *psum, float *pmax,
                                        int64_t out_width, const dsk_tune *tune,
                                        hipStream_t stream) {
    if (out_width <= 0) return DSK_EINVAL;
    const dsk_tune t = tune ? *tune : default_tune(vol);
    return launch_forward(in, in_is_f32 ? 1 : 0, d, offsets_dev, shift_px, origin, vol, psum,
                          pmax, out_width, t, stream);
}

// ---------------------------------------------------------------- backward

namespace {

constexpr int kBwdBlock = 256;

// Rows per backward workgroup: about 8192 raw columns per workgroup.
int bwd_rows_per_block(dsk_dims d) {
    int64_t rpb = 8192 / (int64_t)d.cols;
    if (rpb < 1) rpb = 1;
    if (rpb > d.rows) rpb = d.rows;
    return (int)rpb;
}

int bwd_groups(dsk_dims d) {
    const int rpb = bwd_rows_per_block(d);
    return (d.rows + rpb - 1) / rpb;
}

bool gvol_ok(const float *gvol, const double *offs, dsk_dims d, const float *gin,
             const double *goff) {
    return gvol && offs && dims_ok(d) && (gin || goff);
}

int launch_backward(const float *in, const float *gvol, dsk_dims d, const double *offs,
                    int64_t origin, int64_t width, float *gin, double *goff, void *ws,
                    size_t ws_bytes, hipStream_t stream) {
    if (!gvol || !offs || !dims_ok(d) || (!gin && !goff)) return DSK_EINVAL;
    if (goff && (!in || !ws)) return DSK_EINVAL;
    int st = check_frame(d, origin, width);
    if (st != DSK_OK) return st;
    const int G = bwd_groups(d);
    const int64_t blocks = (int64_t)G * d.planes;
    if (blocks > kMaxI32) return DSK_ESHAPE;
    if (goff && ws_bytes < dsk_shear_grad_workspace_bytes(d)) return DSK_ESHAPE;
    BwdArgs a{in, gvol, gin, (double *)ws, offs, 0.0, (double)origin, width,
              d.planes, d.rows, d.cols, bwd_rows_per_block(d), G};
    const dim3 grid((unsigned)blocks), block(kBwdBlock);
    // 4 columns per thread when the rows of the stack and of the adjoint
    // start 16-byte aligned
    const bool vec = d.cols % 4 == 0 && (!goff || ((uintptr_t)in & 15) == 0) &&
                     (!gin || ((uintptr_t)gin & 15) == 0) && ((uintptr_t)gvol & 3) == 0;
    auto go = [&](auto V) {
        constexpr bool v = decltype(V)::value;
        if (gin && goff)
            hipLaunchKernelGGL((k_backward<kBwdBlock, true, true, v>), grid, block, 0, stream, a);
        else if (gin)
            hipLaunchKernelGGL((k_backward<kBwdBlock, true, false, v>), grid, block, 0, stream, a);
        else
            hipLaunchKernelGGL((k_backward<kBwdBlock, false, true, v>), grid, block, 0, stream, a);
    };
    if (vec)
        go(std::true_type{});
    else
        go(std::false_type{});
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return DSK_EHIP;
    if (goff) {
        hipLaunchKernelGGL(k_backward_finalize<0>, dim3((unsigned)d.planes), dim3(64), 0, stream,
                           (const double *)ws, d.planes, G, goff);
        e = hipGetLastError();
    }
    return hip_status(e);
}

}  // namespace

extern "C" size_t dsk_shear_grad_workspace_bytes(dsk_dims d) {
    if (!dims_ok(d)) return 0;
    return (size_t)bwd_groups(d) * (size_t)d.planes * sizeof(double);
}

extern "C" int dsk_deskew_adjoint_f32(const float *grad_vol, dsk_dims d,
                                      const double *offsets_dev, int64_t origin,
                                      int64_t out_width, float *grad_in, hipStream_t stream) {
    if (!grad_in) return DSK_EINVAL;
    return launch_backward(nullptr, grad_vol, d, offsets_dev, origin, out_width, grad_in,
                           nullptr, nullptr, 0, stream);
}

extern "C" int dsk_shear_grad_f32(const float *in, const float *grad_vol, dsk_dims d,
                                  const double *offsets_dev, int64_t origin, int64_t out_width,
                                  double *grad_offsets, void *workspace, size_t workspace_bytes,
                                  hipStream_t stream) {
    if (!grad_offsets) return DSK_EINVAL;
    return launch_backward(in, grad_vol, d, offsets_dev, origin, out_width, nullptr,
                           grad_offsets, workspace, workspace_bytes, stream);
}

extern "C" int dsk_backward_f32(const float *in, const float *grad_vol, dsk_dims d,
                                const double *offsets_dev, int64_t origin, int64_t out_width,
                                float *grad_in, double *grad_offsets, void *workspace,
                                size_t workspace_bytes, hipStream_t stream) {
    return launch_backward(in, grad_vol, d, offsets_dev, origin, out_width, grad_in,
                           grad_offsets, workspace, workspace_bytes, stream);
}

// ------------------------------------------------- backward, no allocation
//
// The shear gradient's per-(plane, row-group) partial sums live in a
// file-scope device array instead of a caller workspace.  Each device holds
// its own copy of the array; host code reaches it only through the address
// hipGetSymbolAddress returns for that device (the array's name is a host
// stand-in, not a device address).  Every partial is written by the
// backward kernel before the finalize kernel reads it, so nothing needs
// clearing between calls.

namespace {

constexpr size_t kScratchBytes = size_t(1) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {nullptr};

// Address of the current device's scratch array, looked up once per device.
int scratch_for_current_device(void **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return DSK_EHIP;
    if (dev < 0 || dev >= kMaxDevices) return DSK_EHIP;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return DSK_EHIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return DSK_OK;
}

}  // namespace

extern "C" int dsk_backward_f32_noalloc(const float *in, const float *grad_vol, dsk_dims d,
                                        const double *offsets_dev, int64_t origin,
                                        int64_t out_width, float *grad_in,
                                        double *grad_offsets, hipStream_t stream) {
    if (!gvol_ok(grad_vol, offsets_dev, d, grad_in, grad_offsets)) return DSK_EINVAL;
    void *ws = nullptr;
    if (grad_offsets) {
        if (dsk_shear_grad_workspace_bytes(d) > kScratchBytes) return DSK_ESHAPE;
        const int st = scratch_for_current_device(&ws);
        if (st != DSK_OK) return st;
    }
    return launch_backward(in, grad_vol, d, offsets_dev, origin, out_width, grad_in,
                           grad_offsets, ws, grad_offsets ? kScratchBytes : 0, stream);
}
