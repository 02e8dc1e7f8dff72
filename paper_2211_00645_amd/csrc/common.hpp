// common.hpp -- host-side helpers shared by the translation units of
// libdeskew.so (validation, launch-shape checks, HIP error mapping).
#pragma once

#include <cmath>
#include <cstdint>
#include <type_traits>

#include "deskew.h"

namespace dsk {

constexpr int64_t kMaxI32 = 2147483647;

// Default forward launch shape: 64-thread workgroups, one 4-column group per
// lane, non-temporal stores, 2-plane pipeline (built for 8 waves per SIMD),
// paced at 5700 GB/s.  On the 512x512x2048 stack, back to back, the launch
// time follows the pace (bytes / pace + about 3 us) up to the cliff:
// 5600: 0.853 ms, 5700: 0.839, 5800: 0.824; past it the wavefronts fall
// behind the schedule, stop sleeping and drift apart (unpaced 1.01-1.06
// ms).  With each row's tiles on 128-byte boundaries of the volume that
// frame holds 5800 (0.828 ms over the timed runs) and its cliff lies past
// 5900, but other frames put it anywhere between 5000 and 6000 GB/s, so
// the default keeps a step of margin and dsk_deskew_autotune finds the
// cliff of a given frame on the device at hand.
constexpr dsk_tune kDefaultTune = {64, 4, 1, 2, 0, 5700};

// Default shape of launches without a volume (projections only, the live
// view): a 4-plane load-ahead keeps enough reads in flight (on the
// 512x512x2048 stack 0.228 ms against 0.240 for 2 planes), paced at 9000
// GB/s.  They only read; a pace above what the device reaches never holds a
// running wavefront back, it only makes the wavefronts whose plane range
// starts late (the frame's outer column tiles) wait for their turn instead
// of competing with the others at the start: 0.238 -> 0.219 ms on that
// stack.  A frame with more tiles than resident workgroups is not paced
// (fwd_launch): its second round of tiles would wait out a schedule that
// began before they did (1-3% slower when they were).
constexpr dsk_tune kDefaultProjTune = {64, 4, 1, 4, 0, 9000};

inline const dsk_tune &default_tune(const void *vol) {
    return vol ? kDefaultTune : kDefaultProjTune;
}

inline bool dims_ok(dsk_dims d) {
    return d.planes > 0 && d.rows > 0 && d.cols > 0;
}

inline bool tune_ok(const dsk_tune &t) {
    const bool b = t.block == 64 || t.block == 128 || t.block == 256;
    const bool j = t.per_thread == 1 || t.per_thread == 2 || t.per_thread == 4 ||
                   t.per_thread == 8;
    const bool u = t.unroll == 1 || t.unroll == 2 || t.unroll == 4;
    return b && j && u && (t.nt_store == 0 || t.nt_store == 1) && t.wg_per_cu >= 0 &&
           t.wg_per_cu <= 64 && t.pace_gbs >= 0 && t.pace_gbs <= 1000000;
}

// Compute units of the current device (cached per device).
int device_cus();

// The aligned vector kernel applies when every row's flat volume and stack
// offsets keep one residue mod 4 across planes and the buffers are aligned.
inline bool vec_ok(const dsk_tune &t, dsk_dims d, int64_t width, const void *in, int in_is_f32,
                   const float *vol, int64_t in_plane) {
    if (t.per_thread < 4) return false;
    if ((int64_t)d.planes * d.rows * d.cols < 64 || in_plane < 8) return false;
    if (width >= (int64_t(1) << 27) || d.cols >= (1 << 27)) return false;
    if (((int64_t)d.rows * width) % 4 != 0 || in_plane % 4 != 0) return false;
    const uintptr_t ia = in_is_f32 ? 15 : 7;
    if ((uintptr_t)in & ia) return false;
    if (vol && ((uintptr_t)vol & 15)) return false;
    return true;
}

// Column tiles of one output row.  The vector kernel tiles the row's whole
// 4-aligned groups (at most W/4 of them); the scalar kernel tiles columns.
inline int64_t tiles_x(int64_t width, const dsk_tune &t, bool vec) {
    const int64_t tile = (int64_t)t.block * t.per_thread;
    if (vec) {
        const int64_t groups = width / 4, per = tile / 4;
        const int64_t n = (groups + per - 1) / per;
        return n > 0 ? n : 1;
    }
    return (width + tile - 1) / tile;
}

// Workgroups of the vector kernel for the rows' unaligned edge columns
// (none when the width is a multiple of 4), which it runs first: with a
// volume one lane per (row, slot of 6), without one a wavefront per (row,
// slot), block / 64 wavefronts per workgroup.  The kernel receives the
// count.
inline int64_t edge_blocks(dsk_dims d, int64_t width, const dsk_tune &t, bool vec, bool vol) {
    if (!vec || width % 4 == 0) return 0;
    const int64_t per = vol ? t.block : t.block / 64;
    return (6 * (int64_t)d.rows + per - 1) / per;
}

template <int V>
using IC = std::integral_constant<int, V>;

// Calls f(IC<block>, IC<per_thread>, IC<unroll>, bool_constant<nt>) for a
// validated launch shape.
template <typename F>
auto dispatch_tune(const dsk_tune &t, F &&f) {
    auto with_u = [&](auto B, auto P) {
        auto with_nt = [&](auto U) {
            return t.nt_store ? f(B, P, U, std::true_type{}) : f(B, P, U, std::false_type{});
        };
        switch (t.unroll) {
        case 1: return with_nt(IC<1>{});
        case 2: return with_nt(IC<2>{});
        default: return with_nt(IC<4>{});
        }
    };
    auto with_p = [&](auto B) {
        switch (t.per_thread) {
        case 1: return with_u(B, IC<1>{});
        case 2: return with_u(B, IC<2>{});
        case 4: return with_u(B, IC<4>{});
        default: return with_u(B, IC<8>{});
        }
    };
    switch (t.block) {
    case 64: return with_p(IC<64>{});
    case 128: return with_p(IC<128>{});
    default: return with_p(IC<256>{});
    }
}

// Output width and columns stay below 2^30 so that every column index of the
// kernels (x' and x' - k, with k clamped to +-2^30) fits the index types.
inline int check_frame(dsk_dims d, int64_t origin, int64_t width) {
    if (width <= 0 || width >= (int64_t(1) << 30) || d.cols >= (1 << 30)) return DSK_ESHAPE;
    if (origin < -(int64_t(1) << 52) || origin > (int64_t(1) << 52)) return DSK_ESHAPE;
    return DSK_OK;
}

inline int hip_status(hipError_t e) { return e == hipSuccess ? DSK_OK : DSK_EHIP; }

// Input layout in elements (see FwdArgs): row pitch, plane pitch and the
// readable extent [in - lo, in + hi).
struct InLayout {
    int64_t row, plane, lo, hi;
};

inline InLayout dense_layout(dsk_dims d) {
    return InLayout{d.cols, (int64_t)d.rows * d.cols, 0, (int64_t)d.planes * d.rows * d.cols};
}

#if defined(DSK_CHECK_BOUNDS) && DSK_CHECK_BOUNDS
// Bounds-violation count of the batch kernels' translation unit (batch.hip).
int batch_bounds_violations(unsigned long long *count, bool reset);
#endif

// Launchers (deskew.hip) used by the other translation units.
int launch_forward(const void *in, int in_is_f32, dsk_dims d, const double *offs,
                   double shift, int64_t origin, float *vol, float *psum, float *pmax,
                   int64_t width, const dsk_tune &t, hipStream_t stream);
int launch_forward_layout(const void *in, int in_is_f32, dsk_dims d, const InLayout &lay,
                          const double *offs, double shift, int64_t origin, float *vol,
                          float *psum, float *pmax, int64_t width, const dsk_tune &t,
                          hipStream_t stream);

}  // namespace dsk
