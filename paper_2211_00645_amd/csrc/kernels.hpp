// kernels.hpp -- gfx950 device code for the deskew (remap), its fused
// projections, its adjoint and the per-image shear gradient.
//
// Geometry (Eq. 1 and the remap paragraph of "Physical principles"):
// image n sits at offset o[n] (pixels) in a larger image of origin b; with
// o[n] - b = k + phi, output column x' of image n is
//     D = (1 - phi) * S[x' - k] + phi * S[x' - k - 1],  S = 0 outside [0, C).
// The max over images of D is the widefield-like view (Fig. 2d); the sum is
// accumulated in FP64 per output pixel.
//
// Layout: the forward kernels give every workgroup one (row r, column tile)
// pair and walk all planes n, so both projections stay in registers and are
// written once, with no atomics and no cross-workgroup traffic.  A thread
// owns `J` output columns spaced one workgroup apart, so every store and
// every load instruction of a wavefront covers consecutive addresses.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dsk {

// Per-plane interpolation coefficients, computed in FP64 from the offset
// exactly as the host plan does (no contraction: explicit round-to-nearest
// operations).  whi = 1 - phi and wlo = phi are each rounded once to FP32,
// so both weights keep full relative precision.
struct PlaneCoef {
    int32_t k;
    float wlo, whi;
};

__device__ __forceinline__ PlaneCoef coef_from_offset(double o, double origin) {
    const double t = __dsub_rn(o, origin);
    const double kf = floor(t);
    const double phi = __dsub_rn(t, kf);
    PlaneCoef c;
    // |k| beyond 2^30 only happens for an image entirely outside the frame
    // (width < 2^31); clamping keeps it outside and the index math in int32.
    const double kc = kf < -1073741824.0 ? -1073741824.0 : (kf > 1073741824.0 ? 1073741824.0 : kf);
    c.k = (int32_t)kc;
    c.wlo = (float)phi;
    c.whi = (float)__dsub_rn(1.0, phi);
    return c;
}

__device__ __forceinline__ PlaneCoef plane_coef(const double *offs, double shift,
                                                double origin, int n) {
    const double o = offs ? offs[n] : __dmul_rn((double)n, shift);
    return coef_from_offset(o, origin);
}

// Bounds checks of debug builds (compiled with DSK_CHECK_BOUNDS=1).  The
// forward and backward kernels pass every global address they read or write
// (or, for a row read pixel by pixel, the row's whole span) through
// bounded(), with the extent of the buffer their arguments describe.  A
// checking build counts each address outside its extent in a per-library
// counter (dsk_debug_bounds_violations reads it) and sends that access to
// the extent's first element instead, so that it never touches memory
// outside a buffer; other builds return the address unchanged.
#ifndef DSK_CHECK_BOUNDS
#define DSK_CHECK_BOUNDS 0
#endif

#if DSK_CHECK_BOUNDS
static __device__ unsigned long long g_bounds_violations;
#endif

template <typename T>
__device__ __forceinline__ T *bounded(T *p, int64_t n, const void *lo, const void *hi) {
#if DSK_CHECK_BOUNDS
    const char *c = (const char *)p;
    if (c < (const char *)lo || c + n * (int64_t)sizeof(T) > (const char *)hi) {
        atomicAdd(&g_bounds_violations, 1ull);
        return (T *)lo;
    }
#else
    (void)n;
    (void)lo;
    (void)hi;
#endif
    return p;
}

// Pixel i of a row of n, zero outside [0, n).  The load is unconditional, at
// an index clamped into the row, so neighbouring loads of a thread are
// issued together instead of each behind its own branch.
template <typename T>
__device__ __forceinline__ float load_px(const T *row, int64_t i, int64_t n) {
    const int64_t j = i < 0 ? 0 : (i >= n ? n - 1 : i);
    const float v = (float)row[j];
    return (i == j) ? v : 0.0f;
}

template <bool NT>
__device__ __forceinline__ void store_f32(float *p, float v) {
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// Per-plane coefficients for 64 planes at a time: lane l of every wavefront
// computes (k, wlo, whi) of plane base + l; plane n's values are then
// broadcast from lane n - base into scalar registers.  One FP64 evaluation
// (and, for explicit offsets, one vector load) per 64 planes instead of one
// per plane.
struct CoefCache {
    const double *offs;
    double shift, origin;
    int n_planes, base;
    int k;
    float wlo, whi;

    __device__ __forceinline__ void init(const double *o, double s, double org, int n) {
        offs = o;
        shift = s;
        origin = org;
        n_planes = n;
        base = -64;
        k = 0;
        wlo = whi = 0.0f;
    }

    __device__ __forceinline__ void refresh(int n) {
        base = n;
        const int l = n + (int)(threadIdx.x & 63);
        const int lc = l < n_planes ? l : n_planes - 1;
        double o;
        if (offs) {
            o = offs[lc];
            // consume the load here so the wait for it stays on this path
            asm volatile("" ::"v"(o));
        } else {
            o = __dmul_rn((double)lc, shift);
        }
        const PlaneCoef c = coef_from_offset(o, origin);
        k = c.k;
        wlo = c.wlo;
        whi = c.whi;
    }

    __device__ __forceinline__ PlaneCoef get(int n) {
        if (n - base >= 64) refresh(n);
        const int src = n - base;
        PlaneCoef c;
        c.k = __builtin_amdgcn_readlane(k, src);
        c.wlo = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wlo), src));
        c.whi = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(whi), src));
        return c;
    }
};

template <typename TIn>
struct FwdArgs {
    const TIn *in;
    float *vol, *psum, *pmax;
    const double *offs;  // device offsets or nullptr (o[n] = n * shift)
    double shift, origin;
    int64_t W;
    int32_t N, R, C;
    // Input layout in elements: row pitch, plane pitch, and the readable
    // extent around `in` ([in - in_lo, in + in_hi)).  A dense stack has
    // (C, R*C, 0, N*R*C); a channel of a wider camera frame has the frame's
    // pitches and the frame's extent.
    int64_t in_row, in_plane, in_lo, in_hi;
    // Plane pacing.  Batch launches give the period directly (tau256, in
    // 1/256 ticks of the 100 MHz real-time clock).  Plain launches give one
    // workgroup's share of a plane's time (tau_wg, 1/65536 ticks) and the
    // workgroups resident at once (pace_cap): workgroups start in id order
    // in batches of pace_cap, and a batch of m workgroups moves one plane
    // every m * tau_wg.  pace_cap = 0 and tau256 = 0: no pacing.
    uint32_t tau256;
    uint32_t tau_wg;
    int32_t pace_cap;
    // Workgroups of a vector launch that cover the edge columns, ahead of
    // the tiles (the host's edge_blocks).
    int32_t edge_wg;
    // Volume plane pitch in elements: R * W, or the whole frame's when the
    // launch covers a band of its rows (vol, psum and pmax then point at the
    // band's first row).
    int64_t vol_plane;
    // Vector launches with a volume whose plane pitch is a multiple of 32
    // floats: every row's tiles start on a 128-byte boundary of the volume
    // (the host adds a tile's worth of room: 7 groups per row).
    int32_t align_tiles;
};

// Plane pacing: a wavefront that reaches plane n before t0 + n * tau sleeps
// until then (at most kPaceSleeps short sleeps, so it never stalls for long
// and never depends on another wavefront).  Wavefronts left to themselves
// drift hundreds of planes apart, which scatters the write stream over the
// whole volume; pacing keeps them on neighbouring planes.
constexpr int kPaceSleeps = 4096;

__device__ __forceinline__ uint64_t pace_clock() { return __builtin_amdgcn_s_memrealtime(); }

__device__ __forceinline__ void pace_until(uint64_t t0, uint32_t tau256, int n) {
    if (tau256 == 0) return;
    const uint64_t target = t0 + (((uint64_t)n * tau256) >> 8);
    for (int i = 0; i < kPaceSleeps; ++i) {
        if (pace_clock() >= target) break;
        __builtin_amdgcn_s_sleep(2);
    }
}

// Spread consecutive workgroup ids, which the dispatcher deals round-robin
// to the 8 XCDs, so that each XCD receives a contiguous range of logical
// tiles (neighbouring tiles of a row then share that XCD's L2).  A
// bijection on [0, n).
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t n) {
    constexpr int64_t kXcd = 8;
    const int64_t q = n / kXcd, rem = n % kXcd;
    const int64_t x = b % kXcd, i = b / kXcd;
    return x * q + (x < rem ? x : rem) + i;
}

// ---- scalar variant: any alignment --------------------------------------
// Thread t owns columns x0 + t + j*BLOCK (j < J), so each load and store
// instruction of a wavefront touches consecutive addresses.
template <typename TIn, int BLOCK, int J, bool NT>
__device__ __forceinline__ void fwd_tile_scalar(const FwdArgs<TIn> &a, int r, int64_t x0) {
    double acc[J];
    float mx[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
        acc[j] = 0.0;
        mx[j] = -__builtin_huge_valf();
    }
    const int64_t C = a.C, W = a.W;
    CoefCache cc;
    cc.init(a.offs, a.shift, a.origin, a.N);
    for (int n = 0; n < a.N; ++n) {
        const PlaneCoef pc = cc.get(n);
        const TIn *row = bounded(a.in + (int64_t)n * a.in_plane + (int64_t)r * a.in_row, C,
                                 a.in - a.in_lo, a.in + a.in_hi);
        float *orow = a.vol ? a.vol + (int64_t)n * a.vol_plane + (int64_t)r * W : nullptr;
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int64_t x = x0 + threadIdx.x + (int64_t)j * BLOCK;
            if (x < W) {
                const int64_t i = x - pc.k;
                const float hi = load_px(row, i, C);
                const float lo = load_px(row, i - 1, C);
                const float d = fmaf(pc.whi, hi, pc.wlo * lo);
                if (orow)
                    store_f32<NT>(bounded(orow + x, 1, a.vol, a.vol + (int64_t)a.N * a.vol_plane), d);
                acc[j] += (double)d;
                mx[j] = fmaxf(mx[j], d);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const int64_t x = x0 + threadIdx.x + (int64_t)j * BLOCK;
        if (x < W) {
            const int64_t o = (int64_t)r * W + x, rw = (int64_t)a.R * W;
            if (a.psum) *bounded(a.psum + o, 1, a.psum, a.psum + rw) = (float)acc[j];
            if (a.pmax) *bounded(a.pmax + o, 1, a.pmax, a.pmax + rw) = mx[j];
        }
    }
}

// ---- vector variant ------------------------------------------------------
// Preconditions (checked on the host): rows*W and the plane pitch are
// multiples of 4, the stack is 8-byte (uint16) / 16-byte (float) aligned,
// the volume 16-byte aligned.  Then the flat volume index of (n, r, x') is
// 4-aligned exactly when x' + r*W is, independently of n, so a thread can
// own the same group of 4 columns in every plane and still write it with one
// 16-byte store.  The first tile of a row starts up to 3 columns left of 0 to
// reach that alignment.  A group's 5 source pixels come from one load: 12
// bytes from a dword-aligned uint16 element (then a 0- or 16-bit funnel shift
// that is the same for the whole wavefront), or 16 + 4 bytes of float.

typedef float f32x4 __attribute__((ext_vector_type(4)));

template <bool NT>
__device__ __forceinline__ void store_f32x4(float *p, f32x4 v) {
    if constexpr (NT)
        __builtin_nontemporal_store(v, (f32x4 *)p);
    else
        *(f32x4 *)p = v;
}

// Raw source window of one 4-column group.  uint16: the 6 pixels (12 bytes)
// starting at the even element at or one before the first needed pixel;
// float: the 5 pixels starting at the first needed pixel.  `sh` is the first
// needed pixel's place in the window (0 or 1 for uint16, 0 for float), the
// same for every lane of a wavefront in one plane.
template <typename TIn>
struct RawWin;

template <>
struct RawWin<uint16_t> {
    static constexpr int kAlign = 2;   // window starts are even elements
    static constexpr int kLen = 6;     // elements read
    uint32_t e0, e1, e2;
    __device__ __forceinline__ void load(const uint16_t *p) {
        const uint32_t *q = (const uint32_t *)__builtin_assume_aligned(p, 4);
        e0 = q[0];
        e1 = q[1];
        e2 = q[2];
    }
    // Wait for the load here (an empty asm that reads the registers), so no
    // load is pending across a loop back-edge: the wait counter is in-order
    // and shared with stores, and a pending load there would make the
    // compiler wait for every store issued since.
    __device__ __forceinline__ void settle() const {
        asm volatile("" ::"v"(e0), "v"(e1), "v"(e2));
    }
    __device__ __forceinline__ void extract(int sh, float v[5]) const {
        const uint32_t b = (uint32_t)sh * 16u;
        const uint32_t a0 = __builtin_amdgcn_alignbit(e1, e0, b);
        const uint32_t a1 = __builtin_amdgcn_alignbit(e2, e1, b);
        const uint32_t a2 = e2 >> b;
        v[0] = (float)(a0 & 0xffffu);
        v[1] = (float)(a0 >> 16);
        v[2] = (float)(a1 & 0xffffu);
        v[3] = (float)(a1 >> 16);
        v[4] = (float)(a2 & 0xffffu);
    }
};

template <>
struct RawWin<float> {
    static constexpr int kAlign = 1;
    static constexpr int kLen = 5;
    float4 a;
    float b;
    __device__ __forceinline__ void load(const float *p) {
        __builtin_memcpy(&a, p, sizeof(a));   // 4-byte aligned
        b = p[4];
    }
    __device__ __forceinline__ void settle() const {
        asm volatile("" ::"v"(a.x), "v"(a.y), "v"(a.z), "v"(a.w), "v"(b));
    }
    __device__ __forceinline__ void extract(int, float v[5]) const {
        v[0] = a.x;
        v[1] = a.y;
        v[2] = a.z;
        v[3] = a.w;
        v[4] = b;
    }
};

// Column layout of output row r for the vector kernel.  The flat volume
// index of (n, r, x') has the residue (r*W + x') mod 4 in every plane when
// rows*W is a multiple of 4, so the 4-aligned groups start at column ca and
// there are ng whole groups, [ca, ca + 4 ng).  The at most 3 columns before
// and 3 after (none when W is a multiple of 4) are the row's edge columns.
struct RowGeo {
    int ca, ng;
};

__device__ __forceinline__ RowGeo row_geo(int64_t r, int W) {
    RowGeo g;
    const int m = (int)((r * (int64_t)W) & 3);
    g.ca = (4 - m) & 3;
    g.ng = W > g.ca ? (W - g.ca) / 4 : 0;
    return g;
}

// Edge column j (0..5) of a row, or -1.
__device__ __forceinline__ int edge_col(const RowGeo &g, int W, int j) {
    if (j < 3) return (j < g.ca && j < W) ? j : -1;
    const int x = g.ca + 4 * g.ng + (j - 3);
    return (x < W && x >= g.ca) ? x : -1;
}

// One vector tile: row r, whole groups [tile*BLOCK*G, (tile+1)*BLOCK*G) of
// the row.  With a volume, thread t owns groups tile*BLOCK*G + t + BLOCK*g
// (a wavefront's stores of one group index are contiguous); without one, a
// lane's G groups sit side by side (wavefront w, lane l: groups
// tile*BLOCK*G + 64 G w + G l + g), so a wavefront reads one contiguous run
// of 256 G columns per plane.  Group indices are clamped to the row's last
// group, so every lane writes whole 16-byte groups (lanes past the end
// repeat the last group: identical values to identical addresses).
//
// Per-plane values come 64 planes at a time (a chunk): lane l of every
// wavefront computes plane (c0 + l)'s coefficients and window offset, and
// the wavefront classifies each plane for each of its groups: every pixel it
// reads inside the raw row (IN), every pixel outside (OUT: padding), or
// otherwise (MIXED).  Plane values reach the loop by readlane, so the scalar
// unit -- shared by all wavefronts of a compute unit -- does a handful of
// instructions per plane.
//
// With a volume (VOL) the tile walks chunk by chunk: an all-OUT chunk only
// stores zeros, an all-IN chunk runs a software-pipelined loop with plain
// loads, any other chunk the same loop with clamped loads and masks.  That
// pass is bound by its stores, and its loop is built to keep them in flight.
//
// Without a volume the pass only reads, and a pipeline that drains at every
// chunk or class boundary leaves the memory system idle each time all
// wavefronts drain together.  So the wavefront first finds the range of
// planes that touch any of its columns, then runs one software-pipelined
// loop over that range, all of its groups per plane: loads go out U planes
// ahead across chunk boundaries (the next chunk's values computed in
// advance), always with clamped addresses, and U planes are masked unless
// all of them are IN for every group.  Planes at the unaligned ends of the
// range, and planes whose rows lie at a stack end, go one at a time through
// the exact-bounds path.  A plane's window of a wavefront spans 256 G
// columns plus one: 4 G + 1 cache lines where 4 G carry its share, so wider
// lanes (G = 2) fetch fewer lines twice.
//
// Every path does the same per-voxel arithmetic and adds planes to the FP64
// sum in plane order, so no class or pass split changes a bit of the result.
template <typename TIn, int BLOCK, int G, int UNR, bool NT, bool VOL>
struct VecTile {
    enum { OUT = 0, IN = 1, MIXED = 2 };
    using Win = RawWin<TIn>;
    const FwdArgs<TIn> &a;
    int r, W, C, N, ca, ng, wv, lane, gpar;
    // window starts (elements from the row start) that keep a window of
    // Win::kLen elements, with the load's alignment, inside the stack away
    // from its two ends
    int lo_off, hi_off;
    int first_special, last_special;   // planes whose row lies at a stack end
    int64_t rstep, ostep;
    const TIn *rp0;                    // row r of plane 0
    float *op0;                        // volume row r of plane 0 (or null)
    int gi[G], gfirst[G], glast[G];
    bool alive;
    uint64_t t0;                       // pacing origin (this wavefront's start)
    uint32_t tau;                      // pacing period per plane, 1/256 ticks (0 = none)
    uint32_t taug;                     // per step of the wavefront's walk
    double acc[G][4];
    float mx[G][4];
    // chunk lane data (plane c0 + lane): first needed pixel of group 0 (s0),
    // window start and shift packed as (s0 - sh) * 2 + sh, and the weights
    int ls0, lwin;
    float lwlo, lwhi;

    __device__ __forceinline__ VecTile(const FwdArgs<TIn> &args, int row, int tile)
        : a(args), r(row), W((int)args.W), C(args.C), N(args.N) {
        const RowGeo rg = row_geo(r, W);
        ca = rg.ca;
        ng = rg.ng;
        rstep = a.in_plane;
        ostep = a.vol_plane;
        wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
        lane = (int)threadIdx.x & 63;
        int base = tile * BLOCK * G;
        if constexpr (VOL) {
            // shift the row's tile grid back by the groups that lie between
            // the previous 128-byte boundary of the volume and the row's
            // first group, so that each wavefront's 1 KB stores of a plane
            // cover 8 whole cache lines (a store run straddling lines leaves
            // partial lines that its neighbour completes much later, and the
            // launch then falls off its pacing schedule at paces that
            // line-aligned rows hold); the plane pitch being a multiple of 32
            // floats, the shift is the same in every plane
            if (a.align_tiles)
                base -= (int)((((uintptr_t)(a.vol + (int64_t)r * W + ca) >> 2) & 31) >> 2);
        }
        alive = base + (VOL ? 64 : 64 * G) * wv < ng;
        // the plane pitch is a multiple of 4, so every plane's row start has
        // this residue
        constexpr int K = Win::kAlign;
        gpar = (int)(((int64_t)r * a.in_row) & (K - 1));
        lo_off = -8 + ((K - (gpar + 8) % K) % K);
        hi_off = C - 1 - ((C - 1 + gpar) & (K - 1));
        // plane pitch >= 8: only plane 0 can start closer than 8 elements to
        // the readable start and only plane N-1 can end closer than 8 to its end
        const int64_t g0 = (int64_t)r * a.in_row;
        first_special = (g0 - 8 < -a.in_lo) ? 0 : -1;
        last_special = ((int64_t)(N - 1) * rstep + g0 + C + 8 > a.in_hi) ? N - 1 : -1;
        rp0 = a.in + (int64_t)r * a.in_row;
        op0 = VOL ? a.vol + (int64_t)r * W : nullptr;
        tau = a.tau256;
        if (a.pace_cap > 0) {
            // tiles start in id order after the edge columns' workgroups
            const int64_t eb = a.edge_wg;
            const int64_t cap = a.pace_cap, batch = ((int64_t)blockIdx.x - eb) / cap;
            const int64_t left = (int64_t)gridDim.x - eb - batch * cap;
            const uint64_t t = ((uint64_t)a.tau_wg * (uint64_t)(left < cap ? left : cap)) >> 8;
            tau = t > 4000000000ull ? 4000000000u : (uint32_t)t;
        }
        // with a volume a wavefront covers its G groups one after another,
        // chunk by chunk; without one, all of them per plane
        taug = VOL ? tau / G : tau;
        t0 = tau ? pace_clock() : 0;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            if constexpr (VOL) {
                // lanes before the row's first group (an aligned tile grid)
                // repeat it, as lanes past the last repeat the last
                const int w0 = base + 64 * wv + BLOCK * g;
                gi[g] = max(0, min(base + (int)threadIdx.x + BLOCK * g, ng - 1));
                gfirst[g] = max(0, min(w0, ng - 1));
                glast[g] = max(0, min(w0 + 63, ng - 1));
            } else {
                const int w0 = base + 64 * G * wv + g;
                gi[g] = min(w0 + G * lane, ng - 1);
                gfirst[g] = min(w0, ng - 1);
                glast[g] = min(w0 + G * 63, ng - 1);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                acc[g][i] = 0.0;
                mx[g][i] = -__builtin_huge_valf();
            }
        }
    }

    __device__ __forceinline__ int xcol(int g) const { return ca + 4 * gi[g]; }

    // Pacing position (in plane-groups) of chunk plane li of group g in the
    // chunk at c0: every earlier chunk is full, so G * c0 plane-groups lie
    // before it, and the chunk's groups run one after another.
    __device__ __forceinline__ int pace_pos(int g, int c0, int cn, int li) const {
        return c0 * G + g * cn + li;
    }

    // Positions [s0 + 4 gfirst, s0 + 4 glast + 5) of the wavefront's group g.
    __device__ __forceinline__ int cls_of(int s0, int g) const {
        return cls_range(s0 + 4 * gfirst[g], s0 + 4 * glast[g] + 5);
    }

    // All the wavefront's positions (groups side by side: group 0 holds the
    // lowest column, group G - 1 the highest).
    __device__ __forceinline__ int cls_span(int s0) const {
        return cls_range(s0 + 4 * gfirst[0], s0 + 4 * glast[G - 1] + 5);
    }

    __device__ __forceinline__ int cls_range(int q0, int q1) const {
        if (q0 >= 0 && q1 <= C) return IN;
        if (q1 <= 0 || q0 >= C) return OUT;
        return MIXED;
    }

    __device__ __forceinline__ void chunk(int c0) {
        const int n = min(c0 + lane, N - 1);
        double o;
        if (a.offs) {
            o = a.offs[n];
            // consume the load here so the wait for it stays on this path
            asm volatile("" ::"v"(o));
        } else {
            o = __dmul_rn((double)n, a.shift);
        }
        const PlaneCoef pc = coef_from_offset(o, a.origin);
        // first needed pixel of group 0; beyond +-2^28 every position lies
        // outside the row (rows and widths of this kernel are below 2^27):
        // clamp there
        const int s0l = ca - pc.k - 1;
        const int s0 = s0l < -(1 << 28) ? -(1 << 28) : (s0l > (1 << 28) ? (1 << 28) : s0l);
        const int sh = (gpar + s0) & (Win::kAlign - 1);
        ls0 = s0;
        lwin = (s0 - sh) * 2 + sh;
        lwlo = pc.wlo;
        lwhi = pc.whi;
    }

    __device__ __forceinline__ void interp(int g, const float v[5], float wlo, float whi,
                                           float d[4]) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            d[i] = fmaf(whi, v[i + 1], wlo * v[i]);
            acc[g][i] += (double)d[i];
            mx[g][i] = fmaxf(mx[g][i], d[i]);
        }
    }

    // Window of one plane: the packed start/shift v, clamped into [lo, hi]
    // when MASK (lanes reaching outside the row only read values that are
    // masked afterwards).
    template <bool MASK>
    __device__ __forceinline__ void fetch(int g, const TIn *rp, int v, Win &w) const {
        int off = (v >> 1) + 4 * gi[g];
        if (MASK) off = off < lo_off ? lo_off : (off > hi_off ? hi_off : off);
        w.load(bounded(rp + off, Win::kLen, a.in - a.in_lo, a.in + a.in_hi));
    }

    // Interpolate one plane from its window (v its packed start/shift).
    template <bool MASK>
    __device__ __forceinline__ void compute(int g, const Win &w, int v, float wlo, float whi,
                                            float d[4]) {
        const int sh = v & 1;
        float vv[5];
        w.extract(sh, vv);
        if (MASK) {
            const int p = (v >> 1) + sh + 4 * gi[g];
#pragma unroll
            for (int i = 0; i < 5; ++i)
                if ((unsigned)(p + i) >= (unsigned)C) vv[i] = 0.0f;
        }
        interp(g, vv, wlo, whi, d);
    }

    __device__ __forceinline__ float lane_f(float x, int li) const {
        return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), li));
    }

    // One plane with the window clamped to the stack's exact readable
    // extent when its row lies at a stack end (else to the row's
    // neighbourhood); lanes whose window moved reload per pixel.  win, wlo,
    // whi: the plane's chunk lane values, li its lane.
    __device__ __forceinline__ void single(int g, int n, int li, int win, float wlo_l, float whi_l,
                                           float d[4]) {
        constexpr int K = Win::kAlign;
        const TIn *rp = rp0 + (int64_t)n * rstep;
        const int v = __builtin_amdgcn_readlane(win, li);
        const int sh = v & 1;
        const float wlo = lane_f(wlo_l, li), whi = lane_f(whi_l, li);
        const int off = (v >> 1) + 4 * gi[g];
        const int p = off + sh;
        int lo = lo_off, hi = hi_off;
        if (n == first_special || n == last_special) {
            // the readable extent [in - in_lo, in + in_hi), as window starts
            // of this row with the load's alignment
            const int64_t grow = rp - a.in;
            int64_t lo_ok = -grow - a.in_lo, hi_ok = a.in_hi - Win::kLen - grow;
            lo_ok += (K - ((grow + lo_ok) % K + K) % K) % K;
            hi_ok -= ((grow + hi_ok) % K + K) % K;
            lo = (int)(lo_ok > (int64_t)lo ? lo_ok : (int64_t)lo);
            hi = (int)(hi_ok < (int64_t)hi ? hi_ok : (int64_t)hi);
        }
        const int oc = off < lo ? lo : (off > hi ? hi : off);
        Win raw;
        raw.load(bounded(rp + oc, Win::kLen, a.in - a.in_lo, a.in + a.in_hi));
        float vv[5];
        raw.extract(sh, vv);
#pragma unroll
        for (int i = 0; i < 5; ++i)
            if ((unsigned)(p + i) >= (unsigned)C) vv[i] = 0.0f;
        if (oc != off) {
#pragma unroll
            for (int i = 0; i < 5; ++i)
                vv[i] = load_px(bounded(rp, C, a.in - a.in_lo, a.in + a.in_hi), p + i, C);
        }
        interp(g, vv, wlo, whi, d);
    }

    // ---- with a volume ---------------------------------------------------

    __device__ __forceinline__ void store(int g, float *orow, const float d[4]) const {
        store_f32x4<NT>(bounded(orow + xcol(g), 4, a.vol, a.vol + (int64_t)N * a.vol_plane),
                        f32x4{d[0], d[1], d[2], d[3]});
    }

    // Chunk planes [l0, l1) of a chunk of cn planes for group g,
    // software-pipelined: the loads of the next U planes go out before the
    // current U planes are interpolated and stored, and are waited for after
    // those stores.  Each plane issues exactly one 16-byte store per lane
    // with no branch around it, so the compiler counts the stores and the
    // wait for the loads leaves them in flight: stores never hold up the
    // plane loop.
    template <int U, bool MASK>
    __device__ __forceinline__ void pipe_loop(int g, int c0, int cn, int l0, int l1,
                                              const TIn *rpc, float *op) {
        const int groups = (l1 - l0) / U;
        float *orow = op + (int64_t)l0 * ostep;
        int li = l0;
        if (groups > 0) {
            Win cur[U];
#pragma unroll
            for (int u = 0; u < U; ++u)
                fetch<MASK>(g, rpc + (int64_t)(l0 + u) * rstep,
                            __builtin_amdgcn_readlane(lwin, l0 + u), cur[u]);
#pragma unroll
            for (int u = 0; u < U; ++u) cur[u].settle();
            for (int k = 0; k < groups; ++k) {
                // the next U planes (past the range's end: its last plane,
                // in bounds, never used)
                Win nxt[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int ln = min(li + U + u, l1 - 1);
                    fetch<MASK>(g, rpc + (int64_t)ln * rstep, __builtin_amdgcn_readlane(lwin, ln),
                                nxt[u]);
                }
                // a paced wavefront sleeps with the next loads in flight
                pace_until(t0, taug, pace_pos(g, c0, cn, li));
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    float d[4];
                    compute<MASK>(g, cur[u], __builtin_amdgcn_readlane(lwin, li + u),
                                  lane_f(lwlo, li + u), lane_f(lwhi, li + u), d);
                    store(g, orow, d);
                    orow += ostep;
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    nxt[u].settle();
                    cur[u] = nxt[u];
                }
                li += U;
            }
        }
        for (; li < l1; ++li) {
            Win one;
            fetch<MASK>(g, rpc + (int64_t)li * rstep, __builtin_amdgcn_readlane(lwin, li), one);
            float d[4];
            compute<MASK>(g, one, __builtin_amdgcn_readlane(lwin, li), lane_f(lwlo, li),
                          lane_f(lwhi, li), d);
            store(g, orow, d);
            orow += ostep;
        }
    }

    // A plane whose row lies at a stack end (the chunk's plane li) through
    // the exact-bounds path.
    __device__ __forceinline__ void special_plane(int g, int c0, int li, float *op) {
        float d[4];
        single(g, c0 + li, li, lwin, lwlo, lwhi, d);
        store(g, op + (int64_t)li * ostep, d);
    }

    __device__ __forceinline__ void run_volume() {
        for (int c0 = 0; c0 < N; c0 += 64) {
            const int cn = min(64, N - c0);
            chunk(c0);
            // only plane 0 and plane N - 1 can be special, and only the
            // special plane itself leaves the chunk's loop: the others,
            // [l0, l1), run as in any chunk (a special chunk's planes at the
            // end of a launch, one at a time, held every other wavefront up)
            const bool sp_first = first_special == c0;
            const bool sp_last = last_special == c0 + cn - 1 && !(sp_first && cn == 1);
            const int l0 = sp_first ? 1 : 0;
            const int l1 = sp_last ? cn - 1 : (cn > l0 ? cn : l0);
            const TIn *rp = rp0 + (int64_t)c0 * rstep;
            float *op = op0 + (int64_t)c0 * ostep;
            const uint64_t valid = __builtin_amdgcn_ballot_w64(lane >= l0 && lane < l1);
#pragma unroll
            for (int g = 0; g < G; ++g) {
                if (sp_first) special_plane(g, c0, 0, op);
                const int cl = cls_of(ls0, g);
                const uint64_t bin = __builtin_amdgcn_ballot_w64(lane >= l0 && lane < l1 && cl == IN);
                const uint64_t bout =
                    __builtin_amdgcn_ballot_w64(lane >= l0 && lane < l1 && cl == OUT);
                if (valid == 0) {
                    // no plane besides the special ones
                } else if (bout == valid) {
                    // padding: zero output, nothing added to the sum
#pragma unroll
                    for (int i = 0; i < 4; ++i) mx[g][i] = fmaxf(mx[g][i], 0.0f);
                    float *orow = op + (int64_t)l0 * ostep;
                    const float z[4] = {0.0f, 0.0f, 0.0f, 0.0f};
                    for (int li = l0; li < l1; ++li) {
                        if ((li & 3) == 0) pace_until(t0, taug, pace_pos(g, c0, cn, li));
                        store(g, orow, z);
                        orow += ostep;
                    }
                } else if (bin == valid) {
                    pipe_loop<UNR, false>(g, c0, cn, l0, l1, rp, op);
                } else {
                    pipe_loop<UNR, true>(g, c0, cn, l0, l1, rp, op);
                }
                if (sp_last) special_plane(g, c0, cn - 1, op);
            }
        }
    }

    // ---- projections only ------------------------------------------------

    // Lane values of the chunk at c0 and the wavefront's IN / OUT ballots over
    // all its groups (bits of planes past the stack end clear).
    struct Chunk {
        int c0, win;
        float wlo, whi;
        uint64_t bin, bout;
    };

    __device__ __forceinline__ void load_chunk(int c0, Chunk &k) {
        chunk(c0);
        const int cn = min(64, N - c0);
        const int cl = cls_span(ls0);
        k.c0 = c0;
        k.win = lwin;
        k.wlo = lwlo;
        k.whi = lwhi;
        k.bin = __builtin_amdgcn_ballot_w64(lane < cn && cl == IN);
        k.bout = __builtin_amdgcn_ballot_w64(lane < cn && cl == OUT);
    }

    // Planes [n0, n1) one at a time (ascending), every group, each plane with
    // its chunk's values (k holds the chunk last loaded).
    __device__ __forceinline__ void singles(int n0, int n1, Chunk &k) {
        for (int n = n0; n < n1; ++n) {
            if (n < k.c0 || n >= k.c0 + 64) load_chunk(n & ~63, k);
            pace_until(t0, taug, n);
#pragma unroll
            for (int g = 0; g < G; ++g) {
                float d[4];
                single(g, n, n - k.c0, k.win, k.wlo, k.whi, d);
            }
        }
    }

    // Issue the window loads of planes n .. n + U - 1 (or U times plane n
    // with rep set), every group, each plane taking its values from the
    // chunk it lies in: cur or the next one.  n is a multiple of U (or rep),
    // so the planes lie in one chunk; when all of them are IN the addresses
    // need no clamping.
    template <int U>
    __device__ __forceinline__ void issue_planes(int n, bool rep, const Chunk &cur,
                                                 const Chunk &nxt, Win w[U][G], int v[U]) const {
        const Chunk &ch = n >= cur.c0 + 64 ? nxt : cur;
        const uint64_t full = rep ? 1ull : ((U == 64) ? ~0ull : ((1ull << U) - 1));
        if (((ch.bin >> (n - ch.c0)) & full) == full)
            issue_planes_as<U, false>(n, rep, ch, w, v);
        else
            issue_planes_as<U, true>(n, rep, ch, w, v);
    }

    template <int U, bool MASK>
    __device__ __forceinline__ void issue_planes_as(int n, bool rep, const Chunk &ch, Win w[U][G],
                                                    int v[U]) const {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int p = rep ? n : n + u;
            const int vv = __builtin_amdgcn_readlane(ch.win, p - ch.c0);
            v[u] = vv;
#pragma unroll
            for (int g = 0; g < G; ++g) fetch<MASK>(g, rp0 + (int64_t)p * rstep, vv, w[u][g]);
        }
    }

    template <int U>
    __device__ __forceinline__ static void settle_planes(const Win w[U][G]) {
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int g = 0; g < G; ++g) w[u][g].settle();
    }

    // Interpolate and accumulate planes n .. n + U - 1 (all in chunk cur),
    // masked unless all of them are IN.
    template <int U>
    __device__ __forceinline__ void compute_planes(int n, const Chunk &cur, const Win w[U][G],
                                                   const int v[U]) {
        const int li = n - cur.c0;
        const uint64_t full = (U == 64) ? ~0ull : ((1ull << U) - 1);
        float d[4];
        if (((cur.bin >> li) & full) == full) {
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int g = 0; g < G; ++g)
                    compute<false>(g, w[u][g], v[u], lane_f(cur.wlo, li + u),
                                   lane_f(cur.whi, li + u), d);
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int g = 0; g < G; ++g)
                    compute<true>(g, w[u][g], v[u], lane_f(cur.wlo, li + u),
                                  lane_f(cur.whi, li + u), d);
        }
    }

    __device__ __forceinline__ void run_projections() {
        constexpr int U = UNR;
        // planes that touch any of the wavefront's columns: [n_lo, n_hi);
        // per group, whether some plane misses all of its columns
        int n_lo = N, n_hi = 0;
        bool any_out[G];
#pragma unroll
        for (int g = 0; g < G; ++g) any_out[g] = false;
        Chunk k;
        for (int c0 = 0; c0 < N; c0 += 64) {
            load_chunk(c0, k);
            const int cn = min(64, N - c0);
#pragma unroll
            for (int g = 0; g < G; ++g)
                any_out[g] = any_out[g] ||
                             __builtin_amdgcn_ballot_w64(lane < cn && cls_of(ls0, g) == OUT) != 0;
            const uint64_t valid = cn == 64 ? ~0ull : ((1ull << cn) - 1);
            const uint64_t act = valid & ~k.bout;
            if (act) {
                n_lo = min(n_lo, c0 + (int)__builtin_ctzll(act));
                n_hi = max(n_hi, c0 + 64 - (int)__builtin_clzll(act));
            }
        }
        // a plane that misses all of a group's columns is zero at each of
        // them (inside the range such planes also come out zero, masked)
#pragma unroll
        for (int g = 0; g < G; ++g) {
            if (any_out[g]) {
#pragma unroll
                for (int i = 0; i < 4; ++i) mx[g][i] = fmaxf(mx[g][i], 0.0f);
            }
        }
        if (n_lo >= n_hi) return;
        // the pipelined range: whole steps of U planes, aligned (so a step
        // never spans two chunks), rows at a stack end excluded
        const int lo = n_lo + ((first_special == 0 && n_lo == 0) ? 1 : 0);
        const int hi = n_hi - ((last_special == N - 1 && n_hi == N) ? 1 : 0);
        int mlo = (lo + U - 1) / U * U, mhi = hi / U * U;
        if (mlo >= mhi) mlo = mhi = n_hi;
        singles(n_lo, mlo, k);
        if (mlo < mhi) {
            Chunk cur, nxt;
            load_chunk(mlo & ~63, cur);
            nxt = cur;
            if (cur.c0 + 64 < N) load_chunk(cur.c0 + 64, nxt);
            Win A[U][G], B[U][G];
            int va[U], vb[U];
            pace_until(t0, taug, mlo);
            issue_planes<U>(mlo, false, cur, nxt, A, va);
            settle_planes<U>(A);
            int n = mlo;
            // two steps per trip, alternating the window registers; a paced
            // wavefront sleeps with the next loads in flight
            while (true) {
                bool rep = n + U >= mhi;
                issue_planes<U>(rep ? mhi - 1 : n + U, rep, cur, nxt, B, vb);
                pace_until(t0, taug, n + U);
                compute_planes<U>(n, cur, A, va);
                settle_planes<U>(B);
                n += U;
                if (n >= mhi) break;
                if (n >= cur.c0 + 64) {
                    cur = nxt;
                    if (cur.c0 + 64 < N) load_chunk(cur.c0 + 64, nxt);
                }
                rep = n + U >= mhi;
                issue_planes<U>(rep ? mhi - 1 : n + U, rep, cur, nxt, A, va);
                pace_until(t0, taug, n + U);
                compute_planes<U>(n, cur, B, vb);
                settle_planes<U>(A);
                n += U;
                if (n >= mhi) break;
                if (n >= cur.c0 + 64) {
                    cur = nxt;
                    if (cur.c0 + 64 < N) load_chunk(cur.c0 + 64, nxt);
                }
            }
            k = cur;
        }
        singles(mhi, n_hi, k);
    }

    __device__ __forceinline__ void run() {
        if (!alive) return;
        if constexpr (VOL)
            run_volume();
        else
            run_projections();
#pragma unroll
        for (int g = 0; g < G; ++g) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t o = (int64_t)r * W + xcol(g) + i, rw = (int64_t)a.R * W;
                if (a.psum) *bounded(a.psum + o, 1, a.psum, a.psum + rw) = (float)acc[g][i];
                if (a.pmax) *bounded(a.pmax + o, 1, a.pmax, a.pmax + rw) = mx[g][i];
            }
        }
    }
};

// Edge columns of launches with a volume (the at most 3 unaligned columns
// at each end of every row, present only when W is not a multiple of 4,
// and then at least one per row): lane e handles slot e % 6 of row e / 6;
// empty slots and rows past
// the end repeat their row's first edge column (identical values to
// identical addresses), so every lane stays active -- the per-plane
// coefficients are shared across lanes -- and every store is unconditional.
// Two pixel loads per plane, issued UNR planes ahead of the stores.  Same
// per-voxel arithmetic and plane order as every other path.  Few lanes
// trickle through the planes beside the paced tiles for most of the
// launch; a burst of edge work at the start (the wavefront form below)
// puts the tiles behind their pacing schedule for good.
template <typename TIn, int UNR, bool NT>
__device__ __forceinline__ void fwd_edge_lane(const FwdArgs<TIn> &a, int e) {
    const int W = (int)a.W, C = a.C;
    const int r = min(e / 6, a.R - 1);
    const RowGeo rg = row_geo(r, W);
    int x = edge_col(rg, W, e - 6 * (e / 6));
    for (int j = 0; j < 6 && x < 0; ++j) x = edge_col(rg, W, j);
    if (x < 0) x = 0;   // unreachable when W % 4 != 0
    const int64_t rstep = a.in_plane, ostep = a.vol_plane;
    const TIn *rp = a.in + (int64_t)r * a.in_row;
    float *op = a.vol ? a.vol + (int64_t)r * W + x : nullptr;
    CoefCache cc;
    cc.init(a.offs, a.shift, a.origin, a.N);
    double acc = 0.0;
    float mx = -__builtin_huge_valf();
    float lo[UNR], hi[UNR], wlo[UNR], whi[UNR];
    auto issue = [&](int n0, float l[UNR], float h[UNR], float wl[UNR], float wh[UNR]) {
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const int n = min(n0 + u, a.N - 1);
            const PlaneCoef pc = cc.get(n);
            const int64_t i = (int64_t)x - pc.k;
            const TIn *row = bounded(rp + (int64_t)n * rstep, C, a.in - a.in_lo, a.in + a.in_hi);
            h[u] = load_px(row, i, (int64_t)C);
            l[u] = load_px(row, i - 1, (int64_t)C);
            wl[u] = pc.wlo;
            wh[u] = pc.whi;
        }
    };
    issue(0, lo, hi, wlo, whi);
#pragma unroll
    for (int u = 0; u < UNR; ++u) asm volatile("" ::"v"(lo[u]), "v"(hi[u]));
    for (int n0 = 0; n0 < a.N; n0 += UNR) {
        float lo2[UNR], hi2[UNR], wlo2[UNR], whi2[UNR];
        issue(n0 + UNR, lo2, hi2, wlo2, whi2);
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            if (n0 + u < a.N) {
                const float d = fmaf(whi[u], hi[u], wlo[u] * lo[u]);
                acc += (double)d;
                mx = fmaxf(mx, d);
                if (op)
                    store_f32<NT>(bounded(op + (int64_t)(n0 + u) * ostep, 1, a.vol,
                                          a.vol + (int64_t)a.N * a.vol_plane),
                                  d);
            }
        }
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            asm volatile("" ::"v"(lo2[u]), "v"(hi2[u]));
            lo[u] = lo2[u];
            hi[u] = hi2[u];
            wlo[u] = wlo2[u];
            whi[u] = whi2[u];
        }
    }
    const int64_t o = (int64_t)r * W + x, rw = (int64_t)a.R * W;
    if (a.psum) *bounded(a.psum + o, 1, a.psum, a.psum + rw) = (float)acc;
    if (a.pmax) *bounded(a.pmax + o, 1, a.pmax, a.pmax + rw) = mx;
}

// Edge columns of launches without a volume (the at most 3 unaligned columns at each end of every row,
// present only when W is not a multiple of 4, and then at least one per
// row): wavefront e handles slot e % 6 of row e / 6 (empty slots exit at
// once).  Its lanes take 64 planes at a time, one plane each: coefficients,
// the two pixel loads and the volume store run in parallel; the FP64 sum
// then adds the chunk's values in plane order, lane 0 first, as every other
// path does, and the maximum takes them in the same pass.  (One lane per
// column walking every plane alone took about 250 us for 512 planes, longer
// than the rest of a projections-only launch.)
template <typename TIn, bool NT>
__device__ __forceinline__ void fwd_edge_wave(const FwdArgs<TIn> &a, int64_t e) {
    const int W = (int)a.W, C = a.C, N = a.N;
    const int r = (int)(e / 6);
    if (r >= a.R) return;
    const RowGeo rg = row_geo(r, W);
    const int x = edge_col(rg, W, (int)(e - 6 * (e / 6)));
    if (x < 0) return;
    const int lane = (int)threadIdx.x & 63;
    const int64_t ostep = a.vol_plane;
    const TIn *rp = a.in + (int64_t)r * a.in_row;
    float *op = a.vol ? a.vol + (int64_t)r * W + x : nullptr;
    double acc = 0.0;
    float mx = -__builtin_huge_valf();
    for (int c0 = 0; c0 < N; c0 += 64) {
        const int cn = min(64, N - c0);
        const int n = min(c0 + lane, N - 1);
        const PlaneCoef pc = plane_coef(a.offs, a.shift, a.origin, n);
        const int64_t i = (int64_t)x - pc.k;
        const TIn *row =
            bounded(rp + (int64_t)n * a.in_plane, C, a.in - a.in_lo, a.in + a.in_hi);
        const float d = fmaf(pc.whi, load_px(row, i, (int64_t)C),
                             pc.wlo * load_px(row, i - 1, (int64_t)C));
        if (op && lane < cn)
            store_f32<NT>(bounded(op + (int64_t)n * ostep, 1, a.vol, a.vol + (int64_t)N * ostep),
                          d);
        for (int l = 0; l < cn; ++l) {
            const float dl = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(d), l));
            acc += (double)dl;
            mx = fmaxf(mx, dl);
        }
    }
    if (lane == 0) {
        const int64_t o = (int64_t)r * W + x, rw = (int64_t)a.R * W;
        if (a.psum) *bounded(a.psum + o, 1, a.psum, a.psum + rw) = (float)acc;
        if (a.pmax) *bounded(a.pmax + o, 1, a.pmax, a.pmax + rw) = mx;
    }
}

// Plain launches: one workgroup per (row, tile); vector launches add
// `edge_blocks` workgroups for the edge columns.
template <typename TIn, int BLOCK, int J, bool NT>
__global__ __launch_bounds__(BLOCK) void k_forward_scalar(FwdArgs<TIn> a, int tiles_x) {
    const int64_t b = xcd_remap(blockIdx.x, gridDim.x);
    const int r = (int)(b / tiles_x);
    const int xt = (int)(b - (int64_t)r * tiles_x);
    fwd_tile_scalar<TIn, BLOCK, J, NT>(a, r, (int64_t)xt * (BLOCK * J));
}

// Column tile of rank k in middle-out order over T tiles: the centre tile,
// then alternately right and left of it.  A bijection on [0, T).
__device__ __forceinline__ int middle_out(int k, int T) {
    const int c = (T - 1) / 2;
    return k == 0 ? c : ((k & 1) ? c + (k + 1) / 2 : c - k / 2);
}

// Block b of a plain launch.  With a volume: row-major tiles (paced launches
// start workgroups in id order, a batch of resident ones at a time).
// Without: the tiles of one column rank for every row, ranks middle-out, so
// the heaviest tiles start first (in a uniform scan a column tile meets the
// most planes at the frame's centre, the fewest at its ends) and lighter
// ones fill in behind them.
template <typename TIn, int BLOCK, int G, int UNR, bool NT, bool VOL>
__device__ __forceinline__ void fwd_vec_block(const FwdArgs<TIn> &a, int tiles_x, int64_t b) {
    // the edge columns' workgroups come first: they are short and start
    // with the first wave of tiles instead of waiting for free slots
    const int64_t eb = a.edge_wg;
    if (b < eb) {
        if constexpr (VOL)
            fwd_edge_lane<TIn, UNR, NT>(a, (int)(b * BLOCK + threadIdx.x));
        else
            fwd_edge_wave<TIn, NT>(a, b * (BLOCK / 64) + ((int)threadIdx.x >> 6));
        return;
    }
    b -= eb;
    {
        int r, xt;
        if constexpr (VOL) {
            r = (int)(b / tiles_x);
            xt = (int)(b - (int64_t)r * tiles_x);
        } else {
            const int k = (int)(b / a.R);
            r = (int)(b - (int64_t)k * a.R);
            xt = middle_out(k, tiles_x);
        }
        VecTile<TIn, BLOCK, G, UNR, NT, VOL> vt(a, r, xt);
        vt.run();
    }
}

// One group per lane with a shallow plane pipeline (UNR <= 2) writing the
// volume is built for 8 wavefronts per SIMD, so that a 512-row stack's tiles
// are all resident at once (plane pacing then holds every wavefront of the
// launch to one schedule).  Launches without a volume get the most
// wavefronts that leave room for their registers: about 36 besides the
// G groups' sums and maxima (12 each) and 2 U G plane windows (3 registers
// for 16-bit input, 5 for 32-bit), out of 512 per lane.  A 4-plane
// pipeline of 16-bit windows, one group per lane, fits 7 (72 registers),
// so the 512-row stack's 7168 tiles are again all resident at once.
constexpr int vec_waves_per_eu(int g, int unr, bool vol, int in_bytes) {
    if (vol) return g == 1 && unr <= 2 ? 8 : 1;
    const int need = 36 + 12 * g + 2 * unr * g * (in_bytes > 2 ? 5 : 3);
    const int w = 512 / ((need + 7) / 8 * 8);
    return w > 8 ? 8 : (w < 1 ? 1 : w);
}

template <typename TIn, int BLOCK, int G, int UNR, bool NT, bool VOL>
__global__ __launch_bounds__(BLOCK, vec_waves_per_eu(G, UNR, VOL, (int)sizeof(TIn))) void k_forward_vec(
    FwdArgs<TIn> a, int tiles_x) {
    // edge-column workgroups first, in dispatch order (spread over the
    // XCDs); with a volume the tiles after them are remapped so that each
    // XCD gets a contiguous range of them
    const int64_t eb = a.edge_wg, d = blockIdx.x;
    const int64_t lb = (VOL && d >= eb) ? eb + xcd_remap(d - eb, (int64_t)gridDim.x - eb) : d;
    fwd_vec_block<TIn, BLOCK, G, UNR, NT, VOL>(a, tiles_x, lb);
}

// Job record of the persistent ragged-batch kernel (device-resident table).
struct JobDev {
    const uint16_t *in;
    float *vol, *psum, *pmax;
    const double *offs;
    double shift, origin;
    int64_t W;
    int64_t tile_begin;  // first global tile index of this job
    int32_t N, R, C, tiles_x;
    int32_t vec, edge_blocks;
    uint32_t tau256;     // plane pacing period (see FwdArgs)
};

// Persistent launch: workgroups stride over the concatenated tile lists of
// all jobs (job-major).  Each tile runs exactly the code of the plain launch
// for that job, so outputs are bitwise equal.  One launch covers jobs that
// all write a volume (VOL) or all do not.
template <int BLOCK, int PT, int UNR, bool NT, bool VOL>
__global__ __launch_bounds__(BLOCK, vec_waves_per_eu(PT >= 8 ? 2 : 1, UNR, VOL, 2)) void k_forward_jobs(
    const JobDev *__restrict__ jobs, int n_jobs, int64_t total_tiles) {
    const int64_t grid = gridDim.x;
    const int64_t me = blockIdx.x;
    for (int64_t base = 0; base < total_tiles; base += grid) {
        const int64_t span = total_tiles - base < grid ? total_tiles - base : grid;
        if (me >= span) break;
        const int64_t t = base + xcd_remap(me, span);
        int lo = 0, hi = n_jobs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (jobs[mid].tile_begin <= t) lo = mid;
            else hi = mid - 1;
        }
        const JobDev &jb = jobs[lo];
        FwdArgs<uint16_t> a;
        a.in = jb.in;
        a.vol = jb.vol;
        a.psum = jb.psum;
        a.pmax = jb.pmax;
        a.offs = jb.offs;
        a.shift = jb.shift;
        a.origin = jb.origin;
        a.W = jb.W;
        a.N = jb.N;
        a.R = jb.R;
        a.C = jb.C;
        a.in_row = jb.C;
        a.in_plane = (int64_t)jb.R * jb.C;
        a.in_lo = 0;
        a.in_hi = (int64_t)jb.N * jb.R * jb.C;
        a.tau256 = jb.tau256;
        a.tau_wg = 0;
        a.pace_cap = 0;
        a.edge_wg = jb.edge_blocks;
        a.vol_plane = (int64_t)jb.R * jb.W;
        a.align_tiles = 0;
        const int64_t lt = t - jb.tile_begin;
        if constexpr (PT >= 4) {
            if (jb.vec) {
                fwd_vec_block<uint16_t, BLOCK, PT / 4, UNR, NT, VOL>(a, jb.tiles_x, lt);
                continue;
            }
        }
        const int r = (int)(lt / jb.tiles_x);
        const int xt = (int)(lt - (int64_t)r * jb.tiles_x);
        fwd_tile_scalar<uint16_t, BLOCK, PT, NT>(a, r, (int64_t)xt * (BLOCK * PT));
    }
}

// ---------------------------------------------------------------- backward

struct BwdArgs {
    const float *in;        // stack (for the shear gradient)
    const float *gvol;      // dLoss/dD  [N][R][W]
    float *gin;             // adjoint output [N][R][C] or nullptr
    double *partial;        // [N][G] shear-gradient partial sums or nullptr
    const double *offs;
    double shift, origin;
    int64_t W;
    int32_t N, R, C;
    int32_t rows_per_block, G;
};

// Deterministic sum of one FP64 value per thread over a workgroup.
template <int BLOCK>
__device__ __forceinline__ double block_sum(double v, double *lds) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) lds[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int w = 0; w < BLOCK / 64; ++w) s += lds[w];
    }
    return s;
}

// Adjoint as a gather over raw columns c of one image:
//   gin[c] = whi * gD[c + k] + wlo * gD[c + k + 1]
// and, from the same two reads, the shear-gradient contribution
//   S[c] * (gD[c + k + 1] - gD[c + k])
// (equal to summing gD[x'] * (S[x'-k-1] - S[x'-k]) over x').
// Workgroups are plane-major: block = n * G + g covers rows
// [g * rows_per_block, ...) of plane n.
template <int BLOCK, bool GIN, bool GOFF, bool VEC>
__global__ __launch_bounds__(BLOCK) void k_backward(BwdArgs a) {
    __shared__ double lds[BLOCK / 64];
    const int n = blockIdx.x / a.G;
    const int g = blockIdx.x - n * a.G;
    const PlaneCoef pc = plane_coef(a.offs, a.shift, a.origin, n);
    const int r0 = g * a.rows_per_block;
    const int r1 = min(a.R, r0 + a.rows_per_block);
    const int64_t C = a.C, W = a.W;
    double part = 0.0;
    for (int r = r0; r < r1; ++r) {
        const int64_t rowi = (int64_t)n * a.R + r, nr = (int64_t)a.N * a.R;
        const float *grow = bounded(a.gvol + rowi * W, W, a.gvol, a.gvol + nr * W);
        const float *srow = a.in;
        if constexpr (GOFF) srow = bounded(a.in + rowi * C, C, a.in, a.in + nr * C);
        float *orow = nullptr;
        if constexpr (GIN) orow = bounded(a.gin + rowi * C, C, a.gin, a.gin + nr * C);
        if constexpr (VEC) {
            // 4 adjacent raw columns per thread: their 5 gradient values
            // from one 16-byte and one 4-byte load (per pixel where the
            // window leaves [0, W)), the stack and the adjoint in 16 bytes
            for (int64_t c = 4 * (int64_t)threadIdx.x; c < C; c += 4 * BLOCK) {
                const int64_t x = c + pc.k;
                float gv[5];
                if (x >= 0 && x + 5 <= W) {
                    float4 q;
                    __builtin_memcpy(&q, grow + x, sizeof(q));   // 4-byte aligned
                    gv[0] = q.x;
                    gv[1] = q.y;
                    gv[2] = q.z;
                    gv[3] = q.w;
                    gv[4] = grow[x + 4];
                } else {
#pragma unroll
                    for (int i = 0; i < 5; ++i) gv[i] = load_px(grow, x + i, W);
                }
                if constexpr (GIN) {
                    f32x4 o;
                    o.x = fmaf(pc.whi, gv[0], pc.wlo * gv[1]);
                    o.y = fmaf(pc.whi, gv[1], pc.wlo * gv[2]);
                    o.z = fmaf(pc.whi, gv[2], pc.wlo * gv[3]);
                    o.w = fmaf(pc.whi, gv[3], pc.wlo * gv[4]);
                    store_f32x4<true>(orow + c, o);
                }
                if constexpr (GOFF) {
                    const float4 sv = *(const float4 *)(srow + c);   // 16-byte aligned
                    part += (double)sv.x * ((double)gv[1] - (double)gv[0]);
                    part += (double)sv.y * ((double)gv[2] - (double)gv[1]);
                    part += (double)sv.z * ((double)gv[3] - (double)gv[2]);
                    part += (double)sv.w * ((double)gv[4] - (double)gv[3]);
                }
            }
        } else {
            for (int64_t c = threadIdx.x; c < C; c += BLOCK) {
                const int64_t x = c + pc.k;
                const float g0 = load_px(grow, x, W);
                const float g1 = load_px(grow, x + 1, W);
                if constexpr (GIN) orow[c] = fmaf(pc.whi, g0, pc.wlo * g1);
                if constexpr (GOFF) part += (double)srow[c] * ((double)g1 - (double)g0);
            }
        }
    }
    if constexpr (GOFF) {
        const double s = block_sum<BLOCK>(part, lds);
        if (threadIdx.x == 0) a.partial[(int64_t)n * a.G + g] = s;
    }
}

// Fixed-order sum of the G partials of each plane, one wavefront per plane
// (blockIdx.x = plane, 64 threads): lane l adds partials l, l + 64, ... in
// turn (adjacent lanes read adjacent partials), then the 64 lane sums are
// halved pairwise (lane l + o into lane l for o = 32, 16, ..., 1), so the
// order of the additions is the same in every call.
template <int UNUSED = 0>
__global__ void __launch_bounds__(64) k_backward_finalize(const double *__restrict__ partial,
                                                          int N, int G,
                                                          double *__restrict__ gout) {
    const int n = blockIdx.x, l = threadIdx.x;
    if (n >= N) return;
    const double *p = partial + (int64_t)n * G;
    double s = 0.0;
    for (int g = l; g < G; g += 64) s += p[g];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    if (l == 0) gout[n] = s;
}

// ---------------------------------------------------------------- rolling
//
// Rolling update (the paper's rolling display mode, Fig. 4a): after every
// camera image the projections are refreshed.  Image n is remapped into
// leaf n of the volume; the FP64 running sum takes the difference between
// the new and the old leaf; the maximum is refreshed along a max-tree over
// images (level l holds ceil(N / 2^l) nodes of R x W, node j = max of nodes
// 2j and 2j+1 of level l-1; level 0 is the volume), since a maximum cannot be
// un-applied.  One thread per output pixel walks its path to the root.

struct RollArgs {
    const void *plane;     // raw image n, [R][C]
    float *vol;            // level 0: [N][R][W]
    float *tree;           // levels 1..L concatenated
    double *sum64;         // [R][W]
    float *psum, *pmax;    // [R][W]
    const double *offs;
    double shift, origin;
    int64_t W;
    int32_t N, R, C, n, levels;
};

template <typename TIn>
__global__ __launch_bounds__(256) void k_rolling_update(RollArgs a) {
    const int64_t RW = (int64_t)a.R * a.W;
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= RW) return;
    const int r = (int)(idx / a.W);
    const int64_t x = idx - (int64_t)r * a.W;
    const PlaneCoef pc = plane_coef(a.offs, a.shift, a.origin, a.n);
    const TIn *row = (const TIn *)a.plane + (int64_t)r * a.C;
    const int64_t i = x - pc.k;
    const float d = fmaf(pc.whi, load_px(row, i, (int64_t)a.C), pc.wlo * load_px(row, i - 1, (int64_t)a.C));
    float *leaf = a.vol + (int64_t)a.n * RW + idx;
    const float old = *leaf;
    *leaf = d;
    const double sum = a.sum64[idx] + ((double)d - (double)old);
    a.sum64[idx] = sum;
    a.psum[idx] = (float)sum;
    float m = d;
    int j = a.n, cnt = a.N;
    const float *below = a.vol;
    float *lev = a.tree;
    for (int l = 0; l < a.levels; ++l) {
        const int sib = j ^ 1;
        if (sib < cnt) m = fmaxf(m, below[(int64_t)sib * RW + idx]);
        j >>= 1;
        const int next = (cnt + 1) >> 1;
        lev[(int64_t)j * RW + idx] = m;
        below = lev;
        lev += (int64_t)next * RW;
        cnt = next;
    }
    a.pmax[idx] = m;
}

// The same update, 4 consecutive pixels of the R x W plane per thread
// (R*W a multiple of 4 and every array 16-byte aligned): the leaf, the
// running sum, both projections and every tree node move in 16-byte
// accesses instead of one 4- or 8-byte access per pixel and lane.  The
// per-pixel arithmetic is the one-pixel kernel's.
template <typename TIn>
__global__ __launch_bounds__(256) void k_rolling_update4(RollArgs a) {
    const int64_t RW = (int64_t)a.R * a.W;
    const int64_t idx = 4 * ((int64_t)blockIdx.x * 256 + threadIdx.x);
    if (idx >= RW) return;
    const PlaneCoef pc = plane_coef(a.offs, a.shift, a.origin, a.n);
    int64_t r = idx / a.W;
    int64_t x = idx - r * a.W;
    float d[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        while (x >= a.W) {
            x -= a.W;
            ++r;
        }
        const TIn *row = (const TIn *)a.plane + r * a.C;
        const int64_t i = x - pc.k;
        d[e] = fmaf(pc.whi, load_px(row, i, (int64_t)a.C), pc.wlo * load_px(row, i - 1, (int64_t)a.C));
        ++x;
    }
    float *leaf = a.vol + (int64_t)a.n * RW + idx;
    const f32x4 old = *(const f32x4 *)leaf;
    *(f32x4 *)leaf = f32x4{d[0], d[1], d[2], d[3]};
    double2 s01 = *(const double2 *)(a.sum64 + idx);
    double2 s23 = *(const double2 *)(a.sum64 + idx + 2);
    s01.x = s01.x + ((double)d[0] - (double)old.x);
    s01.y = s01.y + ((double)d[1] - (double)old.y);
    s23.x = s23.x + ((double)d[2] - (double)old.z);
    s23.y = s23.y + ((double)d[3] - (double)old.w);
    *(double2 *)(a.sum64 + idx) = s01;
    *(double2 *)(a.sum64 + idx + 2) = s23;
    *(f32x4 *)(a.psum + idx) = f32x4{(float)s01.x, (float)s01.y, (float)s23.x, (float)s23.y};
    f32x4 m = f32x4{d[0], d[1], d[2], d[3]};
    int j = a.n, cnt = a.N;
    const float *below = a.vol;
    float *lev = a.tree;
    for (int l = 0; l < a.levels; ++l) {
        const int sib = j ^ 1;
        if (sib < cnt) {
            const f32x4 b = *(const f32x4 *)(below + (int64_t)sib * RW + idx);
            m.x = fmaxf(m.x, b.x);
            m.y = fmaxf(m.y, b.y);
            m.z = fmaxf(m.z, b.z);
            m.w = fmaxf(m.w, b.w);
        }
        j >>= 1;
        const int next = (cnt + 1) >> 1;
        *(f32x4 *)(lev + (int64_t)j * RW + idx) = m;
        below = lev;
        lev += (int64_t)next * RW;
        cnt = next;
    }
    *(f32x4 *)(a.pmax + idx) = m;
}

// Fill n floats (or doubles) with zero; a kernel, so it is safe inside a
// captured graph.
template <typename T>
__global__ __launch_bounds__(256) void k_zero(T *p, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) p[i] = T(0);
}

#if DSK_CHECK_BOUNDS
// Host side: this translation unit's count of addresses outside their
// extents, zeroed after reading when asked.  0, or -1 on a HIP error.
static inline int read_bounds_violations(unsigned long long *count, bool reset) {
    unsigned long long v = 0;
    if (hipMemcpyFromSymbol(&v, HIP_SYMBOL(g_bounds_violations), sizeof v) != hipSuccess)
        return -1;
    if (reset) {
        const unsigned long long z = 0;
        if (hipMemcpyToSymbol(HIP_SYMBOL(g_bounds_violations), &z, sizeof z) != hipSuccess)
            return -1;
    }
    *count = v;
    return 0;
}
#endif

}  // namespace dsk
