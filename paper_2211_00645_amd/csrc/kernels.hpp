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
};

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
        const int64_t rowi = (int64_t)n * a.R + r;
        const TIn *row = a.in + rowi * C;
        float *orow = a.vol ? a.vol + rowi * W : nullptr;
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int64_t x = x0 + threadIdx.x + (int64_t)j * BLOCK;
            if (x < W) {
                const int64_t i = x - pc.k;
                const float hi = load_px(row, i, C);
                const float lo = load_px(row, i - 1, C);
                const float d = fmaf(pc.whi, hi, pc.wlo * lo);
                if (orow) store_f32<NT>(orow + x, d);
                acc[j] += (double)d;
                mx[j] = fmaxf(mx[j], d);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const int64_t x = x0 + threadIdx.x + (int64_t)j * BLOCK;
        if (x < W) {
            if (a.psum) a.psum[(int64_t)r * W + x] = (float)acc[j];
            if (a.pmax) a.pmax[(int64_t)r * W + x] = mx[j];
        }
    }
}

// ---- vector variant ------------------------------------------------------
// Preconditions (checked on the host): rows*W and rows*C are multiples of 4,
// the stack is 8-byte (uint16) / 16-byte (float) aligned, the volume 16-byte
// aligned.  Then the flat volume index of (n, r, x') is 4-aligned exactly
// when x' + r*W is, independently of n, so a thread can own the same group
// of 4 columns in every plane and still write it with one 16-byte store.
// The first tile of a row starts up to 3 columns left of 0 to reach that
// alignment.  Its 5 source pixels come from two aligned 8-byte (16-byte for
// float) loads and a funnel shift whose amount is the same for the whole
// tile.

typedef float f32x4 __attribute__((ext_vector_type(4)));

template <bool NT>
__device__ __forceinline__ void store_f32x4(float *p, f32x4 v) {
    if constexpr (NT)
        __builtin_nontemporal_store(v, (f32x4 *)p);
    else
        *(f32x4 *)p = v;
}

// Raw source window of one 4-column group: 8 uint16 (16 bytes) starting at
// a 4-aligned element, or 5 floats starting at the first needed element.
template <typename TIn>
struct RawWin;

template <>
struct RawWin<uint16_t> {
    uint4 q;
    // sh: position of the first needed element inside the aligned window
    __device__ __forceinline__ void load(const uint16_t *row, int p, int sh) {
        __builtin_memcpy(&q, row + (p - sh), sizeof(q));   // 8-byte aligned
    }
    __device__ __forceinline__ void extract(int sh, float v[5]) const {
        const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#define DSK_LO(e) (float)(w[(e) >> 1] & 0xffffu)
#define DSK_HI(e) (float)(w[(e) >> 1] >> 16)
#define DSK_EL(e) (((e)&1) ? DSK_HI(e) : DSK_LO(e))
        switch (sh) {
        case 0: v[0] = DSK_EL(0); v[1] = DSK_EL(1); v[2] = DSK_EL(2); v[3] = DSK_EL(3); v[4] = DSK_EL(4); break;
        case 1: v[0] = DSK_EL(1); v[1] = DSK_EL(2); v[2] = DSK_EL(3); v[3] = DSK_EL(4); v[4] = DSK_EL(5); break;
        case 2: v[0] = DSK_EL(2); v[1] = DSK_EL(3); v[2] = DSK_EL(4); v[3] = DSK_EL(5); v[4] = DSK_EL(6); break;
        default: v[0] = DSK_EL(3); v[1] = DSK_EL(4); v[2] = DSK_EL(5); v[3] = DSK_EL(6); v[4] = DSK_EL(7); break;
        }
#undef DSK_EL
#undef DSK_HI
#undef DSK_LO
    }
};

template <>
struct RawWin<float> {
    float4 a;
    float b;
    __device__ __forceinline__ void load(const float *row, int p, int) {
        __builtin_memcpy(&a, row + p, sizeof(a));   // 4-byte aligned
        b = row[p + 4];
    }
    __device__ __forceinline__ void extract(int, float v[5]) const {
        v[0] = a.x;
        v[1] = a.y;
        v[2] = a.z;
        v[3] = a.w;
        v[4] = b;
    }
};

// One vector tile: row r, columns [x0, x0 + 4*BLOCK*G).  Thread t owns the
// 4-column groups starting at x0 + 4*(t + BLOCK*g).
template <typename TIn, int BLOCK, int G, bool NT>
struct VecTile {
    static constexpr int T = 4 * BLOCK * G;
    enum { OUT = 0, IN = 1, EDGE = 2 };
    const FwdArgs<TIn> &a;
    int r, W, C, x0, wv;
    int64_t total;
    bool full[G], wfull[G];
    double acc[G][4];
    float mx[G][4];
    CoefCache cc;

    __device__ __forceinline__ VecTile(const FwdArgs<TIn> &args, int row, int x0_)
        : a(args), r(row), W((int)args.W), C(args.C), x0(x0_) {
        total = (int64_t)a.N * a.R * C;
        wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int xg = x0 + 4 * ((int)threadIdx.x + BLOCK * g);
            full[g] = xg >= 0 && xg + 4 <= W;
            // every group of this wavefront is whole
            const int w0 = x0 + 4 * (64 * wv + BLOCK * g);
            wfull[g] = w0 >= 0 && w0 + 256 <= W;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                acc[g][i] = 0.0;
                mx[g][i] = -__builtin_huge_valf();
            }
        }
        cc.init(a.offs, a.shift, a.origin, a.N);
    }

    __device__ __forceinline__ int xg(int g) const {
        return x0 + 4 * ((int)threadIdx.x + BLOCK * g);
    }

    __device__ __forceinline__ void store(float *orow, int g, const float d[4]) const {
        float *o = orow + xg(g);
        if (wfull[g] || full[g]) {
            store_f32x4<NT>(o, f32x4{d[0], d[1], d[2], d[3]});
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (xg(g) + i >= 0 && xg(g) + i < W) store_f32<NT>(o + i, d[i]);
        }
    }

    // Planes [n0, n0 + U): loads of all U planes first, then interpolation.
    template <int U>
    __device__ __forceinline__ void planes(int n0) {
        RawWin<TIn> raw[U][G];
        PlaneCoef pc[U];
        const TIn *row[U];
        int s0[U], sh[U], cls[U][G];
        bool moved[U][G];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int n = n0 + u;
            pc[u] = cc.get(n);
            const int64_t grow = ((int64_t)n * a.R + r) * C;
            row[u] = a.in + grow;
            // window start; beyond +-2^28 every position lies outside the row
            // (rows and widths of this kernel are below 2^27), so clamp there
            const int s0l = x0 - pc[u].k - 1;
            s0[u] = s0l < -(1 << 28) ? -(1 << 28) : (s0l > (1 << 28) ? (1 << 28) : s0l);
            sh[u] = (int)((grow + s0[u]) & 3);   // same for every group
            // window starts the stack bounds allow, relative to the row
            const int lo_off = (int)(grow < 8 ? -grow : -8);
            const int64_t hi64 = total - grow - 8;
            const int hi_off = (int)(hi64 < (int64_t)C + 8 ? hi64 : (int64_t)C + 8);
#pragma unroll
            for (int g = 0; g < G; ++g) {
                // positions [q0, q0 + 256 + 1) of this wavefront's groups
                const int q0 = s0[u] + 4 * (64 * wv + BLOCK * g);
                const int q1 = q0 + 4 * 63 + 5;
                cls[u][g] = (q0 >= 0 && q1 <= C) ? IN : ((q1 <= 0 || q0 >= C) ? OUT : EDGE);
                const int p = s0[u] + 4 * ((int)threadIdx.x + BLOCK * g);
                moved[u][g] = false;
                if (cls[u][g] == IN) {
                    raw[u][g].load(row[u], p, sh[u]);
                } else if (cls[u][g] == EDGE) {
                    const int off = p - sh[u];
                    const int oc = off < lo_off ? lo_off : (off > hi_off ? hi_off : off);
                    moved[u][g] = oc != off;
                    raw[u][g].load(row[u], oc + sh[u], sh[u]);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int n = n0 + u;
            float *orow = a.vol ? a.vol + ((int64_t)n * a.R + r) * W : nullptr;
#pragma unroll
            for (int g = 0; g < G; ++g) {
                float d[4];
                if (cls[u][g] == OUT) {
                    // padding: zero output, nothing to add to the sum
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        d[i] = 0.0f;
                        mx[g][i] = fmaxf(mx[g][i], 0.0f);
                    }
                } else {
                    float v[5];
                    raw[u][g].extract(sh[u], v);
                    if (cls[u][g] == EDGE) {
                        const int p = s0[u] + 4 * ((int)threadIdx.x + BLOCK * g);
#pragma unroll
                        for (int i = 0; i < 5; ++i)
                            if (p + i < 0 || p + i >= C) v[i] = 0.0f;
                        if (moved[u][g]) {
#pragma unroll
                            for (int i = 0; i < 5; ++i) v[i] = load_px(row[u], p + i, C);
                        }
                    }
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        d[i] = fmaf(pc[u].whi, v[i + 1], pc[u].wlo * v[i]);
                        acc[g][i] += (double)d[i];
                        mx[g][i] = fmaxf(mx[g][i], d[i]);
                    }
                }
                if (orow) store(orow, g, d);
            }
        }
    }

    __device__ __forceinline__ void finish() {
#pragma unroll
        for (int g = 0; g < G; ++g) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int x = xg(g) + i;
                if (x >= 0 && x < W) {
                    if (a.psum) a.psum[(int64_t)r * W + x] = (float)acc[g][i];
                    if (a.pmax) a.pmax[(int64_t)r * W + x] = mx[g][i];
                }
            }
        }
    }
};

template <typename TIn, int BLOCK, int G, int UNR, bool NT>
__device__ __forceinline__ void fwd_tile_vec(const FwdArgs<TIn> &a, int r, int tile) {
    constexpr int T = 4 * BLOCK * G;
    const int m = (int)(((int64_t)r * a.W) & 3);
    const int ca = (4 - m) & 3;
    const int x0 = (ca ? ca - 4 : 0) + tile * T;
    if (x0 >= a.W) return;
    VecTile<TIn, BLOCK, G, NT> vt(a, r, x0);
    int n = 0;
    for (; n + UNR <= a.N; n += UNR) vt.template planes<UNR>(n);
    for (; n < a.N; ++n) vt.template planes<1>(n);
    vt.finish();
}

// Plain launches: one workgroup per (row, column tile).
template <typename TIn, int BLOCK, int J, bool NT>
__global__ __launch_bounds__(BLOCK) void k_forward_scalar(FwdArgs<TIn> a, int tiles_x) {
    const int64_t b = xcd_remap(blockIdx.x, gridDim.x);
    const int r = (int)(b / tiles_x);
    const int xt = (int)(b - (int64_t)r * tiles_x);
    fwd_tile_scalar<TIn, BLOCK, J, NT>(a, r, (int64_t)xt * (BLOCK * J));
}

template <typename TIn, int BLOCK, int G, int UNR, bool NT>
__global__ __launch_bounds__(BLOCK) void k_forward_vec(FwdArgs<TIn> a, int tiles_x) {
    const int64_t b = xcd_remap(blockIdx.x, gridDim.x);
    const int r = (int)(b / tiles_x);
    const int xt = (int)(b - (int64_t)r * tiles_x);
    fwd_tile_vec<TIn, BLOCK, G, UNR, NT>(a, r, xt);
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
    int32_t vec, pad_;
};

// Persistent launch: workgroups stride over the concatenated tile lists of
// all jobs (job-major, then row, then column tile).  Each tile runs exactly
// the code of the plain launch for that job, so outputs are bitwise equal.
template <int BLOCK, int PT, int UNR, bool NT>
__global__ __launch_bounds__(BLOCK) void k_forward_jobs(const JobDev *__restrict__ jobs,
                                                        int n_jobs, int64_t total_tiles) {
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
        const int64_t lt = t - jb.tile_begin;
        const int r = (int)(lt / jb.tiles_x);
        const int xt = (int)(lt - (int64_t)r * jb.tiles_x);
        if constexpr (PT >= 4) {
            if (jb.vec) {
                fwd_tile_vec<uint16_t, BLOCK, PT / 4, UNR, NT>(a, r, xt);
                continue;
            }
        }
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
template <int BLOCK, bool GIN, bool GOFF>
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
        const int64_t rowi = (int64_t)n * a.R + r;
        const float *grow = a.gvol + rowi * W;
        const float *srow = a.in + rowi * C;
        float *orow = nullptr;
        if constexpr (GIN) orow = a.gin + rowi * C;
        for (int64_t c = threadIdx.x; c < C; c += BLOCK) {
            const int64_t x = c + pc.k;
            const float g0 = load_px(grow, x, W);
            const float g1 = load_px(grow, x + 1, W);
            if constexpr (GIN) orow[c] = fmaf(pc.whi, g0, pc.wlo * g1);
            if constexpr (GOFF) part += (double)srow[c] * ((double)g1 - (double)g0);
        }
    }
    if constexpr (GOFF) {
        const double s = block_sum<BLOCK>(part, lds);
        if (threadIdx.x == 0) a.partial[(int64_t)n * a.G + g] = s;
    }
}

// Fixed-order sum of the G partials of each plane.
template <int UNUSED = 0>
__global__ void k_backward_finalize(const double *__restrict__ partial, int N, int G,
                                    double *__restrict__ gout) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n < N) {
        double s = 0.0;
        for (int g = 0; g < G; ++g) s += partial[(int64_t)n * G + g];
        gout[n] = s;
    }
}

}  // namespace dsk
