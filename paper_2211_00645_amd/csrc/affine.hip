// Real-space (affine) deskew: the stack resampled onto a Cartesian grid of
// the sample, the alternative the paper contrasts the remap with
// ("Physical principles", remap paragraph).  Raw image n, row x, column z
// images the point X = x p, Z = z p sin(a), Y = n s_z + z p cos(a)
// (s_z the scan step).  With the output's Z on the raw column grid, voxel
// (y, x, z) at Y = Y0 + y dy lies on raw column z between images
// floor(u) and floor(u) + 1, u = (Y - z p cos(a)) / s_z, and is their linear
// interpolation (zero outside the stack).
//
// The output is several times the remap's volume and each output row
// crosses many images, so a plain gather would fetch a cache line per pixel.
// The kernels keep the images a 64-column strip needs in an LDS ring while
// they sweep y.  The main one (k_affine_rows) sweeps four rows of a strip at
// once, so that each voxel's weights, which depend on (y, z) only, serve four
// voxels; k_affine_ring (one row, a lane per column) covers the layouts it
// does not take, and the one-shot kernel (k_affine, one lane per 4 output
// columns in output order) the geometries no ring takes (the band moving a
// whole image or more per y, or wider than the ring).
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

// Ring kernel: one wavefront per (y chunk, row x, 64 columns), sweeping its
// y chunk in the direction in which u grows.  The images the 64 columns
// need at one y form a band of about 64 |uz| + 2 consecutive images, moving
// by |uy| < 1 images per y.  The band lives in an LDS ring of 32 image rows
// (64 floats each, row n mod 32); each image row enters once, with one
// coalesced 128-byte load issued a few steps before its first use and
// written to the ring when it is consumed.  Every voxel then reads its two
// images from LDS instead of gathering them from L2.
constexpr int kAffAhead = 8;

template <typename TIn>
struct RingArgs {
    AffArgs<TIn> a;
    int64_t ychunk;       // y values per wavefront
    int32_t ztiles;       // 64-column tiles per row
};

// YQ y values per step (1, or 4 when the band moves less than half an
// image per y, i.e. at most 2 new images per step); AHEAD steps of
// look-ahead.  The ring has 32 rows plus a copy of row 0 after row 31, so
// the two images a voxel needs are always in consecutive rows.  The host
// keeps every u within +-1e9, so floors fit an int.
template <typename TIn, int YQ, int AHEAD>
__global__ __launch_bounds__(64) void k_affine_ring(RingArgs<TIn> ra) {
    constexpr int NF = YQ == 1 ? 1 : 2;        // fetches per step
    __shared__ float ring[33 * 64];
    const AffArgs<TIn> &a = ra.a;
    const int lane = (int)threadIdx.x;
    const int64_t b = blockIdx.x;
    const int64_t per_chunk = (int64_t)a.R * ra.ztiles;
    const int64_t yc = b / per_chunk;
    const int64_t rem = b - yc * per_chunk;
    const int x = (int)(rem / ra.ztiles);
    const int zb = 64 * (int)(rem - (int64_t)x * ra.ztiles);
    const int ze = zb + 63 < a.C ? zb + 63 : a.C - 1;
    const bool zok = zb + lane < a.C;
    const int zc = zok ? zb + lane : ze;       // the column this lane reads and writes
    const int64_t y_lo = yc * ra.ychunk;
    const int64_t y_hi = (y_lo + ra.ychunk < a.ny ? y_lo + ra.ychunk : a.ny);
    const int ny_c = (int)(y_hi - y_lo);
    const int steps = (ny_c + YQ - 1) / YQ;
    // y runs in the direction in which u grows; u = P(y) - z uz, where the
    // chain P(next y) = P(y) + |uy| gives the one value both the band
    // bookkeeping and the voxels use, so they always agree on which images
    // are needed
    const bool up = a.uy > 0.0;
    const int64_t y_first = up ? y_lo : y_hi - 1;
    const double ds = fabs(a.uy);
    const double uzl = __dmul_rn((double)zc, a.uz);
    const double uzb = __dmul_rn((double)zb, a.uz), uze = __dmul_rn((double)ze, a.uz);
    const double uz_min = uzb < uze ? uzb : uze, uz_max = uzb < uze ? uze : uzb;
    auto fl = [](double v) { return (int)floor(v); };
    // P of the first y of each of the next AHEAD steps, and of step AHEAD
    double Pq[AHEAD];
    Pq[0] = __dadd_rn(a.u0, __dmul_rn((double)y_first, a.uy));
#pragma unroll
    for (int k = 1; k < AHEAD; ++k) {
        double p = Pq[k - 1];
#pragma unroll
        for (int i = 0; i < YQ; ++i) p = __dadd_rn(p, ds);
        Pq[k] = p;
    }
    double Pa = Pq[AHEAD - 1];
#pragma unroll
    for (int i = 0; i < YQ; ++i) Pa = __dadd_rn(Pa, ds);
    // last P of a step whose first P is p
    auto last_p = [&](double p) {
#pragma unroll
        for (int i = 1; i < YQ; ++i) p = __dadd_rn(p, ds);
        return p;
    };
    // images outside the stack read image 0 or N-1 and enter the ring
    // scaled by 0, so every fetch is one unconditional coalesced load and
    // the ring holds zeros for them
    const TIn *rowx = a.in + (int64_t)x * a.C;    // wave-uniform base
    const int64_t plane = (int64_t)a.R * a.C;
    auto load = [&](int n) {
        const TIn *base = rowx + (int64_t)(n < 0 ? 0 : (n >= a.N ? a.N - 1 : n)) * plane;
        return base[zc];
    };
    auto scale = [&](int n) { return (n >= 0 && n < a.N) ? 1.0f : 0.0f; };
    auto put = [&](int m, float v) {
        const int r = m & 31;
        ring[r * 64 + lane] = v;
        if (r == 0) ring[32 * 64 + lane] = v;
    };
    // fill: the band of the first AHEAD steps, 8 loads at a time
    int have;
    {
        const int lo0 = fl(__dsub_rn(Pq[0], uz_max));
        const int last = steps - 1 < AHEAD - 1 ? steps - 1 : AHEAD - 1;
        const int top = fl(__dsub_rn(last_p(Pq[last]), uz_min)) + 1;
        for (int n = lo0; n <= top; n += 8) {
            TIn t[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) t[i] = load(n + i <= top ? n + i : top);
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int m = n + i <= top ? n + i : top;
                put(m, (float)t[i] * scale(m));
            }
        }
        have = top;
    }
    // per step exactly NF fetches and YQ stores: the images the step AHEAD
    // later first needs, or again the newest image (its ring row is
    // rewritten with the same values)
    TIn q[AHEAD][NF];
    int qn[AHEAD][NF];
#pragma unroll
    for (int k = 0; k < AHEAD; ++k)
#pragma unroll
        for (int i = 0; i < NF; ++i) {
            q[k][i] = 0;
            qn[k][i] = have;
        }
    const int64_t ostep = (up ? 1 : -1) * (int64_t)a.R * a.C;
    float *orow = a.vol + (y_first * a.R + x) * (int64_t)a.C;   // wave-uniform

    auto step = [&](int k, int j, bool tail) {
        // the images fetched AHEAD steps ago enter the ring
        if (j >= AHEAD) {
#pragma unroll
            for (int i = 0; i < NF; ++i) put(qn[k][i], (float)q[k][i] * scale(qn[k][i]));
        }
        const double p0 = Pq[k];                // P of this step's first y
        int m = have;
        if (j + AHEAD < steps) {
            const int h = fl(__dsub_rn(last_p(Pa), uz_min)) + 1;  // leading edge
            m = h > have ? h : have;
        }
        Pq[k] = Pa;
#pragma unroll
        for (int i = 0; i < YQ; ++i) Pa = __dadd_rn(Pa, ds);
        // at most NF new images: have + 1 .. m
#pragma unroll
        for (int i = 0; i < NF; ++i) {
            const int mi = have + 1 + i <= m ? have + 1 + i : m;
            q[k][i] = load(mi);
            qn[k][i] = mi;
        }
        have = m;
        {
            double p = p0;
#pragma unroll
            for (int i = 0; i < YQ; ++i) {
                if (i) p = __dadd_rn(p, ds);
                const double u = __dsub_rn(p, uzl);
                const double fi = floor(u);
                const int r = (int)fi & 31;
                const double f = __dsub_rn(u, fi);
                // both weights rounded once from FP64 (1 - wlo in FP32 would
                // lose the relative precision of a small 1 - f)
                const float wlo = (float)f, whi = (float)__dsub_rn(1.0, f);
                const float lo = ring[r * 64 + lane];
                const float hi = ring[r * 64 + 64 + lane];
                // lanes past the last column repeat the last column's value
                // to its address: one unconditional store per y
                if (!tail || j * YQ + i < ny_c)
                    store_f32<true>(orow + zc, fmaf(wlo, hi, whi * lo));
                orow += ostep;
            }
        }
    };
    const int full = (ny_c / YQ) / AHEAD * AHEAD;   // steps with all YQ y values, whole groups
    for (int j0 = 0; j0 < full; j0 += AHEAD) {
#pragma unroll
        for (int k = 0; k < AHEAD; ++k) step(k, j0 + k, false);
    }
#pragma unroll
    for (int k = 0; k < AHEAD; ++k)
        if (full + k < steps) step(k, full + k, true);
}

// Row kernel: persistent wavefronts, each taking work items (y range, strip
// of kAffRows rows x 64 columns) in turn, consecutive wavefronts on
// neighbouring strips of one y range, so that the wavefronts write
// neighbouring output rows of the same planes.  Each sweeps its y range in
// the direction in which u grows, 4 y values per step:
//  * the weights of a voxel depend on (y, z) only: lane group y (16 lanes,
//    4 adjacent columns each) computes them once, in FP64 as the ring
//    kernel does, and applies them to all kAffRows rows;
//  * the rows share one LDS ring of 32 image rows with the rows interleaved
//    (ring[((n mod 32) * 64 + column) * kAffRows + row]), so one 16-byte LDS
//    read returns an image's value in all rows and one 16-byte write enters
//    it;
//  * the at most 2 images a step needs first arrive in one 4-byte load per
//    row: the wavefront's halves read the two images, 2 columns per lane,
//    AHEAD steps before the step that needs them;
//  * the y chain P(y + 1) = P(y) + |uy| restarts from the exact
//    u0 + y uy every kAffRestart values of the sweep (as the ring kernel's
//    512-y work items do), so its rounding never accumulates over more than
//    that many adds.
// Requires (host): C a multiple of 4, the stack 4-byte and the volume 16-byte
// aligned, at most 2 new images per step and the band within the ring
// (the YQ = 4 ring conditions).  Rows past the last repeat the last row
// (identical values to identical addresses).
constexpr int kAffRows = 4;
constexpr int kAffRestart = 512;
constexpr int kAffRowsAhead = 4;
// Workgroups per compute unit: the 32 KB ring allows 5; 4 (one wavefront
// per SIMD) gave each of them the same number of work items on the
// 512x512x2048 stack (4096 strips over 1024 wavefronts).  Measured there:
// 3.37 ms against 4.40 ms for the lane-per-column ring kernel.
constexpr int kAffRowsPerCU = 4;

struct RowsArgs {
    AffArgs<uint16_t> a;
    int64_t ylen;      // y values per work item, a multiple of kAffRestart
    int64_t strips;    // ceil(R / kAffRows) * ztiles
    int64_t items;     // strips * ceil(ny / ylen)
    int32_t ztiles;
};

__device__ __forceinline__ void affine_rows_item(const AffArgs<uint16_t> &a, float *ring, int x0,
                                                 int zb, int64_t y_lo, int64_t y_hi) {
    constexpr int AHEAD = kAffRowsAhead;
    constexpr int NR = kAffRows;
    const int lane = (int)threadIdx.x;
    const int ze = zb + 63 < a.C ? zb + 63 : a.C - 1;
    // this lane's y within a step and its 4 columns (lanes past the last
    // group repeat it)
    const int yq = lane >> 4;
    const int ngrp = (ze - zb + 1) / 4;
    const int zq = zb + 4 * ((lane & 15) < ngrp ? (lane & 15) : ngrp - 1);
    const int ny_c = (int)(y_hi - y_lo);
    const int steps = (ny_c + 3) / 4;
    const bool up = a.uy > 0.0;
    const int64_t y_first = up ? y_lo : y_hi - 1;
    const double ds = fabs(a.uy);
    double uzq[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) uzq[i] = __dmul_rn((double)(zq + i), a.uz);
    const double uzb = __dmul_rn((double)zb, a.uz), uze = __dmul_rn((double)ze, a.uz);
    const double uz_min = uzb < uze ? uzb : uze, uz_max = uzb < uze ? uze : uzb;
    auto fl = [](double v) { return (int)floor(v); };
    const int64_t plane = (int64_t)a.R * a.C;
    // loads: half h of the wavefront reads the step's image h, columns
    // pcol, pcol + 1 (the last pair repeated past the strip's end)
    const int pl = 2 * (lane & 31);
    const bool second = lane >= 32;
    const int pcol = zb + pl <= a.C - 2 ? zb + pl : a.C - 2;
    const uint16_t *rowp[NR];
    float *orow[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int x = x0 + r < a.R ? x0 + r : a.R - 1;
        rowp[r] = a.in + (int64_t)x * a.C + pcol;
        orow[r] = a.vol + (y_first * a.R + x) * (int64_t)a.C;
    }
    // images outside the stack read image 0 or N-1 and enter the ring
    // scaled by 0
    auto load2 = [&](int r, int m0, int m1) {
        const int n = second ? m1 : m0;
        const int64_t nc = n < 0 ? 0 : (n >= a.N ? a.N - 1 : n);
        return *(const uint32_t *)(rowp[r] + nc * plane);
    };
    auto put2 = [&](int m0, int m1, const uint32_t *v) {
        const int n = second ? m1 : m0;
        const float sc = (n >= 0 && n < a.N) ? 1.0f : 0.0f;
        float *p = ring + ((n & 31) * 64 + pl) * NR;
        f32x4 e, o;
        e.x = (float)(v[0] & 0xffffu) * sc;
        e.y = (float)(v[1] & 0xffffu) * sc;
        e.z = (float)(v[2] & 0xffffu) * sc;
        e.w = (float)(v[3] & 0xffffu) * sc;
        o.x = (float)(v[0] >> 16) * sc;
        o.y = (float)(v[1] >> 16) * sc;
        o.z = (float)(v[2] >> 16) * sc;
        o.w = (float)(v[3] >> 16) * sc;
        *(f32x4 *)p = e;
        *(f32x4 *)(p + NR) = o;
    };
    // the chain: the step prepared next starts at sweep index 4 * prep; each
    // step's 4 chain values are computed once, when it is prepared AHEAD
    // steps ahead, and each lane keeps the one of its y
    double Pc = 0.0, cfirst = 0.0;
    double Psel[AHEAD];
    int top = 0;           // last image the prepared step needs
    auto prepare = [&](int k, int prep) {
        const int i0 = 4 * prep;
        const int64_t y = up ? y_first + i0 : y_first - i0;
        const double c0 = (i0 % kAffRestart == 0) ? __dadd_rn(a.u0, __dmul_rn((double)y, a.uy)) : Pc;
        const double c1 = __dadd_rn(c0, ds), c2 = __dadd_rn(c1, ds), c3 = __dadd_rn(c2, ds);
        // this lane's value, picked without a branch (integer selects on the
        // two halves)
        int plo = __double2loint(c0), phi = __double2hiint(c0);
        plo = yq == 1 ? __double2loint(c1) : plo;
        phi = yq == 1 ? __double2hiint(c1) : phi;
        plo = yq == 2 ? __double2loint(c2) : plo;
        phi = yq == 2 ? __double2hiint(c2) : phi;
        plo = yq == 3 ? __double2loint(c3) : plo;
        phi = yq == 3 ? __double2hiint(c3) : phi;
        Psel[k] = __hiloint2double(phi, plo);
        cfirst = c0;
        top = fl(__dsub_rn(c3, uz_min)) + 1;
        Pc = __dadd_rn(c3, ds);
    };
    prepare(0, 0);
    const int lo0 = fl(__dsub_rn(cfirst, uz_max));   // the first step's lowest image
#pragma unroll
    for (int k = 1; k < AHEAD; ++k)
        if (k < steps) prepare(k, k);
    // fill: the band of the first AHEAD steps, 8 images per round
    for (int n = lo0; n <= top; n += 8) {
        uint32_t t[4][NR];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int m0 = n + 2 * i <= top ? n + 2 * i : top;
            const int m1 = n + 2 * i + 1 <= top ? n + 2 * i + 1 : top;
#pragma unroll
            for (int r = 0; r < NR; ++r) t[i][r] = load2(r, m0, m1);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int m0 = n + 2 * i <= top ? n + 2 * i : top;
            const int m1 = n + 2 * i + 1 <= top ? n + 2 * i + 1 : top;
            put2(m0, m1, t[i]);
        }
    }
    int have = top;
    uint32_t q[AHEAD][NR];
    int qn[AHEAD][2];
#pragma unroll
    for (int k = 0; k < AHEAD; ++k) {
        qn[k][0] = qn[k][1] = have;
#pragma unroll
        for (int r = 0; r < NR; ++r) q[k][r] = 0;
    }
    const int64_t ostep = (up ? 1 : -1) * plane;
#pragma unroll
    for (int r = 0; r < NR; ++r) orow[r] += (int64_t)yq * ostep + zq;

    auto step = [&](int k, int j, bool tail) {
        // the images fetched AHEAD steps ago enter the ring
        if (j >= AHEAD) put2(qn[k][0], qn[k][1], q[k]);
        const double p = Psel[k];
        int m = have;
        if (j + AHEAD < steps) {
            prepare(k, j + AHEAD);
            m = top > have ? top : have;
        }
        // at most 2 new images: have + 1 .. m (or again the newest)
        const int mi0 = have + 1 <= m ? have + 1 : m, mi1 = have + 2 <= m ? have + 2 : m;
#pragma unroll
        for (int r = 0; r < NR; ++r) q[k][r] = load2(r, mi0, mi1);
        qn[k][0] = mi0;
        qn[k][1] = mi1;
        have = m;
        float wl[4], wh[4];
        f32x4 lo[4], hi[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const double u = __dsub_rn(p, uzq[i]);
            const double fi = floor(u);
            const int n0 = (int)fi;
            const int c = zq - zb + i;
            const double f = __dsub_rn(u, fi);
            // both weights rounded once from FP64
            wl[i] = (float)f;
            wh[i] = (float)__dsub_rn(1.0, f);
            lo[i] = *(const f32x4 *)(ring + ((n0 & 31) * 64 + c) * NR);
            hi[i] = *(const f32x4 *)(ring + (((n0 + 1) & 31) * 64 + c) * NR);
        }
        f32x4 v[NR];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            v[0][i] = fmaf(wl[i], hi[i].x, wh[i] * lo[i].x);
            v[1][i] = fmaf(wl[i], hi[i].y, wh[i] * lo[i].y);
            v[2][i] = fmaf(wl[i], hi[i].z, wh[i] * lo[i].z);
            v[3][i] = fmaf(wl[i], hi[i].w, wh[i] * lo[i].w);
        }
        if (!tail || j * 4 + yq < ny_c) {
#pragma unroll
            for (int r = 0; r < NR; ++r) store_f32x4<true>(orow[r], v[r]);
        }
#pragma unroll
        for (int r = 0; r < NR; ++r) orow[r] += 4 * ostep;
    };
    const int full = (ny_c / 4) / AHEAD * AHEAD;   // steps with all 4 y values, whole groups
    for (int j0 = 0; j0 < full; j0 += AHEAD) {
#pragma unroll
        for (int k = 0; k < AHEAD; ++k) step(k, j0 + k, false);
    }
#pragma unroll
    for (int k = 0; k < AHEAD; ++k)
        if (full + k < steps) step(k, full + k, true);
}

__global__ __launch_bounds__(64) void k_affine_rows(RowsArgs ra) {
    __shared__ __align__(16) float ring[kAffRows * 32 * 64];
    for (int64_t it = blockIdx.x; it < ra.items; it += gridDim.x) {
        const int64_t c = it / ra.strips, s = it - c * ra.strips;
        const int xi = (int)(s / ra.ztiles);
        const int zb = 64 * (int)(s - (int64_t)xi * ra.ztiles);
        const int64_t y_lo = c * ra.ylen;
        const int64_t y_hi = y_lo + ra.ylen < ra.a.ny ? y_lo + ra.ylen : ra.a.ny;
        affine_rows_item(ra.a, ring, xi * kAffRows, zb, y_lo, y_hi);
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
    // ring kernels when the band moves less than one image per y and fits
    // 32 ring rows; otherwise the one-shot kernel
    // y values per wavefront: long sweeps amortise the ring fill (measured
    // on 512x512x2048: 32 -> 5.08 ms, 128 -> 4.56 ms, 512 -> 4.43 ms)
    const int64_t ychunk = 512;
    const int32_t ztiles = (d.cols + 63) / 64;
    const int64_t chunks = (ny + ychunk - 1) / ychunk;
    const int64_t blocks = ychunk > 0 ? chunks * d.rows * ztiles : kMaxI32;
    const double band4 = 63.0 * std::fabs(a.uz) + (4 * 4 + 4) * std::fabs(a.uy) + 4.0;
    const double band1 = 63.0 * std::fabs(a.uz) + (kAffAhead + 1) * std::fabs(a.uy) + 4.0;
    // the ring kernels take floors of u as ints: every u of the grid
    // (u0 + y uy - z uz over the whole output) must stay within +-1e9
    const double ue[4] = {a.u0, a.u0 + (double)(ny - 1) * a.uy, a.u0 - (double)(d.cols - 1) * a.uz,
                          a.u0 + (double)(ny - 1) * a.uy - (double)(d.cols - 1) * a.uz};
    bool u_ok = true;
    for (double v : ue) u_ok = u_ok && std::fabs(v) < 1.0e9;
    if (u_ok && blocks < kMaxI32 && std::fabs(a.uy) <= 0.499 && band4 <= 32.0) {
        if (d.cols % 4 == 0 && ((uintptr_t)vol & 15) == 0 && ((uintptr_t)in & 3) == 0 &&
            ny < (int64_t(1) << 30)) {
            // row kernel: persistent, kAffRows-row strips; when the strips
            // do not fill the resident wavefronts, the y range is split in
            // multiples of kAffRestart
            const int64_t strips = ((int64_t)d.rows + kAffRows - 1) / kAffRows * ztiles;
            const int64_t resident = (int64_t)kAffRowsPerCU * device_cus();
            const int64_t ychunks = (ny + kAffRestart - 1) / kAffRestart;
            int64_t split = strips >= resident ? 1 : (resident + strips - 1) / strips;
            split = split < ychunks ? split : ychunks;
            const int64_t ylen = (ychunks + split - 1) / split * kAffRestart;
            const int64_t items = strips * ((ny + ylen - 1) / ylen);
            const int64_t grid = items < resident ? items : resident;
            const RowsArgs ra{a, ylen, strips, items, ztiles};
            hipLaunchKernelGGL(k_affine_rows, dim3((unsigned)grid), dim3(64), 0, stream, ra);
            return hip_status(hipGetLastError());
        }
        const RingArgs<uint16_t> ra{a, ychunk, ztiles};
        hipLaunchKernelGGL((k_affine_ring<uint16_t, 4, 4>), dim3((unsigned)blocks), dim3(64), 0,
                           stream, ra);
        return hip_status(hipGetLastError());
    }
    if (u_ok && blocks < kMaxI32 && std::fabs(a.uy) <= 0.999 && band1 <= 32.0) {
        const RingArgs<uint16_t> ra{a, ychunk, ztiles};
        hipLaunchKernelGGL((k_affine_ring<uint16_t, 1, kAffAhead>), dim3((unsigned)blocks),
                           dim3(64), 0, stream, ra);
        return hip_status(hipGetLastError());
    }
    const bool vec = d.cols % 4 == 0 && ((uintptr_t)vol & 15) == 0;
    if (vec)
        hipLaunchKernelGGL((k_affine<uint16_t, true>), grid, dim3(kAffBlock), 0, stream, a);
    else
        hipLaunchKernelGGL((k_affine<uint16_t, false>), grid, dim3(kAffBlock), 0, stream, a);
    return hip_status(hipGetLastError());
}
