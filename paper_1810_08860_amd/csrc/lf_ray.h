// Per-ray arithmetic of the renderer, shared by the HIP kernels and usable
// from host code (LF_HD = __host__ __device__): storage-format loads, the exact
// disk test, the inverse-depth mesh walk and bilinear sampling.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include "lf_internal.h"

#define LF_HD __host__ __device__ __forceinline__

namespace lf {

// Hardware reciprocal and square root (about 1 ulp) on the device; the host
// build (CPU tests) uses the exact operations.
LF_HD float fast_rcp(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}
// Product of two operands below 2^24 (a full-rate multiply on the device).
LF_HD uint32_t mul24(uint32_t a, uint32_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __umul24(a, b);
#else
    return a * b;
#endif
}
LF_HD float fast_sqrt(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_sqrtf(x);
#else
    return sqrtf(x);
#endif
}

// ---------------------------------------------------------------------------------------------
// storage formats

struct Rgb {
    float r, g, b;
};

// Element idx of an array that starts at base, with the byte offset formed in
// 32 bits: every array indexed this way is one view's share (well under
// 4 GiB), so a wave-uniform base plus a 32-bit per-lane offset addresses it.
// On the device the base is a global-memory pointer (address space 1): the
// per-view bases come from the view records in memory, and a generic pointer
// would make every access a flat load.
template <typename T>
LF_HD T at(const void *__restrict__ base, uint32_t idx) {
#if defined(__HIP_DEVICE_COMPILE__)
    typedef const __attribute__((address_space(1))) char gchar;
    typedef const __attribute__((address_space(1))) T gT;
    return *(gT *)((gchar *)base + idx * (uint32_t)sizeof(T));
#else
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + idx * (uint32_t)sizeof(T));
#endif
}

// Texel idx (row-major) of one view's image.
template <int IMG>
LF_HD Rgb texel(const void *__restrict__ img, uint32_t idx);

template <>
LF_HD Rgb texel<0>(const void *__restrict__ img, uint32_t idx) {  // RGBA8, 0..255
    const uint32_t p = at<uint32_t>(img, idx);
    return {(float)(p & 255u), (float)((p >> 8) & 255u), (float)((p >> 16) & 255u)};
}
template <>
LF_HD Rgb texel<1>(const void *__restrict__ img, uint32_t idx) {  // RGBA16F
    uint2 p = at<uint2>(img, idx);
    __half2 rg = *reinterpret_cast<__half2 *>(&p.x);
    __half2 ba = *reinterpret_cast<__half2 *>(&p.y);
    return {__low2float(rg), __high2float(rg), __low2float(ba)};
}
template <>
LF_HD Rgb texel<2>(const void *__restrict__ img, uint32_t idx) {  // RGBA32F
    float4 p = at<float4>(img, idx);
    return {p.x, p.y, p.z};
}

// Address of texel idx of one view's image (RGBA8, RGBA16F or RGBA32F).
template <int IMG>
LF_HD const void *texel_row(const void *__restrict__ img, uint32_t idx) {
    constexpr uint32_t bytes = IMG == 0 ? 4u : IMG == 1 ? 8u : 16u;
#if defined(__HIP_DEVICE_COMPILE__)
    typedef const __attribute__((address_space(1))) char gchar;
    return (const void *)((gchar *)img + idx * bytes);
#else
    return reinterpret_cast<const char *>(img) + idx * bytes;
#endif
}

// scale from stored texel units to [0,1]
template <int IMG>
LF_HD float texel_scale() { return (IMG == 0 || IMG >= 3) ? (1.0f / 255.0f) : 1.0f; }

// Corner inverse depths of one mesh cell: (w00, w10, w01, w11) with j to the
// right and k downwards.
// idx is the cell's index within one view (k * (M - 1) + j).
template <int GEO>
LF_HD float4 load_cell(const void *__restrict__ cells, uint32_t idx);

template <>
LF_HD float4 load_cell<0>(const void *__restrict__ cells, uint32_t idx) {
    return at<float4>(cells, idx);
}
template <>
LF_HD float4 load_cell<1>(const void *__restrict__ cells, uint32_t idx) {
    uint2 p = at<uint2>(cells, idx);
    __half2 a = *reinterpret_cast<__half2 *>(&p.x);
    __half2 b = *reinterpret_cast<__half2 *>(&p.y);
    return make_float4(__low2float(a), __high2float(a), __low2float(b), __high2float(b));
}
// Per-view linear 16-bit codes: w = base + code * scale, with (base, scale)
// in the 8 bytes that precede the view's cells (a load that does not depend
// on the cell, so the compiler keeps it out of the walk's loop).
template <>
LF_HD float4 load_cell<2>(const void *__restrict__ cells, uint32_t idx) {
#if defined(__HIP_DEVICE_COMPILE__)
    typedef const __attribute__((address_space(1))) char gchar;
    typedef const __attribute__((address_space(1))) float2 gF2;
    const float2 q = *(gF2 *)((gchar *)cells - sizeof(float2));
#else
    const float2 q = *(reinterpret_cast<const float2 *>(cells) - 1);
#endif
    const uint2 p = at<uint2>(cells, idx);
    return make_float4(fmaf((float)(p.x & 0xffffu), q.y, q.x), fmaf((float)(p.x >> 16), q.y, q.x),
                       fmaf((float)(p.y & 0xffffu), q.y, q.x), fmaf((float)(p.y >> 16), q.y, q.x));
}

// Bytes per mesh cell and bytes of the header before each view's cells.
template <int GEO>
LF_HD constexpr int geo_cell_bytes() { return GEO == 0 ? 16 : 8; }
template <int GEO>
LF_HD constexpr int geo_head_bytes() { return GEO == 2 ? 8 : 0; }
// View v's cells in a light field of views with `per` cells each.
template <int GEO>
LF_HD const void *geo_view(const void *cells, int64_t v, int64_t per) {
    return static_cast<const char *>(cells) + v * (geo_head_bytes<GEO>() + per * geo_cell_bytes<GEO>()) +
           geo_head_bytes<GEO>();
}

// ---------------------------------------------------------------------------------------------
// per-ray pieces

struct RayView {
    float Vx, Vy, Dx, Dy, rho;
};

// The ray's vanishing point V and disk-plane coordinates D in view v's frame;
// returns e'z (> 0 for a disk facing the ray).
LF_HD float disk_coords(const EyeView &v, float X, float Y, RayView &rv) {
    const float ez = fmaf(v.m[6], X, fmaf(v.m[7], Y, v.m[8]));
    const float iz = fast_rcp(ez);
    rv.Vx = fmaf(v.m[0], X, fmaf(v.m[1], Y, v.m[2])) * iz;
    rv.Vy = fmaf(v.m[3], X, fmaf(v.m[4], Y, v.m[5])) * iz;
    rv.Dx = fmaf(-v.o[2], rv.Vx, v.o[0]);
    rv.Dy = fmaf(-v.o[2], rv.Vy, v.o[1]);
    return ez;
}

// Exact disk test of one ray against one view (Sec. 4.1: linear falloff, disk
// in the view's tangent plane). False for a back-facing disk or rho <= 0.
// Evaluated without early exits (a back-facing view gives garbage that the
// final test discards, NaN included).
LF_HD bool disk_test(const EyeView &v, float X, float Y, float invR, RayView &rv) {
    const float ez = disk_coords(v, X, Y, rv);
    rv.rho = fmaf(-fast_sqrt(fmaf(rv.Dx, rv.Dx, rv.Dy * rv.Dy)), invR, 1.0f);
    return ez > 0.0f && rv.rho > 0.0f;
}

// Asymmetric oval disk (Sec. 4.4): the linear falloff runs in the radius
// normalised by the extents of D's quadrant; ie = (1/e+u, 1/e-u, 1/e+v,
// 1/e-v) times s.
LF_HD bool disk_test_oval(const EyeView &v, float X, float Y, float4 ie, float s, RayView &rv) {
    const float ez = disk_coords(v, X, Y, rv);
    const float su = rv.Dx * (rv.Dx >= 0.0f ? ie.x : ie.y) * s, sv = rv.Dy * (rv.Dy >= 0.0f ? ie.z : ie.w) * s;
    rv.rho = 1.0f - fast_sqrt(fmaf(su, su, sv * sv));
    return ez > 0.0f && rv.rho > 0.0f;
}

LF_HD float sat01(float x) { return fminf(fmaxf(x, 0.0f), 1.0f); }

// Tolerances of the per-cell root test: a root counts if it lies on the
// cell's piece of the line up to kTolW x (largest w of the walk) and on its
// triangle's side of the diagonal up to kTolD cells. Both sit far below the
// rounding of a sample position yet far above the rounding of the root, so a
// crossing on an edge shared by two cells or triangles is found from either
// side (the mesh is continuous, so both sides give the same point).
constexpr float kTolW = 4e-6f;
constexpr float kTolD = 1e-5f;

// x clamped into [lo, hi] (x not NaN, lo <= hi)
LF_HD float clamp_range(float x, float lo, float hi) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_fmed3f(x, lo, hi);
#else
    return fminf(fmaxf(x, lo), hi);
#endif
}

// Largest root of (mesh inverse depth - w) on one cell's piece of the line,
// the part with w in [lo, hi]. In the cell's local coordinates the line is
// (fx, fy) = (px + bx w, py + by w), with (px, py) its point at w = 0 and
// dbb = bx - by. Triangle A (fx >= fy) interpolates (w00, w10, w11) and
// triangle B (fx < fy) interpolates (w00, w11, w01); on each the mesh is
// linear in w along the line, so the root is num / den in closed form. The
// root depends on the cell and the line only, not on where a walk entered
// the cell, so every walk that reaches the cell computes the same value.
LF_HD bool cell_root(const float4 &c, float px, float py, float bx, float by, float dbb, float lo, float hi,
                     float &w) {
    const float d0 = px - py;
    const float a1 = c.y - c.x, a2 = c.w - c.y;
    const float wA = fmaf(py, a2, fmaf(px, a1, c.x)) * fast_rcp(fmaf(-by, a2, fmaf(-bx, a1, 1.0f)));
    const float b1 = c.w - c.z, b2 = c.z - c.x;
    const float wB = fmaf(py, b2, fmaf(px, b1, c.x)) * fast_rcp(fmaf(-by, b2, fmaf(-bx, b1, 1.0f)));
    const bool okA = wA <= hi && wA >= lo && fmaf(dbb, wA, d0) >= -kTolD;
    const bool okB = wB <= hi && wB >= lo && fmaf(dbb, wB, d0) <= kTolD;
    // the larger accepted root (accepted roots are never NaN)
    const float tA = okA ? wA : -INFINITY;
    w = okB && wB > tA ? wB : tA;
    return okA || okB;
}

// Walk the cells of the box [j0, j1] x [k0, k1] (at most max_steps of them)
// along the line g = (ax + w bx, ay + w by) from w = ws down to w = we
// (ws >= we), starting in the cell that holds the line at ws. True with w_hit
// at the first (largest-w) root. wxe / wye hold the w at which the line
// leaves the current cell through its x / y edge; a step moves them by
// -|1/bx| / -|1/by| (the slopes are nonzero: grid_line). A root is accepted
// within tol of the cell's piece of the line.
template <int GEO>
LF_HD bool walk_cells(const void *__restrict__ cells, int Mc, float ax, float bx, float ibx, float ay, float by,
                      float iby, float tol, int j0, int j1, int k0, int k1, float ws, float we, int max_steps,
                      float &w_hit, int &n_cells) {
    const int sx = bx > 0.0f ? -1 : 1, sy = by > 0.0f ? -1 : 1;  // cell steps as w decreases
    const float dwx = -fabsf(ibx), dwy = -fabsf(iby);
    const float dbb = bx - by;
    float w0 = ws;
    // the first cell, clamped into the box as a float (exact: whole numbers)
    const float jf = clamp_range(floorf(fmaf(w0, bx, ax)), (float)j0, (float)j1);
    const float kf = clamp_range(floorf(fmaf(w0, by, ay)), (float)k0, (float)k1);
    int j = (int)jf, k = (int)kf;
    // exit edge in local coordinates: 0 when the coordinate falls as w does, else 1
    float wxe = ((bx > 0.0f ? 0.0f : 1.0f) - (ax - jf)) * ibx;
    float wye = ((by > 0.0f ? 0.0f : 1.0f) - (ay - kf)) * iby;
    bool found = false, more = true;
    for (int it = 0; it < max_steps && more; ++it) {
        const bool xs = wxe >= wye, ys = wye >= wxe;  // exit edge(s): both at a corner
        const float wn = xs ? wxe : wye;
        const bool last = !(wn > we);
        const float w1 = last ? we : (wn < w0 ? wn : w0);
        const float4 c = load_cell<GEO>(cells, mul24(k, Mc) + j);
        ++n_cells;
        found = cell_root(c, ax - (float)j, ay - (float)k, bx, by, dbb, w1 - tol, w0 + tol, w_hit);
#if defined(__HIP_DEVICE_COMPILE__)
        // the root is chosen inside the step: left to itself the compiler
        // defers the choice past the loop and keeps per-step lane masks
        // for it in scalar registers instead (more instructions per step)
        asm volatile("" : "+v"(w_hit));
#endif
        j += xs ? sx : 0;
        wxe += xs ? dwx : 0.0f;
        k += ys ? sy : 0;
        wye += ys ? dwy : 0.0f;
        // callers pass non-empty boxes (j0 <= j1, k0 <= k1): one unsigned compare per axis
        more = !found && !last && (unsigned)(j - j0) <= (unsigned)(j1 - j0) && (unsigned)(k - k0) <= (unsigned)(k1 - k0);
        w0 = w1;
    }
    return found;
}

// FP16 bit pattern of the smallest half-precision value >= x, for x > 0
// (+inf above the FP16 range). Positive FP16 values order like their bit
// patterns, so a maximum of such bounds is an integer maximum.
LF_HD uint16_t half_up_bits(float x) {
    const __half h = __float2half_rn(x);
    uint16_t b;
    memcpy(&b, &h, 2);
    return (uint16_t)(__half2float(h) < x ? b + 1 : b);
}
LF_HD float half_bits_to_float(uint32_t b) {
    const uint16_t q = (uint16_t)b;
    __half h;
    memcpy(&h, &q, 2);
    return __half2float(h);
}

// The four corner rays of the image-plane rectangle [X0, X1] x [Y1, Y0] in
// view v's frame (corners (X0, Y0), (X1, Y0), (X1, Y1), (X0, Y1)): for each,
// the vanishing point V and the disk-plane coordinates D, and npos = how many
// of them cross the disk plane from behind (e'z > 0). Shared by the culling's
// disk test and the cell box of a tile.
struct TileCorners {
    float vx[4], vy[4], dx[4], dy[4];
    int npos;
};
LF_HD TileCorners tile_corners(const EyeView &v, float X0, float X1, float Y0, float Y1) {
    const float cx[4] = {X0, X1, X1, X0}, cy[4] = {Y0, Y0, Y1, Y1};
    TileCorners C;
    C.npos = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float ez = fmaf(v.m[6], cx[q], fmaf(v.m[7], cy[q], v.m[8]));
        C.npos += ez > 0.0f;
        const float iz = fast_rcp(ez);
        C.vx[q] = fmaf(v.m[0], cx[q], fmaf(v.m[1], cy[q], v.m[2])) * iz;
        C.vy[q] = fmaf(v.m[3], cx[q], fmaf(v.m[4], cy[q], v.m[5])) * iz;
        C.dx[q] = fmaf(-v.o[2], C.vx[q], v.o[0]);
        C.dy[q] = fmaf(-v.o[2], C.vy[q], v.o[1]);
    }
    return C;
}

// Mesh cells of view v that a ray through the rectangle of corners C can
// reach over w in [v.wmin, v.wmax]: the box [j0, j1] x [k0, k1] (clamped to
// the grid). For a fixed w the points V + w D of the rectangle's rays form
// the central projection of the rectangle followed by an affine map, a convex
// quad spanned by its corner rays, and each ray's points are affine in w, so
// every reachable point lies in the convex hull of the corner rays' points at
// the two ends of the range. The box is widened by a quarter cell against
// FP32 rounding. False (no box) when a corner ray does not cross the disk
// plane from behind (the projection is unbounded); true with an empty box
// (j0 > j1) when the hull misses the mesh domain.
LF_HD bool tile_cell_box(const EyeView &v, const TileCorners &C, int M, float sM, float cM, int &j0, int &j1,
                         int &k0, int &k1) {
    float gx0 = INFINITY, gx1 = -INFINITY, gy0 = INFINITY, gy1 = -INFINITY;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const float w = e ? v.wmax : v.wmin;
            const float gx = fmaf(fmaf(w, C.dx[q], C.vx[q]), sM, cM), gy = fmaf(-fmaf(w, C.dy[q], C.vy[q]), sM, cM);
            gx0 = fminf(gx0, gx);
            gx1 = fmaxf(gx1, gx);
            gy0 = fminf(gy0, gy);
            gy1 = fmaxf(gy1, gy);
        }
    }
    if (C.npos < 4 || !(gx0 <= gx1 && gy0 <= gy1)) return false;  // NaN included
    gx0 -= 0.25f;
    gx1 += 0.25f;
    gy0 -= 0.25f;
    gy1 += 0.25f;
    const float lim = (float)(M - 1);
    if (gx1 < 0.0f || gx0 > lim || gy1 < 0.0f || gy0 > lim) {
        j0 = k0 = 1;
        j1 = k1 = 0;
        return true;
    }
    // cells 0 .. M-2; the domain edge g = M-1 belongs to the last cell
    const float top = (float)(M - 2);
    j0 = (int)floorf(fminf(fmaxf(gx0, 0.0f), top));
    j1 = (int)floorf(fminf(fmaxf(gx1, 0.0f), top));
    k0 = (int)floorf(fminf(fmaxf(gy0, 0.0f), top));
    k1 = (int)floorf(fminf(fmaxf(gy1, 0.0f), top));
    return true;
}
LF_HD bool tile_cell_box(const EyeView &v, float X0, float X1, float Y0, float Y1, int M, float sM, float cM,
                         int &j0, int &j1, int &k0, int &k1) {
    return tile_cell_box(v, tile_corners(v, X0, X1, Y0, Y1), M, sM, cM, j0, j1, k0, k1);
}

// Windows of the per-cell window table (the bound over kWin x kWin cells
// from each cell) that cover a cell box b = (j0, j1, k0, k1): nx x ny windows
// starting every kWin cells from (j0, k0), the last of each row and column
// moved back to end on the box's edge (a box narrower than kWin takes one
// window from its corner, which reaches past the box: still a bound). False
// when nothing is to be read: then mx is the bound already, +inf without a
// box (j0 < 0) and 0 (+0.0: no root can exist) for an empty box.
LF_HD bool box_windows(const int4 &b, int &nx, int &ny, uint32_t &mx) {
    if (b.x < 0) {
        mx = 0x7c00u;
        return false;
    }
    if (b.x > b.y || b.z > b.w) {
        mx = 0u;
        return false;
    }
    nx = (b.y - b.x + kWin) / kWin;
    ny = (b.w - b.z + kWin) / kWin;
    return true;
}
LF_HD uint32_t box_window_index(const int4 &b, int tx, int ty, int Mc) {
    const int j = min(b.x + kWin * tx, max(b.y - (kWin - 1), b.x));
    const int k = min(b.z + kWin * ty, max(b.w - (kWin - 1), b.z));
    return (uint32_t)(k * Mc + j);
}

// The ray's line in view grid coordinates, g = (ax + w bx, ay + w by), with
// 1 / bx and 1 / by, clipped to the mesh domain 0 <= g <= M-1 on both axes:
// [wlo, whi] shrinks to the part of the line over the domain. False when
// nothing is left. A slope below 1e-20 in magnitude is raised to 1e-20 (same
// sign): over any inverse-depth range the line then stays in one column or
// row of cells, and its interval over the domain is every w or none, as for
// a line that does not move along the axis at all.
struct GridLine {
    float ax, bx, ibx, ay, by, iby;
};
// b with its magnitude raised to at least 1e-20 (b finite)
LF_HD float min_slope(float b) { return copysignf(clamp_range(fabsf(b), 1e-20f, FLT_MAX), b); }
LF_HD bool grid_line(int M, float sM, float cM, float Vx, float Vy, float Dx, float Dy, float &wlo, float &whi,
                     GridLine &L) {
    const float lim = (float)(M - 1);
    L.ax = fmaf(Vx, sM, cM);
    L.bx = min_slope(Dx * sM);
    L.ay = fmaf(-Vy, sM, cM);
    L.by = min_slope(-Dy * sM);
    L.ibx = fast_rcp(L.bx);
    L.iby = fast_rcp(L.by);
    // per axis the domain is w in [x1, x1 + lim / b] (either order)
    const float x1 = -L.ax * L.ibx, xl = lim * L.ibx;
    const float y1 = -L.ay * L.iby, yl = lim * L.iby;
    wlo = fmaxf(wlo, fmaxf(x1 + fminf(xl, 0.0f), y1 + fminf(yl, 0.0f)));
    whi = fminf(whi, fminf(x1 + fmaxf(xl, 0.0f), y1 + fmaxf(yl, 0.0f)));
    return wlo <= whi;
}

// Largest w in [wlo, whi] at which the line (V + w D, w) meets the view's
// mesh, when no root lies above w = wtop (an upper bound of the mesh's inverse
// depth over every cell the line can reach, e.g. from tile_cell_box): one
// walk over the cells from min(whi, wtop) down, without the block level.
template <int GEO>
LF_HD bool march_top(const void *__restrict__ cells, int M, float sM, float cM, float wlo, float whi, float wtop,
                     float Vx, float Vy, float Dx, float Dy, float &w_hit, int &n_cells) {
    GridLine L;
    if (!grid_line(M, sM, cM, Vx, Vy, Dx, Dy, wlo, whi, L)) return false;
    const float ws = whi < wtop ? whi : wtop;  // neither is NaN here
    if (!(ws >= wlo)) return false;
    const int Mc = M - 1;
    // a segment crosses at most 2 Mc - 1 cells of the Mc x Mc grid
    return walk_cells<GEO>(cells, Mc, L.ax, L.bx, L.ibx, L.ay, L.by, L.iby, kTolW * fabsf(whi), 0, Mc - 1, 0,
                           Mc - 1, ws, wlo, 2 * Mc + 2, w_hit, n_cells);
}

// Largest w in [wlo, whi] at which the line (V + w D, w) meets the view's
// mesh; false if it never does. Two levels: blocks of kBlk x kBlk cells
// carry the min / max inverse depth of their vertices, and a root inside a
// block lies in that range, so each block's cells are walked only over the
// part of the line whose w falls inside the block's range.
template <int GEO>
LF_HD bool march(const void *__restrict__ cells, const float2 *__restrict__ blk, int M, int NB, float sM,
                 float cM, float wlo, float whi, float Vx, float Vy, float Dx, float Dy, float &w_hit,
                 int &n_cells) {
    GridLine L;
    if (!grid_line(M, sM, cM, Vx, Vy, Dx, Dy, wlo, whi, L)) return false;
    const float ax = L.ax, bx = L.bx, ibx = L.ibx, ay = L.ay, by = L.by, iby = L.iby;

    const int Mc = M - 1;
    const int sbx = bx > 0.0f ? -1 : 1, sby = by > 0.0f ? -1 : 1;
    const float tol = kTolW * fabsf(whi);
    float w0 = whi;
    int bi = (int)((unsigned)min(max((int)floorf(fmaf(w0, bx, ax)), 0), Mc - 1) / kBlk);
    int bk = (int)((unsigned)min(max((int)floorf(fmaf(w0, by, ay)), 0), Mc - 1) / kBlk);
    bool found = false, more = true;
    for (int it = 0; it < 2 * NB + 4 && more; ++it) {
        const int j0 = bi * kBlk, j1 = min(j0 + kBlk, Mc) - 1;
        const int k0 = bk * kBlk, k1 = min(k0 + kBlk, Mc) - 1;
        // inverse depth at which the line leaves the block
        const float wxe = ((float)(bx > 0.0f ? j0 : j1 + 1) - ax) * ibx;
        const float wye = ((float)(by > 0.0f ? k0 : k1 + 1) - ay) * iby;
        const float wn = fmaxf(wxe, wye);
        const bool last = !(wn > wlo);
        const float wb1 = last ? wlo : fminf(wn, w0);
        const float2 bb = at<float2>(blk, mul24(bk, NB) + bi);
        const float ws = fminf(w0, bb.y), we = fmaxf(wb1, bb.x);
        if (ws >= we)
            found = walk_cells<GEO>(cells, Mc, ax, bx, ibx, ay, by, iby, tol, j0, j1, k0, k1, ws, we, 2 * kBlk + 2,
                                    w_hit, n_cells);
        bi += wxe == wn ? sbx : 0;
        bk += wye == wn ? sby : 0;
        more = !found && !last && bi >= 0 && bi < NB && bk >= 0 && bk < NB;
        w0 = wb1;
    }
    return found;
}

// Inverse depth w of a view's mesh at its image-plane point (X, Y): the
// plane of the cell triangle holding the point (triangle A for fx >= fy,
// B otherwise, as in cell_root). False outside the mesh domain (the square
// spanned by the depth-pixel centres).
template <int GEO>
LF_HD bool mesh_point(const void *__restrict__ cells, int M, float sM, float cM, float X, float Y, float &w) {
    const float gx = fmaf(X, sM, cM), gy = fmaf(-Y, sM, cM);
    const float lim = (float)(M - 1);
    if (!(gx >= 0.0f && gx <= lim && gy >= 0.0f && gy <= lim)) return false;
    const int Mc = M - 1;
    const int j = min((int)gx, Mc - 1), k = min((int)gy, Mc - 1);
    const float fx = gx - (float)j, fy = gy - (float)k;
    const float4 c = load_cell<GEO>(cells, mul24(k, Mc) + j);
    w = fx >= fy ? fmaf(fy, c.w - c.y, fmaf(fx, c.y - c.x, c.x)) : fmaf(fy, c.z - c.x, fmaf(fx, c.w - c.z, c.x));
    return true;
}

// Bilinear taps along one axis of n texels with clamp-to-edge, at position p
// in texel units with texel i's centre at i: taps i0, i1 = i0 + 1 (cut at the
// edge) and the weight f of i1. Clamping p into [0, n-1] first yields the
// same sample as clamping each tap (outside, both taps are the edge texel).
LF_HD void taps(float p, int n, int &i0, int &i1, float &f) {
    const float q = fminf(fmaxf(p, 0.0f), (float)(n - 1));
    i0 = (int)q;
    f = q - (float)i0;
    i1 = min(i0 + 1, n - 1);
}

// The same taps for n >= 2 texels, with the second tap always i0 + 1: the
// position clamped into [0, lim] (lim = n - 1 as a float), i0 = min(floor,
// n - 2) and the weight f in [0, 1] of i0 + 1. The sample equals the one of
// taps() (at the last texel the whole weight sits on i0 + 1 = n - 1), and
// the four taps of a bilinear sample sit at fixed offsets from the first.
LF_HD float clamp_to(float p, float lim) {  // p clamped into [0, lim] (p finite, lim >= 0)
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_fmed3f(p, 0.0f, lim);
#else
    return fminf(fmaxf(p, 0.0f), lim);
#endif
}
LF_HD void taps_next(float p, int n, float lim, int &i0, float &f) {
    const float q = clamp_to(p, lim);
    i0 = min((int)q, n - 2);
    f = q - (float)i0;
}

// Bilinear sample at normalised image-plane point (Xs, Ys): texel centres at
// half-integers, clamp-to-edge (result in texel units; see texel_scale).
// W, H >= 2; limx = W - 1, limy = H - 1.
template <int IMG>
LF_HD Rgb bilinear(const void *__restrict__ img, int W, int H, float limx, float limy, float px, float py) {
    int x0, y0;
    float fx, fy;
    taps_next(px, W, limx, x0, fx);
    taps_next(py, H, limy, y0, fy);
    const uint32_t r0 = mul24(y0, W) + x0, r1 = r0 + W;
    // the right-hand taps through a fixed byte offset from their row's first
    // tap (an address offset, not an index: one 32-bit offset per row)
    const void *p0 = texel_row<IMG>(img, r0), *p1 = texel_row<IMG>(img, r1);
    const Rgb a = texel<IMG>(p0, 0), b = texel<IMG>(p0, 1);
    const Rgb c = texel<IMG>(p1, 0), d = texel<IMG>(p1, 1);
    // the four tap weights; FP16 taps then feed mixed-precision FMAs directly
    const float w11 = fx * fy, w10 = fx - w11, w01 = fy - w11, w00 = (1.0f - fx) - w01;
    return {fmaf(w11, d.r, fmaf(w01, c.r, fmaf(w10, b.r, fmaf(w00, a.r, 0.0f)))),
            fmaf(w11, d.g, fmaf(w01, c.g, fmaf(w10, b.g, fmaf(w00, a.g, 0.0f)))),
            fmaf(w11, d.b, fmaf(w01, c.b, fmaf(w10, b.b, fmaf(w00, a.b, 0.0f))))};
}

// YUV420 sample (result in 0..255 units): luma bilinear at full resolution,
// chroma bilinear at half resolution with chroma sample (i, j) at the centre
// of luma block (2i..2i+1, 2j..2j+1), i.e. at chroma coordinate
// ((px - 1/2) / 2, (py - 1/2) / 2); clamp-to-edge on both planes; recombined
// with the full-range BT.601 inverse.
LF_HD Rgb bilinear_yuv(const void *__restrict__ yp, const void *__restrict__ uvp, int W, int H, float px, float py) {
    float lum;
    {
        int x0, x1, y0, y1;
        float fx, fy;
        taps(px, W, x0, x1, fx);
        taps(py, H, y0, y1, fy);
        const uint32_t r0 = mul24(y0, W), r1 = mul24(y1, W);
        const float a = at<uint8_t>(yp, r0 + x0), b = at<uint8_t>(yp, r0 + x1);
        const float c = at<uint8_t>(yp, r1 + x0), d = at<uint8_t>(yp, r1 + x1);
        const float w11 = fx * fy, w10 = fx - w11, w01 = fy - w11, w00 = (1.0f - fx) - w01;
        lum = fmaf(w11, d, fmaf(w01, c, fmaf(w10, b, w00 * a)));
    }
    float cb, cr;
    {
        const int Wc = W >> 1, Hc = H >> 1;
        const float cx = 0.5f * (px - 0.5f), cy = 0.5f * (py - 0.5f);
        int x0, x1, y0, y1;
        float fx, fy;
        taps(cx, Wc, x0, x1, fx);
        taps(cy, Hc, y0, y1, fy);
        const uint32_t r0 = mul24(y0, Wc), r1 = mul24(y1, Wc);
        const uint32_t a = at<uint16_t>(uvp, r0 + x0), b = at<uint16_t>(uvp, r0 + x1);
        const uint32_t c = at<uint16_t>(uvp, r1 + x0), d = at<uint16_t>(uvp, r1 + x1);
        const float w11 = fx * fy, w10 = fx - w11, w01 = fy - w11, w00 = (1.0f - fx) - w01;
        cb = fmaf(w11, (float)(d & 255u), fmaf(w01, (float)(c & 255u), fmaf(w10, (float)(b & 255u), w00 * (float)(a & 255u)))) - 128.0f;
        cr = fmaf(w11, (float)(d >> 8), fmaf(w01, (float)(c >> 8), fmaf(w10, (float)(b >> 8), w00 * (float)(a >> 8)))) - 128.0f;
    }
    return {fmaf(1.402f, cr, lum), fmaf(-0.714136f, cr, fmaf(-0.344136f, cb, lum)), fmaf(1.772f, cb, lum)};
}

// Paged RGBA8 images (tile streaming): texel (x, y) lives in image tile
// (x >> 6, y >> 6), whose cache page pt[tile] holds it at (y & 63, x & 63);
// pages are 16 KB apart in pool. A sample is taken only if the pages of all
// four taps are in the cache (pt >= 0); otherwise the view is left out for
// this ray (result false).
LF_HD uint32_t paged_texel(const char *__restrict__ pool, int32_t page, int x, int y) {
    return at<uint32_t>(pool + (int64_t)page * (kPage * kPage * 4), (uint32_t)(((y & (kPage - 1)) << kPageShift) | (x & (kPage - 1))));
}
LF_HD bool bilinear_paged(const void *__restrict__ pt, const char *__restrict__ pool, int tiles_x, int W, int H,
                          float px, float py, Rgb &out) {
    int x0, x1, y0, y1;
    float fx, fy;
    taps(px, W, x0, x1, fx);
    taps(py, H, y0, y1, fy);
    const uint32_t r0 = mul24(y0 >> kPageShift, tiles_x), r1 = mul24(y1 >> kPageShift, tiles_x);
    const int32_t p00 = at<int32_t>(pt, r0 + (x0 >> kPageShift)), p10 = at<int32_t>(pt, r0 + (x1 >> kPageShift));
    const int32_t p01 = at<int32_t>(pt, r1 + (x0 >> kPageShift)), p11 = at<int32_t>(pt, r1 + (x1 >> kPageShift));
    if ((p00 | p10 | p01 | p11) < 0) return false;
    const uint32_t ta = paged_texel(pool, p00, x0, y0), tb = paged_texel(pool, p10, x1, y0);
    const uint32_t tc = paged_texel(pool, p01, x0, y1), td = paged_texel(pool, p11, x1, y1);
    const float w11 = fx * fy, w10 = fx - w11, w01 = fy - w11, w00 = (1.0f - fx) - w01;
    float c[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const uint32_t sh = 8u * k;
        c[k] = fmaf(w11, (float)((td >> sh) & 255u),
                    fmaf(w01, (float)((tc >> sh) & 255u), fmaf(w10, (float)((tb >> sh) & 255u), fmaf(w00, (float)((ta >> sh) & 255u), 0.0f))));
    }
    out = {c[0], c[1], c[2]};
    return true;
}

// Visibility pass: mark the image tiles of the four taps of a sample.
LF_HD void mark_taps(uint8_t *__restrict__ vis, int tiles_x, int W, int H, float px, float py) {
    int x0, x1, y0, y1;
    float fx, fy;
    taps(px, W, x0, x1, fx);
    taps(py, H, y0, y1, fy);
    const int r0 = (y0 >> kPageShift) * tiles_x, r1 = (y1 >> kPageShift) * tiles_x;
    vis[r0 + (x0 >> kPageShift)] = 1;
    vis[r0 + (x1 >> kPageShift)] = 1;
    vis[r1 + (x0 >> kPageShift)] = 1;
    vis[r1 + (x1 >> kPageShift)] = 1;
}

// One texel of an RGTC1 (BC4 unsigned) block held as two little-endian words:
// endpoints e0 = byte 0, e1 = byte 1, then the 3-bit code of texel t = 4 y + x
// at bit 16 + 3 t. Code 0 is e0, code 1 is e1 and codes 2..7 are the sevenths
// from e0 towards e1 (code c at c - 1 sevenths); result in 0..255 units. Only
// the eight-point form is decoded: the blocks come from this library's own
// encoder, which writes e0 > e1, or e0 = e1 with every code 0 (where both
// forms give e0), never the five-point form's codes.
LF_HD float rgtc1_texel(uint32_t lo, uint32_t hi, uint32_t t) {
    const uint64_t bits = ((uint64_t)hi << 32) | lo;
    const uint32_t c = (uint32_t)(bits >> (16u + 3u * t)) & 7u;
    // sevenths from e0 by code: 0, 7, 1, 2, 3, 4, 5, 6 (3-bit fields of an octal constant)
    const uint32_t p = (065432170u >> (3u * c)) & 7u;
    const float f0 = (float)(lo & 255u), f1 = (float)((lo >> 8) & 255u);
    return fmaf((float)p * (1.0f / 7.0f), f1 - f0, f0);
}

// RGTC form of the YUV420 planes (result in 0..255 units): the luma plane as
// RGTC1 blocks (8 bytes per 4 x 4 texels) and the chroma plane as RGTC2 blocks
// (16 bytes: the Cb block, then the Cr block), both row-major over blocks;
// texels decoded from their blocks, then sampled and recombined as in
// bilinear_yuv. W and H are multiples of 8.
LF_HD float rgtc_luma(const void *__restrict__ yp, int Wb, int x, int y) {
    const uint2 b = at<uint2>(yp, mul24(y >> 2, Wb) + (x >> 2));
    return rgtc1_texel(b.x, b.y, (uint32_t)(((y & 3) << 2) | (x & 3)));
}
LF_HD void rgtc_chroma(const void *__restrict__ uvp, int Wb, int x, int y, float &cb, float &cr) {
    const uint4 b = at<uint4>(uvp, mul24(y >> 2, Wb) + (x >> 2));
    const uint32_t t = (uint32_t)(((y & 3) << 2) | (x & 3));
    cb = rgtc1_texel(b.x, b.y, t);
    cr = rgtc1_texel(b.z, b.w, t);
}
LF_HD Rgb bilinear_rgtc(const void *__restrict__ yp, const void *__restrict__ uvp, int W, int H, float px, float py) {
    float lum;
    {
        int x0, x1, y0, y1;
        float fx, fy;
        taps(px, W, x0, x1, fx);
        taps(py, H, y0, y1, fy);
        const int Wb = W >> 2;
        const float a = rgtc_luma(yp, Wb, x0, y0), b = rgtc_luma(yp, Wb, x1, y0);
        const float c = rgtc_luma(yp, Wb, x0, y1), d = rgtc_luma(yp, Wb, x1, y1);
        const float w11 = fx * fy, w10 = fx - w11, w01 = fy - w11, w00 = (1.0f - fx) - w01;
        lum = fmaf(w11, d, fmaf(w01, c, fmaf(w10, b, w00 * a)));
    }
    float cb, cr;
    {
        const int Wc = W >> 1, Hc = H >> 1, Wb = W >> 3;
        const float cx = 0.5f * (px - 0.5f), cy = 0.5f * (py - 0.5f);
        int x0, x1, y0, y1;
        float fx, fy;
        taps(cx, Wc, x0, x1, fx);
        taps(cy, Hc, y0, y1, fy);
        float ab, ar, bb, br, cb_, cr_, db, dr;
        rgtc_chroma(uvp, Wb, x0, y0, ab, ar);
        rgtc_chroma(uvp, Wb, x1, y0, bb, br);
        rgtc_chroma(uvp, Wb, x0, y1, cb_, cr_);
        rgtc_chroma(uvp, Wb, x1, y1, db, dr);
        const float w11 = fx * fy, w10 = fx - w11, w01 = fy - w11, w00 = (1.0f - fx) - w01;
        cb = fmaf(w11, db, fmaf(w01, cb_, fmaf(w10, bb, w00 * ab))) - 128.0f;
        cr = fmaf(w11, dr, fmaf(w01, cr_, fmaf(w10, br, w00 * ar))) - 128.0f;
    }
    return {fmaf(1.402f, cr, lum), fmaf(-0.714136f, cr, fmaf(-0.344136f, cb, lum)), fmaf(1.772f, cb, lum)};
}

}  // namespace lf
