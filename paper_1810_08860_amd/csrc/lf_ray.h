// Per-ray arithmetic of the renderer, shared by the HIP kernels and usable
// from host code (LF_HD = __host__ __device__): storage-format loads, the exact
// disk test, the inverse-depth mesh walk and bilinear sampling.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

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

template <int IMG>
LF_HD Rgb texel(const void *__restrict__ img, int64_t idx);

template <>
LF_HD Rgb texel<0>(const void *__restrict__ img, int64_t idx) {  // RGBA8, 0..255
    const uint32_t p = reinterpret_cast<const uint32_t *>(img)[idx];
    return {(float)(p & 255u), (float)((p >> 8) & 255u), (float)((p >> 16) & 255u)};
}
template <>
LF_HD Rgb texel<1>(const void *__restrict__ img, int64_t idx) {  // RGBA16F
    uint2 p = reinterpret_cast<const uint2 *>(img)[idx];
    __half2 rg = *reinterpret_cast<__half2 *>(&p.x);
    __half2 ba = *reinterpret_cast<__half2 *>(&p.y);
    return {__low2float(rg), __high2float(rg), __low2float(ba)};
}
template <>
LF_HD Rgb texel<2>(const void *__restrict__ img, int64_t idx) {  // RGBA32F
    float4 p = reinterpret_cast<const float4 *>(img)[idx];
    return {p.x, p.y, p.z};
}

// scale from stored texel units to [0,1]
template <int IMG>
LF_HD float texel_scale() { return IMG == 0 ? (1.0f / 255.0f) : 1.0f; }

// Corner inverse depths of one mesh cell: (w00, w10, w01, w11) with j to the
// right and k downwards.
template <int GEO>
LF_HD float4 load_cell(const void *__restrict__ cells, int64_t idx);

template <>
LF_HD float4 load_cell<0>(const void *__restrict__ cells, int64_t idx) {
    return reinterpret_cast<const float4 *>(cells)[idx];
}
template <>
LF_HD float4 load_cell<1>(const void *__restrict__ cells, int64_t idx) {
    uint2 p = reinterpret_cast<const uint2 *>(cells)[idx];
    __half2 a = *reinterpret_cast<__half2 *>(&p.x);
    __half2 b = *reinterpret_cast<__half2 *>(&p.y);
    return make_float4(__low2float(a), __high2float(a), __low2float(b), __high2float(b));
}

// ---------------------------------------------------------------------------------------------
// per-ray pieces

struct RayView {
    float Vx, Vy, Dx, Dy, rho;
};

// Exact disk test of one ray against one view (Sec. 3.1: linear falloff, disk
// in the view's tangent plane). False for a back-facing disk or rho <= 0.
LF_HD bool disk_test(const EyeView &v, float X, float Y, float R, float invR,
                                          RayView &rv) {
    const float ez = fmaf(v.m[6], X, fmaf(v.m[7], Y, v.m[8]));
    if (!(ez > 0.0f)) return false;
    const float iz = fast_rcp(ez);
    const float Vx = fmaf(v.m[0], X, fmaf(v.m[1], Y, v.m[2])) * iz;
    const float Vy = fmaf(v.m[3], X, fmaf(v.m[4], Y, v.m[5])) * iz;
    const float Dx = fmaf(-v.o[2], Vx, v.o[0]);
    const float Dy = fmaf(-v.o[2], Vy, v.o[1]);
    const float r2 = fmaf(Dx, Dx, Dy * Dy);
    if (!(r2 < R * R)) return false;
    const float rho = fmaf(-fast_sqrt(r2), invR, 1.0f);
    if (!(rho > 0.0f)) return false;
    rv.Vx = Vx; rv.Vy = Vy; rv.Dx = Dx; rv.Dy = Dy; rv.rho = rho;
    return true;
}

LF_HD float sat01(float x) { return fminf(fmaxf(x, 0.0f), 1.0f); }

// Inverse depth of the cell's mesh at local (fx, fy): triangle (00,10,11) where
// fx >= fy, triangle (00,11,01) otherwise.
LF_HD float field(const float4 &c, float fx, float fy) {
    return fx >= fy ? fmaf(fy, c.w - c.y, fmaf(fx, c.y - c.x, c.x))
                    : fmaf(fx, c.w - c.z, fmaf(fy, c.z - c.x, c.x));
}

LF_HD bool crosses(float g0, float g1) {
    return (g0 < 0.0f && g1 >= 0.0f) || (g0 > 0.0f && g1 <= 0.0f);
}

// Walk the cells of one block from w = ws down to w = we (ws >= we), starting
// in the cell that holds the line at ws (clamped to the block's cells
// [j0, j1] x [k0, k1]). `sgn` is the sign of field - w just above ws (0 if
// unknown); on return it holds the sign at we. True with w_hit on a crossing.
template <int GEO>
LF_HD bool walk_cells(const void *__restrict__ cells, int Mc, float ax, float bx, float ibx,
                                           bool mx, float ay, float by, float iby, bool my, int j0, int j1, int k0,
                                           int k1, float ws, float we, int &sgn, float &w_hit, int &n_cells) {
    const int sx = bx > 0.0f ? -1 : 1, sy = by > 0.0f ? -1 : 1;  // cell steps as w decreases
    const float ox = bx > 0.0f ? 0.0f : 1.0f, oy = by > 0.0f ? 0.0f : 1.0f;
    float w0 = ws;
    const float gx = fmaf(w0, bx, ax), gy = fmaf(w0, by, ay);
    int j = min(max((int)floorf(gx), j0), j1);
    int k = min(max((int)floorf(gy), k0), k1);
    float4 cw = load_cell<GEO>(cells, (int64_t)k * Mc + j);
    ++n_cells;
    float fx0 = sat01(gx - (float)j), fy0 = sat01(gy - (float)k);
    float g0 = field(cw, fx0, fy0) - w0;
    if (g0 == 0.0f || (sgn < 0 && g0 > 0.0f) || (sgn > 0 && g0 < 0.0f)) {
        w_hit = w0;
        return true;
    }
    for (int it = 0; it < 64; ++it) {
        // inverse depth at which the line leaves cell (j, k)
        const float wxe = mx ? ((float)j + ox - ax) * ibx : -INFINITY;
        const float wye = my ? ((float)k + oy - ay) * iby : -INFINITY;
        const float wn = fmaxf(wxe, wye);
        const bool last = !(wn > we);
        const float w1 = last ? we : fminf(wn, w0);
        const float fx1 = sat01(fmaf(w1, bx, ax) - (float)j), fy1 = sat01(fmaf(w1, by, ay) - (float)k);
        const float d0 = fx0 - fy0, d1 = fx1 - fy1;
        if ((d0 > 0.0f && d1 < 0.0f) || (d0 < 0.0f && d1 > 0.0f)) {
            // the segment crosses the cell diagonal: two linear pieces
            const float s = d0 * fast_rcp(d0 - d1);
            const float wd = fmaf(s, w1 - w0, w0);
            const float fd = fmaf(s, fx1 - fx0, fx0);
            const float gd = field(cw, fd, fd) - wd;
            if (crosses(g0, gd)) {
                w_hit = fmaf(wd - w0, g0 * fast_rcp(g0 - gd), w0);
                return true;
            }
            w0 = wd;
            g0 = gd;
            fx0 = fd;
            fy0 = fd;
        }
        const float g1 = field(cw, fx1, fy1) - w1;
        if (crosses(g0, g1)) {
            w_hit = fmaf(w1 - w0, g0 * fast_rcp(g0 - g1), w0);
            return true;
        }
        if (last) {
            sgn = g1 > 0.0f ? 1 : -1;
            return false;
        }
        if (wxe == wn) j += sx;
        if (wye == wn) k += sy;
        if (j < j0 || j > j1 || k < k0 || k > k1) {
            sgn = g1 > 0.0f ? 1 : -1;
            return false;
        }
        cw = load_cell<GEO>(cells, (int64_t)k * Mc + j);
        ++n_cells;
        fx0 = sat01(fmaf(w1, bx, ax) - (float)j);
        fy0 = sat01(fmaf(w1, by, ay) - (float)k);
        w0 = w1;
        g0 = g1;
    }
    sgn = g0 > 0.0f ? 1 : -1;
    return false;
}

// Largest w in [wlo, whi] at which the line (V + w D, w) meets the view's
// mesh; false if it never does. Two levels: blocks of kBlk x kBlk cells
// carry the min / max inverse depth of their vertices, and a crossing inside
// a block must lie in that range, so each block's cells are walked only over
// the part of the line whose w falls inside the block's range.
template <int GEO>
LF_HD bool march(const void *__restrict__ cells, const float2 *__restrict__ blk, int M, int NB, float sM,
                      float cM, float wlo, float whi, float Vx, float Vy, float Dx, float Dy, float &w_hit,
                      int &n_cells) {
    const float lim = (float)(M - 1);
    const float ax = fmaf(Vx, sM, cM), bx = Dx * sM;
    const float ay = fmaf(-Vy, sM, cM), by = -Dy * sM;
    const bool mx = fabsf(bx) > 1e-20f, my = fabsf(by) > 1e-20f;
    const float ibx = mx ? fast_rcp(bx) : 0.0f, iby = my ? fast_rcp(by) : 0.0f;
    // clip to the mesh domain 0 <= g <= M-1 on both axes
    if (mx) {
        const float w1 = -ax * ibx, w2 = (lim - ax) * ibx;
        wlo = fmaxf(wlo, fminf(w1, w2));
        whi = fminf(whi, fmaxf(w1, w2));
    } else if (!(ax >= 0.0f && ax <= lim)) {
        return false;
    }
    if (my) {
        const float w1 = -ay * iby, w2 = (lim - ay) * iby;
        wlo = fmaxf(wlo, fminf(w1, w2));
        whi = fminf(whi, fmaxf(w1, w2));
    } else if (!(ay >= 0.0f && ay <= lim)) {
        return false;
    }
    if (!(wlo <= whi)) return false;

    const int Mc = M - 1;
    const int sbx = bx > 0.0f ? -1 : 1, sby = by > 0.0f ? -1 : 1;
    float w0 = whi;
    int bi = min(max((int)floorf(fmaf(w0, bx, ax)), 0), M - 2) / kBlk;
    int bk = min(max((int)floorf(fmaf(w0, by, ay)), 0), M - 2) / kBlk;
    int sgn = 0;  // sign of field - w just above w0 (0: not known yet)
    for (int it = 0; it < 2 * NB + 4; ++it) {
        const int j0 = bi * kBlk, j1 = min(j0 + kBlk, Mc) - 1;
        const int k0 = bk * kBlk, k1 = min(k0 + kBlk, Mc) - 1;
        // inverse depth at which the line leaves the block
        const float wxe = mx ? ((float)(bx > 0.0f ? j0 : j1 + 1) - ax) * ibx : -INFINITY;
        const float wye = my ? ((float)(by > 0.0f ? k0 : k1 + 1) - ay) * iby : -INFINITY;
        const float wn = fmaxf(wxe, wye);
        const bool last = !(wn > wlo);
        const float wb1 = last ? wlo : fminf(wn, w0);
        const float2 bb = blk[bk * NB + bi];
        const float ws = fminf(w0, bb.y), we = fmaxf(wb1, bb.x);
        if (ws >= we) {
            // part of the line above the block's surface (w > max): field - w < 0
            int s = ws < w0 ? -1 : sgn;
            if (walk_cells<GEO>(cells, Mc, ax, bx, ibx, mx, ay, by, iby, my, j0, j1, k0, k1, ws, we, s, w_hit,
                                n_cells))
                return true;
            sgn = we > wb1 ? 1 : s;  // below the block's surface (w < min): field - w > 0
        } else {
            const int s = w0 < bb.x ? 1 : -1;
            if (sgn != 0 && s != sgn) {  // sign flips exactly on the block boundary
                w_hit = w0;
                return true;
            }
            sgn = s;
        }
        if (last) return false;
        if (wxe == wn) bi += sbx;
        if (wye == wn) bk += sby;
        if (bi < 0 || bi >= NB || bk < 0 || bk >= NB) return false;
        w0 = wb1;
    }
    return false;
}

// Bilinear sample at normalised image-plane point (Xs, Ys): texel centres at
// half-integers, clamp-to-edge (result in texel units; see texel_scale).
template <int IMG>
LF_HD Rgb bilinear(const void *__restrict__ img, int W, int H, float px, float py) {
    const float x0f = floorf(px), y0f = floorf(py);
    const float fx = px - x0f, fy = py - y0f;
    int x0 = (int)x0f, y0 = (int)y0f;
    int x1 = min(max(x0 + 1, 0), W - 1), y1 = min(max(y0 + 1, 0), H - 1);
    x0 = min(max(x0, 0), W - 1);
    y0 = min(max(y0, 0), H - 1);
    const Rgb a = texel<IMG>(img, (int64_t)y0 * W + x0), b = texel<IMG>(img, (int64_t)y0 * W + x1);
    const Rgb c = texel<IMG>(img, (int64_t)y1 * W + x0), d = texel<IMG>(img, (int64_t)y1 * W + x1);
    const float tr = fmaf(fx, b.r - a.r, a.r), tg = fmaf(fx, b.g - a.g, a.g), tb = fmaf(fx, b.b - a.b, a.b);
    const float br = fmaf(fx, d.r - c.r, c.r), bg = fmaf(fx, d.g - c.g, c.g), bb = fmaf(fx, d.b - c.b, c.b);
    return {fmaf(fy, br - tr, tr), fmaf(fy, bg - tg, tg), fmaf(fy, bb - tb, tb)};
}

}  // namespace lf
