// HIP kernels for disk-blended light field reconstruction on CDNA4 (gfx950).
//
// Data path for one eye (Sec. 3.1, Eqs. (1)-(2); Sec. 3.2):
//   k_prep    per (eye, view): the 3x3 map taking an eye-image point (X, Y, 1)
//             to the ray direction in the view's frame, and the eye centre in
//             that frame (FP64 set-up, stored FP32).
//   k_cull    per screen tile, one wavefront: every view's disk is tested
//             against the tile's frustum (conservatively); survivors are
//             compacted into an LDS list with a wavefront ballot and prefix
//             popcount, then written out (the GPU counterpart of the paper's
//             per-tile visibility culling, Sec. 3.2.1 and Sec. 6.2).
//   k_render  per screen tile: the tile's candidate views are staged in LDS;
//             every pixel tests each candidate's disk exactly, intersects its
//             ray with the view's mesh, samples the view's image bilinearly and
//             accumulates rho-weighted colour and rho in FP32 registers; the
//             division of the paper's second pass is the kernel's epilogue.
//
// Mesh intersection. In view i's frame the ray is o' + t e'. With the
// vanishing point V = (e'x, e'y) / e'z and the disk coordinates
// D = (o'x, o'y) - o'z V (exactly the (u, v) at which the ray crosses the disk
// plane), the ray point at inverse depth w = 1/z projects to V + w D. A planar
// triangle stays planar in (X, Y, w), so view i's mesh (vertices at
// depth-pixel centres, Sec. 3.5) is the piecewise-linear field of vertex
// inverse depths over the regular grid, and the ray is the straight line
// w -> (V + w D, w). The nearest hit along the ray (intra-image occlusion,
// Sec. 3.2.2) is the LARGEST w at which the line meets the field; the kernel
// walks grid cells from the view's largest inverse depth downwards, finds the
// first sign change of field(w) - w on each linear piece (cells split along
// their diagonal), and interpolates it. (s, t) = V + w_hit D exactly.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <math.h>

#include "lf_internal.h"

namespace lf {

// ---------------------------------------------------------------------------------------------
// storage formats

struct Rgb {
    float r, g, b;
};

template <int IMG>
__device__ __forceinline__ Rgb texel(const void *__restrict__ img, int64_t idx);

template <>
__device__ __forceinline__ Rgb texel<0>(const void *__restrict__ img, int64_t idx) {  // RGBA8, 0..255
    const uint32_t p = reinterpret_cast<const uint32_t *>(img)[idx];
    return {(float)(p & 255u), (float)((p >> 8) & 255u), (float)((p >> 16) & 255u)};
}
template <>
__device__ __forceinline__ Rgb texel<1>(const void *__restrict__ img, int64_t idx) {  // RGBA16F
    uint2 p = reinterpret_cast<const uint2 *>(img)[idx];
    __half2 rg = *reinterpret_cast<__half2 *>(&p.x);
    __half2 ba = *reinterpret_cast<__half2 *>(&p.y);
    return {__low2float(rg), __high2float(rg), __low2float(ba)};
}
template <>
__device__ __forceinline__ Rgb texel<2>(const void *__restrict__ img, int64_t idx) {  // RGBA32F
    float4 p = reinterpret_cast<const float4 *>(img)[idx];
    return {p.x, p.y, p.z};
}

// scale from stored texel units to [0,1]
template <int IMG>
__device__ __forceinline__ float texel_scale() { return IMG == 0 ? (1.0f / 255.0f) : 1.0f; }

// Corner inverse depths of one mesh cell: (w00, w10, w01, w11) with j to the
// right and k downwards.
template <int GEO>
__device__ __forceinline__ float4 load_cell(const void *__restrict__ cells, int64_t idx);

template <>
__device__ __forceinline__ float4 load_cell<0>(const void *__restrict__ cells, int64_t idx) {
    return reinterpret_cast<const float4 *>(cells)[idx];
}
template <>
__device__ __forceinline__ float4 load_cell<1>(const void *__restrict__ cells, int64_t idx) {
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
__device__ __forceinline__ bool disk_test(const EyeView &v, float X, float Y, float R, float invR,
                                          RayView &rv) {
    const float ez = fmaf(v.m[6], X, fmaf(v.m[7], Y, v.m[8]));
    if (!(ez > 0.0f)) return false;
    const float iz = 1.0f / ez;
    const float Vx = fmaf(v.m[0], X, fmaf(v.m[1], Y, v.m[2])) * iz;
    const float Vy = fmaf(v.m[3], X, fmaf(v.m[4], Y, v.m[5])) * iz;
    const float Dx = fmaf(-v.o[2], Vx, v.o[0]);
    const float Dy = fmaf(-v.o[2], Vy, v.o[1]);
    const float r2 = fmaf(Dx, Dx, Dy * Dy);
    if (!(r2 < R * R)) return false;
    const float rho = fmaf(-sqrtf(r2), invR, 1.0f);
    if (!(rho > 0.0f)) return false;
    rv.Vx = Vx; rv.Vy = Vy; rv.Dx = Dx; rv.Dy = Dy; rv.rho = rho;
    return true;
}

__device__ __forceinline__ float sat01(float x) { return fminf(fmaxf(x, 0.0f), 1.0f); }

// Inverse depth of the cell's mesh at local (fx, fy): triangle (00,10,11) where
// fx >= fy, triangle (00,11,01) otherwise.
__device__ __forceinline__ float field(const float4 &c, float fx, float fy) {
    return fx >= fy ? fmaf(fy, c.w - c.y, fmaf(fx, c.y - c.x, c.x))
                    : fmaf(fx, c.w - c.z, fmaf(fy, c.z - c.x, c.x));
}

__device__ __forceinline__ bool crosses(float g0, float g1) {
    return (g0 < 0.0f && g1 >= 0.0f) || (g0 > 0.0f && g1 <= 0.0f);
}

// Largest w in [wlo, whi] at which the line (V + w D, w) meets the view's
// mesh; false if it never does.
template <int GEO>
__device__ bool march(const void *__restrict__ cells, int M, float sM, float cM, float wlo, float whi, float Vx,
                      float Vy, float Dx, float Dy, float &w_hit, int &n_cells) {
    const float lim = (float)(M - 1);
    const float ax = fmaf(Vx, sM, cM), bx = Dx * sM;
    const float ay = fmaf(-Vy, sM, cM), by = -Dy * sM;
    const bool mx = fabsf(bx) > 1e-20f, my = fabsf(by) > 1e-20f;
    const float ibx = mx ? 1.0f / bx : 0.0f, iby = my ? 1.0f / by : 0.0f;
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
    float w0 = whi;
    float gx = fmaf(w0, bx, ax), gy = fmaf(w0, by, ay);
    int j = min(max((int)floorf(gx), 0), M - 2);
    int k = min(max((int)floorf(gy), 0), M - 2);
    const int sx = bx > 0.0f ? -1 : 1, sy = by > 0.0f ? -1 : 1;  // cell steps as w decreases
    const float ox = bx > 0.0f ? 0.0f : 1.0f, oy = by > 0.0f ? 0.0f : 1.0f;
    float4 cw = load_cell<GEO>(cells, (int64_t)k * Mc + j);
    ++n_cells;
    float fx0 = sat01(gx - (float)j), fy0 = sat01(gy - (float)k);
    float g0 = field(cw, fx0, fy0) - w0;
    if (g0 == 0.0f) {
        w_hit = w0;
        return true;
    }
    for (int it = 0; it < 2 * M + 4; ++it) {
        // inverse depth at which the line leaves cell (j, k)
        const float wxe = mx ? ((float)j + ox - ax) * ibx : -INFINITY;
        const float wye = my ? ((float)k + oy - ay) * iby : -INFINITY;
        const float wn = fmaxf(wxe, wye);
        const bool last = !(wn > wlo);
        const float w1 = last ? wlo : fminf(wn, w0);
        const float fx1 = sat01(fmaf(w1, bx, ax) - (float)j), fy1 = sat01(fmaf(w1, by, ay) - (float)k);
        const float d0 = fx0 - fy0, d1 = fx1 - fy1;
        if ((d0 > 0.0f && d1 < 0.0f) || (d0 < 0.0f && d1 > 0.0f)) {
            // the segment crosses the cell diagonal: two linear pieces
            const float s = d0 / (d0 - d1);
            const float wd = fmaf(s, w1 - w0, w0);
            const float fd = fmaf(s, fx1 - fx0, fx0);
            const float gd = field(cw, fd, fd) - wd;
            if (crosses(g0, gd)) {
                w_hit = fmaf(wd - w0, g0 / (g0 - gd), w0);
                return true;
            }
            w0 = wd;
            g0 = gd;
            fx0 = fd;
            fy0 = fd;
        }
        const float g1 = field(cw, fx1, fy1) - w1;
        if (crosses(g0, g1)) {
            w_hit = fmaf(w1 - w0, g0 / (g0 - g1), w0);
            return true;
        }
        if (last) return false;
        if (wxe == wn) j += sx;
        if (wye == wn) k += sy;
        if (j < 0 || j > M - 2 || k < 0 || k > M - 2) return false;
        cw = load_cell<GEO>(cells, (int64_t)k * Mc + j);
        ++n_cells;
        fx0 = sat01(fmaf(w1, bx, ax) - (float)j);
        fy0 = sat01(fmaf(w1, by, ay) - (float)k);
        w0 = w1;
        g0 = g1;
    }
    return false;
}

// Bilinear sample at normalised image-plane point (Xs, Ys): texel centres at
// half-integers, clamp-to-edge (result in texel units; see texel_scale).
template <int IMG>
__device__ __forceinline__ Rgb bilinear(const void *__restrict__ img, int W, int H, float px, float py) {
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

__device__ __forceinline__ int find_eye(const EyeChunk &ch, int tile) {
    int e = 0;
    while (e + 1 < ch.n_eyes && tile >= ch.e[e + 1].tile_off) ++e;
    return e;
}

// ---------------------------------------------------------------------------------------------
// set-up kernels

template <int FMT>
__global__ void k_convert_images(const uint32_t *__restrict__ src, void *__restrict__ dst, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t p = src[i];
        const float r = (float)(p & 255u) / 255.0f, g = (float)((p >> 8) & 255u) / 255.0f;
        const float b = (float)((p >> 16) & 255u) / 255.0f, a = (float)(p >> 24) / 255.0f;
        if (FMT == 1) {
            __half2 rg = __floats2half2_rn(r, g), ba = __floats2half2_rn(b, a);
            uint2 o;
            o.x = *reinterpret_cast<uint32_t *>(&rg);
            o.y = *reinterpret_cast<uint32_t *>(&ba);
            reinterpret_cast<uint2 *>(dst)[i] = o;
        } else {
            reinterpret_cast<float4 *>(dst)[i] = make_float4(r, g, b, a);
        }
    }
}

// Mesh cells of every view: corner inverse depths (w00, w10, w01, w11).
template <int GEO>
__global__ void k_geo_cells(const float *__restrict__ z, void *__restrict__ cells, int32_t n, int32_t M) {
    const int64_t per = (int64_t)(M - 1) * (M - 1);
    const int64_t total = per * n;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < total;
         c += (int64_t)gridDim.x * blockDim.x) {
        const int64_t v = c / per, r = c % per;
        const int k = (int)(r / (M - 1)), j = (int)(r % (M - 1));
        const float *zv = z + v * (int64_t)M * M;
        const float w00 = 1.0f / zv[(int64_t)k * M + j], w10 = 1.0f / zv[(int64_t)k * M + j + 1];
        const float w01 = 1.0f / zv[(int64_t)(k + 1) * M + j], w11 = 1.0f / zv[(int64_t)(k + 1) * M + j + 1];
        if (GEO == 0) {
            reinterpret_cast<float4 *>(cells)[c] = make_float4(w00, w10, w01, w11);
        } else {
            __half2 a = __floats2half2_rn(w00, w10), b = __floats2half2_rn(w01, w11);
            uint2 o;
            o.x = *reinterpret_cast<uint32_t *>(&a);
            o.y = *reinterpret_cast<uint32_t *>(&b);
            reinterpret_cast<uint2 *>(cells)[c] = o;
        }
    }
}

// Inverse-depth range of each view's mesh, from the stored (possibly FP16)
// values the march reads. One block per view.
template <int GEO>
__global__ __launch_bounds__(256) void k_geo_range(const void *__restrict__ cells, int32_t M,
                                                   float2 *__restrict__ wr) {
    const int64_t per = (int64_t)(M - 1) * (M - 1);
    const int64_t base = (int64_t)blockIdx.x * per;
    float lo = INFINITY, hi = -INFINITY;
    for (int64_t c = threadIdx.x; c < per; c += blockDim.x) {
        const float4 q = load_cell<GEO>(cells, base + c);
        lo = fminf(lo, fminf(fminf(q.x, q.y), fminf(q.z, q.w)));
        hi = fmaxf(hi, fmaxf(fmaxf(q.x, q.y), fmaxf(q.z, q.w)));
    }
    __shared__ float slo[256], shi[256];
    slo[threadIdx.x] = lo;
    shi[threadIdx.x] = hi;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            slo[threadIdx.x] = fminf(slo[threadIdx.x], slo[threadIdx.x + s]);
            shi[threadIdx.x] = fmaxf(shi[threadIdx.x], shi[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) wr[blockIdx.x] = make_float2(slo[0], shi[0]);
}

// Per (eye, view) frame change, computed in FP64 and stored FP32.
__global__ __launch_bounds__(256) void k_prep(const EyeChunk ch, const double *__restrict__ vt,
                                              const float2 *__restrict__ wr, int32_t n, EyeView *__restrict__ ev) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    const int e = blockIdx.y;
    if (v >= n || e >= ch.n_eyes) return;
    const double *c = vt + 12 * (int64_t)v;
    const double *R = c + 3;
    const EyeParam &E = ch.e[e];
    EyeView out;
    for (int a = 0; a < 3; ++a) {
        for (int b = 0; b < 3; ++b) {
            double s = 0.0;
            for (int r = 0; r < 3; ++r) s += R[3 * r + a] * E.rot[3 * r + b];
            out.m[3 * a + b] = (float)s;
        }
        double s = 0.0;
        for (int r = 0; r < 3; ++r) s += R[3 * r + a] * (E.pos[r] - c[r]);
        out.o[a] = (float)s;
    }
    const float2 w = wr[v];
    out.wmin = w.x;
    out.wmax = w.y;
    out.view = v;
    out.pad = 0;
    ev[(int64_t)e * n + v] = out;
}

// ---------------------------------------------------------------------------------------------
// culling

// Does any ray of the tile's pixel rectangle [X0,X1] x [Y1,Y0] cross the disk
// (radius R) of view v? Conservative: the tile's rays hit the disk plane
// inside the convex quad spanned by the four corner rays (a central
// projection of a rectangle), so the test is circle-vs-convex-quad; a tile
// that straddles the plane's horizon is kept.
__device__ __forceinline__ bool tile_overlaps_disk(const EyeView &v, float X0, float X1, float Y0, float Y1,
                                                   float R) {
    const float cx[4] = {X0, X1, X1, X0}, cy[4] = {Y0, Y0, Y1, Y1};
    float dx[4], dy[4];
    int npos = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float ez = fmaf(v.m[6], cx[q], fmaf(v.m[7], cy[q], v.m[8]));
        npos += ez > 0.0f;
        const float iz = 1.0f / ez;
        dx[q] = fmaf(-v.o[2], fmaf(v.m[0], cx[q], fmaf(v.m[1], cy[q], v.m[2])) * iz, v.o[0]);
        dy[q] = fmaf(-v.o[2], fmaf(v.m[3], cx[q], fmaf(v.m[4], cy[q], v.m[5])) * iz, v.o[1]);
    }
    if (npos == 0) return false;
    if (npos < 4) return true;
    bool allp = true, alln = true;
    float best = INFINITY;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int q1 = (q + 1) & 3;
        const float ex = dx[q1] - dx[q], ey = dy[q1] - dy[q];
        const float cr = ex * (-dy[q]) - ey * (-dx[q]);
        allp = allp && cr >= 0.0f;
        alln = alln && cr <= 0.0f;
        const float ee = fmaf(ex, ex, ey * ey);
        float t = ee > 0.0f ? -(dx[q] * ex + dy[q] * ey) / ee : 0.0f;
        t = sat01(t);
        const float px = fmaf(t, ex, dx[q]), py = fmaf(t, ey, dy[q]);
        best = fminf(best, fmaf(px, px, py * py));
    }
    return allp || alln || best <= R * R;
}

__global__ __launch_bounds__(256) void k_cull(const EyeChunk ch, const EyeView *__restrict__ ev, int32_t n,
                                              float R_keep, uint16_t *__restrict__ tile_list,
                                              int32_t *__restrict__ tile_count) {
    __shared__ uint16_t lst[4][kListCap];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int tile = blockIdx.x * 4 + wave;
    const bool active = tile < ch.total_tiles;
    int count = 0;
    if (active) {
        const int e = find_eye(ch, tile);
        const EyeParam &E = ch.e[e];
        const int local = tile - E.tile_off;
        const int x0 = (local % E.tiles_x) * ch.tile_w, y0 = (local / E.tiles_x) * ch.tile_h;
        const int x1 = min(x0 + ch.tile_w, E.W), y1 = min(y0 + ch.tile_h, E.H);
        const float X0 = (2.0f * x0 / E.W - 1.0f) * E.tx, X1 = (2.0f * x1 / E.W - 1.0f) * E.tx;
        const float Y0 = (1.0f - 2.0f * y0 / E.H) * E.ty, Y1 = (1.0f - 2.0f * y1 / E.H) * E.ty;
        const EyeView *eve = ev + (int64_t)e * n;
        const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
        for (int base = 0; base < n; base += 64) {
            const int v = base + lane;
            const bool keep = v < n && tile_overlaps_disk(eve[v], X0, X1, Y0, Y1, R_keep);
            const uint64_t mask = __ballot(keep);
            if (keep) {
                const int slot = count + __popcll(mask & below);
                if (slot < kListCap) lst[wave][slot] = (uint16_t)v;
            }
            count += __popcll(mask);
        }
    }
    __syncthreads();
    if (active) {
        const int m = min(count, kListCap);
        for (int s = lane; s < m; s += 64) tile_list[(int64_t)tile * kListCap + s] = lst[wave][s];
        if (lane == 0) tile_count[tile] = count;
    }
}

// ---------------------------------------------------------------------------------------------
// fused reproject + gather + blend

template <int IMG, int GEO, int MODE>
__global__ __launch_bounds__(256) void k_render(const EyeChunk ch, const RenderArgs a) {
    __shared__ EyeView sv[kStage];
    const int tile = blockIdx.x;
    const int e = find_eye(ch, tile);
    const EyeParam &E = ch.e[e];
    const int local = tile - E.tile_off;
    const int tx0 = (local % E.tiles_x) * ch.tile_w, ty0 = (local / E.tiles_x) * ch.tile_h;
    // one 8x8 pixel block per wavefront
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int bpr = ch.tile_w >> 3;
    const int px = tx0 + (wave % bpr) * 8 + (lane & 7);
    const int py = ty0 + (wave / bpr) * 8 + (lane >> 3);
    const bool inside = px < E.W && py < E.H;

    const float sub_x = MODE == MODE_SUBPIXEL ? a.sub_x : 0.5f, sub_y = MODE == MODE_SUBPIXEL ? a.sub_y : 0.5f;
    const float X = (2.0f * ((float)px + sub_x) / (float)E.W - 1.0f) * E.tx;
    const float Y = (1.0f - 2.0f * ((float)py + sub_y) / (float)E.H) * E.ty;
    const int64_t pix = E.pix_off + (int64_t)py * E.W + px;

    const int cnt = a.tile_count[tile];
    const bool overflow = cnt > kListCap;
    const int total = overflow ? a.n_views : cnt;
    const EyeView *eve = a.ev + (int64_t)e * a.n_views;
    const uint16_t *tl = a.tile_list + (int64_t)tile * kListCap;

    float accr = 0.0f, accg = 0.0f, accb = 0.0f, ws = 0.0f;
    int nc = 0, nh = 0, n_tests = 0, n_cells = 0;
    for (int base = 0; base < total; base += a.cap) {
        const int nb = min(a.cap, total - base);
        // stage nb EyeView entries (64 B each) as float4 quarters
        for (int q = threadIdx.x; q < nb * 4; q += blockDim.x) {
            const int s = q >> 2;
            const int vid = overflow ? base + s : (int)tl[base + s];
            reinterpret_cast<float4 *>(&sv[s])[q & 3] = reinterpret_cast<const float4 *>(&eve[vid])[q & 3];
        }
        __syncthreads();
        if (inside) {
            for (int c = 0; c < nb; ++c) {
                const EyeView &v = sv[c];
                RayView rv;
                ++n_tests;
                if (!disk_test(v, X, Y, a.R, a.invR, rv)) continue;
                if (MODE == MODE_STATS) ++nc;
                if (MODE == MODE_DEBUG) {
                    if (nc < a.dbg_cap) a.dbg_cand[pix * a.dbg_cap + nc] = v.view;
                    ++nc;
                }
                float wh;
                const void *cells = reinterpret_cast<const char *>(a.geo) +
                                    (int64_t)v.view * a.cells_per_view * (GEO == 0 ? 16 : 8);
                if (!march<GEO>(cells, a.M, a.sM, a.cM, v.wmin, v.wmax, rv.Vx, rv.Vy, rv.Dx, rv.Dy, wh, n_cells))
                    continue;
                if (MODE == MODE_DEBUG) {
                    if (nh < a.dbg_cap) a.dbg_contrib[pix * a.dbg_cap + nh] = v.view;
                    ++nh;
                    continue;
                }
                const float Xs = fmaf(wh, rv.Dx, rv.Vx), Ys = fmaf(wh, rv.Dy, rv.Vy);
                const float tpx = fmaf(Xs, a.sW, a.cW), tpy = fmaf(-Ys, a.sH, a.cH);
                const void *img = reinterpret_cast<const char *>(a.img) +
                                  (int64_t)v.view * a.texels_per_view * (IMG == 0 ? 4 : (IMG == 1 ? 8 : 16));
                const Rgb col = bilinear<IMG>(img, a.img_w, a.img_h, tpx, tpy);
                accr = fmaf(rv.rho, col.r, accr);
                accg = fmaf(rv.rho, col.g, accg);
                accb = fmaf(rv.rho, col.b, accb);
                ws += rv.rho;
                ++nh;
            }
        }
        __syncthreads();
    }
    if (MODE == MODE_STATS) {
        // block-wide sums, one atomic per counter per block
        __shared__ unsigned long long red[5];
        if (threadIdx.x < 5) red[threadIdx.x] = 0ull;
        __syncthreads();
        if (inside) {
            atomicAdd(&red[0], 1ull);
            atomicAdd(&red[1], (unsigned long long)n_tests);
            atomicAdd(&red[2], (unsigned long long)nc);
            atomicAdd(&red[3], (unsigned long long)n_cells);
            atomicAdd(&red[4], (unsigned long long)nh);
        }
        __syncthreads();
        if (threadIdx.x < 5) atomicAdd(&a.stats[threadIdx.x], red[threadIdx.x]);
        return;
    }
    if (!inside) return;
    if (MODE == MODE_DEBUG) {
        for (int s = nc; s < a.dbg_cap; ++s) a.dbg_cand[pix * a.dbg_cap + s] = -1;
        for (int s = nh; s < a.dbg_cap; ++s) a.dbg_contrib[pix * a.dbg_cap + s] = -1;
        if (a.dbg_ncand) a.dbg_ncand[pix] = nc;
        return;
    }
    // second pass of the paper: divide numerator by denominator
    const float k = ws > 0.0f ? texel_scale<IMG>() / ws : 0.0f;
    float r = accr * k, g = accg * k, b = accb * k;
    float *o = a.out_rgb + pix * 3;
    if (MODE == MODE_SUBPIXEL) {
        r *= a.scale;
        g *= a.scale;
        b *= a.scale;
        if (a.accumulate) {
            r += o[0];
            g += o[1];
            b += o[2];
        }
    }
    o[0] = r;
    o[1] = g;
    o[2] = b;
    if (MODE == MODE_RENDER) {
        if (a.out_wsum) a.out_wsum[pix] = ws;
        if (a.out_count) a.out_count[pix] = (uint8_t)min(nh, 255);
    }
}

// ---------------------------------------------------------------------------------------------
// launchers

static int grid_for(int64_t n, int block) {
    int64_t g = (n + block - 1) / block;
    return (int)(g > 65536 * 4 ? 65536 * 4 : (g < 1 ? 1 : g));
}

hipError_t launch_convert_images(const uint8_t *src, void *dst, int img_fmt, int64_t n_texels, hipStream_t s) {
    const int g = grid_for(n_texels, 256);
    if (img_fmt == 1)
        hipLaunchKernelGGL(k_convert_images<1>, dim3(g), dim3(256), 0, s, (const uint32_t *)src, dst, n_texels);
    else
        hipLaunchKernelGGL(k_convert_images<2>, dim3(g), dim3(256), 0, s, (const uint32_t *)src, dst, n_texels);
    return hipGetLastError();
}

hipError_t launch_geo_cells(const float *z, void *cells, int geo_fmt, int32_t n, int32_t M, hipStream_t s) {
    const int g = grid_for((int64_t)(M - 1) * (M - 1) * n, 256);
    if (geo_fmt == 0)
        hipLaunchKernelGGL(k_geo_cells<0>, dim3(g), dim3(256), 0, s, z, cells, n, M);
    else
        hipLaunchKernelGGL(k_geo_cells<1>, dim3(g), dim3(256), 0, s, z, cells, n, M);
    return hipGetLastError();
}

hipError_t launch_geo_range(const void *cells, int geo_fmt, int32_t n, int32_t M, float2 *wr, hipStream_t s) {
    if (geo_fmt == 0)
        hipLaunchKernelGGL(k_geo_range<0>, dim3(n), dim3(256), 0, s, cells, M, wr);
    else
        hipLaunchKernelGGL(k_geo_range<1>, dim3(n), dim3(256), 0, s, cells, M, wr);
    return hipGetLastError();
}

hipError_t launch_prep(const EyeChunk &ch, const double *vt, const float2 *wr, int32_t n, EyeView *ev,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_prep, dim3((n + 255) / 256, ch.n_eyes), dim3(256), 0, s, ch, vt, wr, n, ev);
    return hipGetLastError();
}

hipError_t launch_cull(const EyeChunk &ch, const EyeView *ev, int32_t n, float R_keep, uint16_t *tile_list,
                       int32_t *tile_count, hipStream_t s) {
    hipLaunchKernelGGL(k_cull, dim3((ch.total_tiles + 3) / 4), dim3(256), 0, s, ch, ev, n, R_keep, tile_list,
                       tile_count);
    return hipGetLastError();
}

template <int MODE>
static void launch_render_mode(const EyeChunk &ch, const RenderArgs &a, int img_fmt, int geo_fmt, hipStream_t s) {
    const dim3 grid(ch.total_tiles), block(ch.tile_w * ch.tile_h);
#define LF_R(I, G) hipLaunchKernelGGL((k_render<I, G, MODE>), grid, block, 0, s, ch, a)
    if (geo_fmt == 0) {
        if (img_fmt == 0) LF_R(0, 0);
        else if (img_fmt == 1) LF_R(1, 0);
        else LF_R(2, 0);
    } else {
        if (img_fmt == 0) LF_R(0, 1);
        else if (img_fmt == 1) LF_R(1, 1);
        else LF_R(2, 1);
    }
#undef LF_R
}

hipError_t launch_render(const EyeChunk &ch, const RenderArgs &a, int img_fmt, int geo_fmt, int mode,
                         hipStream_t s) {
    if (mode == MODE_RENDER) launch_render_mode<MODE_RENDER>(ch, a, img_fmt, geo_fmt, s);
    else if (mode == MODE_SUBPIXEL) launch_render_mode<MODE_SUBPIXEL>(ch, a, img_fmt, geo_fmt, s);
    else if (mode == MODE_STATS) launch_render_mode<MODE_STATS>(ch, a, img_fmt, geo_fmt, s);
    else launch_render_mode<MODE_DEBUG>(ch, a, img_fmt, geo_fmt, s);
    return hipGetLastError();
}

}  // namespace lf
