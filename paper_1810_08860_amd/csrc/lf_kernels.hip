// HIP kernels for disk-blended light field reconstruction on CDNA4 (gfx950).
//
// Data path for one eye (Sec. 4.1, Eqs. (1)-(2); Sec. 4.2):
//   k_prep    per (eye, view): the 3x3 map taking an eye-image point (X, Y, 1)
//             to the ray direction in the view's frame, and the eye centre in
//             that frame (FP64 set-up, stored FP32).
//   k_cull    per screen tile, one wavefront: every view's disk is tested
//             against the tile's frustum (conservatively); survivors are
//             compacted into an LDS list with a wavefront ballot and prefix
//             popcount, then written out (the GPU counterpart of the paper's
//             per-tile visibility culling, Sec. 4.2.1 and Sec. 7.2).
//   k_render  per screen tile: the tile's candidate list and each candidate's
//             per-view record are wave-uniform and read by the scalar unit;
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
// depth-pixel centres, Sec. 4.5) is the piecewise-linear field of vertex
// inverse depths over the regular grid, and the ray is the straight line
// w -> (V + w D, w). The nearest hit along the ray (intra-image occlusion,
// Sec. 4.2.2) is the LARGEST w at which the line meets the field; the kernel
// walks grid cells from the view's largest inverse depth downwards (blocks of
// cells first, skipping those whose inverse-depth range the line misses) and
// solves, in each cell, the two triangles' planes against the line in closed
// form; the first cell holding a root gives w_hit. (s, t) = V + w_hit D.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <math.h>

#include "lf_internal.h"
#include "lf_ray.h"

namespace lf {

// kernel arguments travel in a 4 KiB segment
static_assert(sizeof(EyeChunk) + sizeof(RenderArgs) <= 4096, "k_render arguments exceed 4 KiB");

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

// YUV420 planes of RGBA8 images (full-range BT.601 in 8-bit fixed point,
// integer arithmetic; arithmetic right shifts floor), one thread per 2x2
// luma block and its chroma sample, the rounded mean of the block's four.
__global__ void k_convert_yuv420(const uint32_t *__restrict__ src, uint8_t *__restrict__ y,
                                 uint8_t *__restrict__ uv, int32_t n, int32_t W, int32_t H) {
    const int Wc = W / 2, Hc = H / 2;
    const int64_t total = (int64_t)n * Wc * Hc;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t v = q / ((int64_t)Wc * Hc);
        const int r = (int)(q % ((int64_t)Wc * Hc));
        const int by = r / Wc, bx = r % Wc;
        int sb = 0, sr = 0;
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                const int64_t p = v * W * H + (int64_t)(2 * by + dy) * W + 2 * bx + dx;
                const uint32_t t = src[p];
                const int R = (int)(t & 255u), G = (int)((t >> 8) & 255u), B = (int)((t >> 16) & 255u);
                y[p] = (uint8_t)((77 * R + 150 * G + 29 * B + 128) >> 8);
                sb += min(((-43 * R - 85 * G + 128 * B + 128) >> 8) + 128, 255);
                sr += min(((128 * R - 107 * G - 21 * B + 128) >> 8) + 128, 255);
            }
        uint8_t *c = uv + 2 * (v * Wc * Hc + (int64_t)by * Wc + bx);
        c[0] = (uint8_t)((sb + 2) >> 2);
        c[1] = (uint8_t)((sr + 2) >> 2);
    }
}

// RGTC1 block of 16 8-bit values (texel t = 4 y + x at src[y * stride +
// x * step]): e0 = maximum, e1 = minimum, a constant block all code 0,
// otherwise each texel the nearest of the eight points, p = round(7 (e0 - x) /
// (e0 - e1)) sevenths from e0 with halves rounded up, coded 0 for p = 0, 1 for
// p = 7 and p + 1 in between (integer arithmetic: any exact implementation
// writes the same bytes).
__device__ uint2 rgtc1_encode(const uint8_t *__restrict__ src, int64_t stride, int step) {
    int v[16], hi = 0, lo = 255;
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        v[t] = src[(t >> 2) * stride + (t & 3) * step];
        hi = max(hi, v[t]);
        lo = min(lo, v[t]);
    }
    uint64_t bits = 0;
    if (hi > lo) {
        const int d = hi - lo;
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            const int p = (14 * (hi - v[t]) + d) / (2 * d);
            const uint64_t code = p == 0 ? 0u : (p == 7 ? 1u : (uint64_t)(p + 1));
            bits |= code << (3 * t);
        }
    }
    const uint64_t word = (uint64_t)hi | ((uint64_t)lo << 8) | (bits << 16);
    return make_uint2((uint32_t)word, (uint32_t)(word >> 32));
}

// RGTC blocks of YUV420 planes: thread q < n (W/4) (H/4) codes one luma
// block, the rest one chroma block each (its Cb block, then its Cr block).
__global__ void k_convert_rgtc(const uint8_t *__restrict__ y, const uint8_t *__restrict__ uv,
                               uint2 *__restrict__ yb, uint4 *__restrict__ uvb, int32_t n, int32_t W, int32_t H) {
    const int Wc = W / 2, Hc = H / 2;
    const int64_t nl = (int64_t)(W / 4) * (H / 4), nc = (int64_t)(Wc / 4) * (Hc / 4);
    const int64_t total = n * (nl + nc);
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
        if (q < n * nl) {
            const int64_t v = q / nl, r = q % nl;
            const int by = (int)(r / (W / 4)), bx = (int)(r % (W / 4));
            yb[q] = rgtc1_encode(y + v * W * H + (int64_t)4 * by * W + 4 * bx, W, 1);
        } else {
            const int64_t qc = q - n * nl;
            const int64_t v = qc / nc, r = qc % nc;
            const int by = (int)(r / (Wc / 4)), bx = (int)(r % (Wc / 4));
            const uint8_t *s0 = uv + 2 * (v * Wc * Hc + (int64_t)4 * by * Wc + 4 * bx);
            const uint2 b0 = rgtc1_encode(s0, 2 * (int64_t)Wc, 2), b1 = rgtc1_encode(s0 + 1, 2 * (int64_t)Wc, 2);
            uvb[qc] = make_uint4(b0.x, b0.y, b1.x, b1.y);
        }
    }
}

// Inverse-depth range (1 / z) of each view's vertices in FP32, before any
// packing: the range the 16-bit codes of LF_GEO_U16 span. One block per view.
__global__ __launch_bounds__(256) void k_z_range(const float *__restrict__ z, int32_t M, float2 *__restrict__ qr) {
    const float *zv = z + (int64_t)blockIdx.x * M * M;
    float lo = INFINITY, hi = -INFINITY;
    for (int q = threadIdx.x; q < M * M; q += blockDim.x) {
        const float w = 1.0f / zv[q];
        lo = fminf(lo, w);
        hi = fmaxf(hi, w);
    }
    __shared__ float slo[256], shi[256];
    slo[threadIdx.x] = lo;
    shi[threadIdx.x] = hi;
    __syncthreads();
    for (int t = 128; t > 0; t >>= 1) {
        if ((int)threadIdx.x < t) {
            slo[threadIdx.x] = fminf(slo[threadIdx.x], slo[threadIdx.x + t]);
            shi[threadIdx.x] = fmaxf(shi[threadIdx.x], shi[threadIdx.x + t]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) qr[blockIdx.x] = make_float2(slo[0], shi[0]);
}

// Mesh cells of every view: corner inverse depths (w00, w10, w01, w11), in
// FP32, FP16 or 16-bit codes over the view's range qr (then each view's
// cells are preceded by its (base, scale)).
template <int GEO>
__global__ void k_geo_cells(const float *__restrict__ z, void *__restrict__ cells, int32_t n, int32_t M,
                            const float2 *__restrict__ qr) {
    const int64_t per = (int64_t)(M - 1) * (M - 1);
    const int64_t total = per * n;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < total;
         c += (int64_t)gridDim.x * blockDim.x) {
        const int64_t v = c / per, r = c % per;
        const int k = (int)(r / (M - 1)), j = (int)(r % (M - 1));
        const float *zv = z + v * (int64_t)M * M;
        const float w00 = 1.0f / zv[(int64_t)k * M + j], w10 = 1.0f / zv[(int64_t)k * M + j + 1];
        const float w01 = 1.0f / zv[(int64_t)(k + 1) * M + j], w11 = 1.0f / zv[(int64_t)(k + 1) * M + j + 1];
        char *view = const_cast<char *>(static_cast<const char *>(geo_view<GEO>(cells, v, per)));
        if (GEO == 0) {
            reinterpret_cast<float4 *>(view)[r] = make_float4(w00, w10, w01, w11);
        } else if (GEO == 1) {
            __half2 a = __floats2half2_rn(w00, w10), b = __floats2half2_rn(w01, w11);
            uint2 o;
            o.x = *reinterpret_cast<uint32_t *>(&a);
            o.y = *reinterpret_cast<uint32_t *>(&b);
            reinterpret_cast<uint2 *>(view)[r] = o;
        } else {
            // code = nearest of base + code * scale, scale = (max - min) / 65535
            const float base = qr[v].x, scale = (qr[v].y - qr[v].x) * (1.0f / 65535.0f);
            const float inv = scale > 0.0f ? 1.0f / scale : 0.0f;
            auto code = [&](float w) { return (uint32_t)fminf(fmaxf(rintf((w - base) * inv), 0.0f), 65535.0f); };
            reinterpret_cast<uint2 *>(view)[r] = make_uint2(code(w00) | (code(w10) << 16), code(w01) | (code(w11) << 16));
            if (r == 0) reinterpret_cast<float2 *>(view)[-1] = make_float2(base, scale);
        }
    }
}

// Inverse-depth range of each view's mesh, from the stored (possibly FP16)
// values the march reads. One block per view.
template <int GEO>
__global__ __launch_bounds__(256) void k_geo_range(const void *__restrict__ cells, int32_t M,
                                                   float2 *__restrict__ wr) {
    const int per = (M - 1) * (M - 1);
    const void *view = geo_view<GEO>(cells, blockIdx.x, per);
    float lo = INFINITY, hi = -INFINITY;
    for (int c = threadIdx.x; c < per; c += blockDim.x) {
        const float4 q = load_cell<GEO>(view, (uint32_t)c);
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

// Min / max inverse depth over the vertices of each kBlk x kBlk block of cells
// of each view (from the stored values). One thread per block.
template <int GEO>
__global__ __launch_bounds__(256) void k_geo_blocks(const void *__restrict__ cells, int32_t n, int32_t M, int32_t NB,
                                                    float2 *__restrict__ blk) {
    const int64_t total = (int64_t)n * NB * NB;
    const int Mc = M - 1;
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < total; b += (int64_t)gridDim.x * blockDim.x) {
        const int64_t v = b / ((int64_t)NB * NB);
        const int r = (int)(b % ((int64_t)NB * NB));
        const int bk = r / NB, bi = r % NB;
        const int j0 = bi * kBlk, j1 = min(j0 + kBlk, Mc), k0 = bk * kBlk, k1 = min(k0 + kBlk, Mc);
        const void *view = geo_view<GEO>(cells, v, (int64_t)Mc * Mc);
        float lo = INFINITY, hi = -INFINITY;
        for (int k = k0; k < k1; ++k)
            for (int j = j0; j < j1; ++j) {
                const float4 q = load_cell<GEO>(view, (uint32_t)(k * Mc + j));
                lo = fminf(lo, fminf(fminf(q.x, q.y), fminf(q.z, q.w)));
                hi = fmaxf(hi, fmaxf(fmaxf(q.x, q.y), fmaxf(q.z, q.w)));
            }
        blk[b] = make_float2(lo, hi);
    }
}

// Per mesh cell (j, k) of each view: the largest inverse depth over the
// corners of the cells [j, j + kWin) x [k, k + kWin) (cut at the grid's
// edge), from the stored values, as FP16 bits rounded up.
template <int GEO>
__global__ __launch_bounds__(256) void k_geo_win(const void *__restrict__ cells, int32_t n, int32_t M,
                                                 uint16_t *__restrict__ win) {
    const int Mc = M - 1;
    const int64_t per = (int64_t)Mc * Mc, total = per * n;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < total; c += (int64_t)gridDim.x * blockDim.x) {
        const int64_t v = c / per;
        const int r = (int)(c % per), k = r / Mc, j = r % Mc;
        const void *view = geo_view<GEO>(cells, v, per);
        float m = 0.0f;
        for (int kk = k; kk < min(k + kWin, Mc); ++kk)
            for (int jj = j; jj < min(j + kWin, Mc); ++jj) {
                const float4 q = load_cell<GEO>(view, (uint32_t)(kk * Mc + jj));
                m = fmaxf(m, fmaxf(fmaxf(q.x, q.y), fmaxf(q.z, q.w)));
            }
        win[c] = half_up_bits(m);
    }
}

// Per (eye, view) frame change, computed in FP64 and stored FP32.
// Can any ray of a plain eye's image rectangle [-tx, tx] x [-ty, ty] cross
// the disk of radius R (view frame: ray direction m (X, Y, 1), eye at o)? The
// tile test of the culling kernel applied to the whole rectangle, in FP64:
// the corner rays of a wide eye can graze a disk plane, where FP32 would lose
// the shape of their quad. Conservative like the tile test, so a view it
// rejects is a candidate for no pixel of the eye.
__device__ bool eye_sees_disk(const double (&m)[9], const double (&o)[3], double R, double tx, double ty) {
    const double cx[4] = {-tx, tx, tx, -tx}, cy[4] = {ty, ty, -ty, -ty};
    double ex[4], ey[4], ez[4], dx[4], dy[4];
    int npos = 0;
    for (int q = 0; q < 4; ++q) {
        ex[q] = m[0] * cx[q] + m[1] * cy[q] + m[2];
        ey[q] = m[3] * cx[q] + m[4] * cy[q] + m[5];
        ez[q] = m[6] * cx[q] + m[7] * cy[q] + m[8];
        npos += ez[q] > 0.0;
        dx[q] = o[0] - o[2] * ex[q] / ez[q];
        dy[q] = o[1] - o[2] * ey[q] / ez[q];
    }
    if (npos == 0) return false;
    if (npos < 4) {
        // the disk's bounding sphere against the four planes of the eye's frustum
        for (int q = 0; q < 4; ++q) {
            const int q1 = (q + 1) & 3, q2 = (q + 2) & 3;
            double nx = ey[q] * ez[q1] - ez[q] * ey[q1];
            double ny = ez[q] * ex[q1] - ex[q] * ez[q1];
            double nz = ex[q] * ey[q1] - ey[q] * ex[q1];
            if (nx * ex[q2] + ny * ey[q2] + nz * ez[q2] < 0.0) {
                nx = -nx;
                ny = -ny;
                nz = -nz;
            }
            const double dist = -(nx * o[0] + ny * o[1] + nz * o[2]);
            if (dist < -R * sqrt(nx * nx + ny * ny + nz * nz)) return false;
        }
        return true;
    }
    // circle against the convex quad of the corner rays' crossings
    bool allp = true, alln = true;
    double best = INFINITY;
    for (int q = 0; q < 4; ++q) {
        const int q1 = (q + 1) & 3;
        const double fx = dx[q1] - dx[q], fy = dy[q1] - dy[q];
        const double cr = fx * (-dy[q]) - fy * (-dx[q]);
        allp = allp && cr >= 0.0;
        alln = alln && cr <= 0.0;
        const double ee = fx * fx + fy * fy;
        double t = ee > 0.0 ? -(dx[q] * fx + dy[q] * fy) / ee : 0.0;
        t = fmin(fmax(t, 0.0), 1.0);
        const double px = dx[q] + t * fx, py = dy[q] + t * fy;
        best = fmin(best, px * px + py * py);
    }
    return allp || alln || best <= R * R;
}

__device__ __forceinline__ EyeView eye_view(const EyeParam &E, const double *__restrict__ vt,
                                            const float2 *__restrict__ wr, int v, const DiskBound &db,
                                            const ViewBases &vb) {
    const double *c = vt + 12 * (int64_t)v;
    const double *R = c + 3;
    EyeView out;
    double md[9], od[3];
    for (int a = 0; a < 3; ++a) {
        for (int b = 0; b < 3; ++b) {
            double s = 0.0;
            for (int r = 0; r < 3; ++r) s += R[3 * r + a] * E.rot[3 * r + b];
            md[3 * a + b] = s;
            out.m[3 * a + b] = (float)s;
        }
        double s = 0.0;
        for (int r = 0; r < 3; ++r) s += R[3 * r + a] * (E.pos[r] - c[r]);
        od[a] = s;
        out.o[a] = (float)s;
    }
    const double oz = od[2];
    const float2 w = wr[v];
    out.wmin = w.x;
    out.wmax = w.y;
    // an eye in front of the view's disk plane (z' = oz > 0 in the view's frame)
    // sees only mesh points beyond its own depth: inverse depth below 1 / oz
    if (oz > 0.0) out.wmax = fminf(out.wmax, (float)(1.0 / oz));
    out.view = v;
    // padded by 1e-4 relative and 1e-7 m: the FP32 tile test may not drop a
    // disk that the exact per-ray test keeps
    out.rk = (float)((db.vrad ? (double)db.vrad[v] * db.vscale : db.R) * (1.0 + 1e-4) + 1e-7);
    if (db.vmask && !db.vmask[v]) out.rk = -1.0f;  // disabled: culled everywhere
    // a view whose disk no ray of a plain eye can cross is culled for that eye
    // (prefilter eyes send their rays off the pixel rectangle: kept)
    if (E.src_view < 0 && out.rk > 0.0f && !eye_sees_disk(md, od, (double)out.rk, E.tx, E.ty)) out.rk = -1.0f;
    out.cells = vb.geo + v * vb.geo_bytes + vb.geo_head;
    out.img = vb.img + v * vb.img_bytes;
    out.blk = vb.blk + v * vb.blk_per_view;
    out.img2 = vb.img2 ? vb.img2 + v * vb.img2_bytes : nullptr;
    return out;
}

// Per eye: the views its eye-level cull keeps (record rk > 0), ascending, so
// the culling kernels test only those. One workgroup per eye; ballot and
// prefix popcount per wave, the four wave counts prefixed across the group.
__global__ __launch_bounds__(256) void k_eye_list(const EyeView *__restrict__ ev, int32_t n,
                                                  uint16_t *__restrict__ elist, int32_t *__restrict__ ecount) {
    __shared__ int wcnt[4];
    const int e = blockIdx.x, wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const EyeView *eve = ev + (int64_t)e * n;
    uint16_t *out = elist + (int64_t)e * n;
    int count = 0;
    for (int base = 0; base < n; base += 256) {
        const int v = base + (int)threadIdx.x;
        const bool keep = v < n && eve[v].rk > 0.0f;
        const uint64_t mask = __ballot(keep);
        if (lane == 0) wcnt[wave] = __popcll(mask);
        __syncthreads();
        int off = count;
        for (int w = 0; w < wave; ++w) off += wcnt[w];
        if (keep) out[off + __popcll(mask & below)] = (uint16_t)v;
        count += wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
        __syncthreads();
    }
    if (threadIdx.x == 0) ecount[e] = count;
}

__global__ __launch_bounds__(256) void k_prep(const EyeChunk ch, const double *__restrict__ vt,
                                              const float2 *__restrict__ wr, int32_t n, const DiskBound db,
                                              const ViewBases vb, EyeView *__restrict__ ev) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    const int e = blockIdx.y;
    if (v >= n || e >= ch.n_eyes) return;
    ev[(int64_t)e * n + v] = eye_view(ch.e[e], vt, wr, v, db, vb);
}

// ---------------------------------------------------------------------------------------------
// culling

// Does any ray of the tile's pixel rectangle [X0,X1] x [Y1,Y0] (corner rays C)
// cross the disk of view v (inside the circle of radius R = v.rk)? Conservative: the tile's rays hit the disk plane
// inside the convex quad spanned by the four corner rays (a central
// projection of a rectangle), so the test is circle-vs-convex-quad; a tile
// that straddles the plane's horizon is kept.
__device__ __forceinline__ bool tile_overlaps_disk(const EyeView &v, const TileCorners &C, float X0, float X1,
                                                   float Y0, float Y1) {
    const float R = v.rk;
    if (!(R > 0.0f)) return false;  // a disabled view
    const float cx[4] = {X0, X1, X1, X0}, cy[4] = {Y0, Y0, Y1, Y1};
    const float(&dx)[4] = C.dx;
    const float(&dy)[4] = C.dy;
    const int npos = C.npos;
    if (npos == 0) return false;
    if (npos < 4) {
        // the tile straddles the disk plane's horizon: test the disk's bounding
        // sphere (centre c, radius R) against the tile's cone of rays instead;
        // in the view's frame the disk centre sits at -o' from the eye
        float ex[4], ey[4], ez[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            ex[q] = fmaf(v.m[0], cx[q], fmaf(v.m[1], cy[q], v.m[2]));
            ey[q] = fmaf(v.m[3], cx[q], fmaf(v.m[4], cy[q], v.m[5]));
            ez[q] = fmaf(v.m[6], cx[q], fmaf(v.m[7], cy[q], v.m[8]));
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int q1 = (q + 1) & 3, q2 = (q + 2) & 3;
            float nx = ey[q] * ez[q1] - ez[q] * ey[q1];
            float ny = ez[q] * ex[q1] - ex[q] * ez[q1];
            float nz = ex[q] * ey[q1] - ey[q] * ex[q1];
            if (nx * ex[q2] + ny * ey[q2] + nz * ez[q2] < 0.0f) {
                nx = -nx;
                ny = -ny;
                nz = -nz;
            }
            const float dist = -(nx * v.o[0] + ny * v.o[1] + nz * v.o[2]);
            if (dist < -R * sqrtf(nx * nx + ny * ny + nz * nz)) return false;
        }
        return true;
    }
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

// Image-plane rectangle [X0,X1] x [Y1,Y0] holding the rays of a prefilter eye
// through the pixels whose plain rectangle is given: pixel (x, y) sends its ray
// to (X - par_u w, Y - par_v w), where (X, Y) is its position shifted by the
// sample offset and w the source mesh's inverse depth there, which the
// inverse-depth blocks of the source view under the shifted rectangle bound.
// False when the shifted rectangle misses the mesh domain (no ray at all).
__device__ __forceinline__ bool prefilter_rect(const EyeParam &E, const CullGeo &g, const float2 *__restrict__ blk,
                                               float &X0, float &X1, float &Y0, float &Y1) {
    X0 = fmaf(E.off_x, E.sx, X0);
    X1 = fmaf(E.off_x, E.sx, X1);
    Y0 = fmaf(-E.off_y, E.sy, Y0);
    Y1 = fmaf(-E.off_y, E.sy, Y1);
    const float lim = (float)(g.M - 1);
    const float gx0 = fmaf(X0, g.sM, g.cM), gx1 = fmaf(X1, g.sM, g.cM);
    const float gy0 = fmaf(-Y0, g.sM, g.cM), gy1 = fmaf(-Y1, g.sM, g.cM);
    if (gx1 < 0.0f || gx0 > lim || gy1 < 0.0f || gy0 > lim) return false;
    const int Mc = g.M - 1;
    const int j0 = min(max((int)floorf(gx0), 0), Mc - 1) / kBlk, j1 = min(max((int)floorf(gx1), 0), Mc - 1) / kBlk;
    const int k0 = min(max((int)floorf(gy0), 0), Mc - 1) / kBlk, k1 = min(max((int)floorf(gy1), 0), Mc - 1) / kBlk;
    float wlo = INFINITY, whi = -INFINITY;
    for (int bk = k0; bk <= k1; ++bk)
        for (int bi = j0; bi <= j1; ++bi) {
            const float2 b = blk[bk * g.NB + bi];
            wlo = fminf(wlo, b.x);
            whi = fmaxf(whi, b.y);
        }
    const float ua = E.par_u * wlo, ub = E.par_u * whi, va = E.par_v * wlo, vb = E.par_v * whi;
    X0 -= fmaxf(ua, ub);
    X1 -= fminf(ua, ub);
    Y0 -= fminf(va, vb);
    Y1 -= fmaxf(va, vb);
    // one part in 1e5 of slack for the FP32 evaluation of the above
    const float sx = 1e-5f * (fabsf(X0) + fabsf(X1)) + 1e-7f, sy = 1e-5f * (fabsf(Y0) + fabsf(Y1)) + 1e-7f;
    X0 -= sx;
    X1 += sx;
    Y0 += sy;
    Y1 -= sy;
    return true;
}

__device__ __forceinline__ int find_eye_super(const EyeChunk &ch, int super) {
    int e = 0;
    while (e + 1 < ch.n_eyes && super >= ch.e[e + 1].super_off) ++e;
    return e;
}

// Culling of one super-tile of kSuper x kSuper screen tiles by one workgroup.
// Phase 1 tests every view against the super-tile's frustum and compacts the
// survivors, in ascending view order, into LDS (per-wave ballot + prefix
// popcount, with a cross-wave prefix of the four wave counts). Phase 2: each
// wavefront takes tiles of the super-tile and tests only the survivors against
// each tile, compacting that tile's list the same way. Lists stay ascending,
// so every pixel later blends its views in the same order whatever the tile
// shape.
struct CullSmem {
    uint16_t slist[kSuperCap];
    uint32_t tlst[4][kListCap];  // view, then view | start bound bits << 16
    int4 tbox[4][kListCap];      // the listed view's cell box (tile_cell_box); x < 0: no box
    int wcnt[4];
};

// Start bounds of the listed views of one tile, by one wavefront: eight lanes
// per listed view (eight views per pass), as 2 rows x 4 columns over the
// windows that cover the view's cell box (box_windows), then the maximum over
// the eight lanes.
// FP16 bits of positive values compare like the values. Entry q of lst
// becomes view | bound << 16.
__device__ __forceinline__ void list_bounds(const CullGeo &g, uint32_t *lst, const int4 *box, int m, int lane) {
    const int Mc = g.M - 1, grp = lane >> 3, sub = lane & 7;
    for (int base = 0; base < m; base += 8) {
        const int q = base + grp;
        uint32_t mx = 0;
        uint32_t v = 0;
        if (q < m) {
            v = lst[q];
            const int4 b = box[q];
            const uint16_t *cw = g.win + (int64_t)v * g.win_per_view;
            int nx, ny;
            if (box_windows(b, nx, ny, mx)) {
                // up to 4 x 4 windows: this lane's (at most two) loads issued together
                const int tx = sub & 3, ty = sub >> 2;
                const bool l0 = tx < nx && ty < ny, l1 = tx < nx && ty + 2 < ny;
                const uint32_t a0 = l0 ? cw[box_window_index(b, tx, ty, Mc)] : 0u;
                const uint32_t a1 = l1 ? cw[box_window_index(b, tx, ty + 2, Mc)] : 0u;
                mx = max(a0, a1);
                // larger boxes: the remaining windows
                if (nx > 4 || ny > 4)
                    for (int yy = ty; yy < ny; yy += 2)
                        for (int xx = tx; xx < nx; xx += 4)
                            if (xx >= 4 || yy >= 4) mx = max(mx, (uint32_t)cw[box_window_index(b, xx, yy, Mc)]);
            }
        }
#pragma unroll
        for (int off = 4; off > 0; off >>= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, off));
        if (q < m && sub == 0) lst[q] = v | (mx << 16);
    }
}

__device__ __forceinline__ void cull_super(const EyeParam &E, int local, int tile_w, int tile_h,
                                           const EyeView *__restrict__ eve, const uint16_t *__restrict__ elist,
                                           int32_t ne, const CullGeo &g, uint32_t *__restrict__ tile_list,
                                           int32_t *__restrict__ tile_count, CullSmem &sm) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int tx0 = (local % E.supers_x) * kSuper, ty0 = (local / E.supers_x) * kSuper;
    const int tx1 = min(tx0 + kSuper, E.tiles_x), ty1 = min(ty0 + kSuper, E.tiles_y);
    const float sxp = E.sx, syp = E.sy;

    const float2 *pblk = E.src_view >= 0 ? eve[E.src_view].blk : nullptr;
    // phase 1: all views against the super-tile
    {
        const int x0 = tx0 * tile_w, x1 = min(tx1 * tile_w, E.W);
        const int y0 = ty0 * tile_h, y1 = min(ty1 * tile_h, E.H);
        float X0 = x0 * sxp - E.tx, X1 = x1 * sxp - E.tx;
        float Y0 = E.ty - y0 * syp, Y1 = E.ty - y1 * syp;
        const bool any = E.src_view < 0 || prefilter_rect(E, g, pblk, X0, X1, Y0, Y1);
        int scount = 0;
        for (int base = 0; base < ne; base += 256) {
            const int q = base + (int)threadIdx.x;
            const int v = q < ne ? (int)elist[q] : 0;
            const bool keep = any && q < ne && tile_overlaps_disk(eve[v], tile_corners(eve[v], X0, X1, Y0, Y1), X0, X1, Y0, Y1);
            const uint64_t mask = __ballot(keep);
            if (lane == 0) sm.wcnt[wave] = __popcll(mask);
            __syncthreads();
            int off = scount;
            for (int w = 0; w < wave; ++w) off += sm.wcnt[w];
            if (keep) {
                const int slot = off + __popcll(mask & below);
                if (slot < kSuperCap) sm.slist[slot] = (uint16_t)v;
            }
            scount += sm.wcnt[0] + sm.wcnt[1] + sm.wcnt[2] + sm.wcnt[3];
            __syncthreads();
        }
        if (threadIdx.x == 0) sm.wcnt[0] = scount;
        __syncthreads();
    }
    const int scount = sm.wcnt[0];
    __syncthreads();
    const bool sover = scount > kSuperCap;
    const int ns = sover ? ne : scount;

    // phase 2: each wavefront tests the survivors against its tiles; with at
    // most 32 survivors a wavefront takes two tiles at once, one per half
    // (lanes 32 h + s test survivor s against tile t0 + h), and each half's
    // list fills its own half of the wave's list space
    const bool pack = !sover && ns <= kListCap / 2;
    const int per = pack ? 2 : 1;
    for (int t0 = wave * per; t0 < kSuper * kSuper; t0 += 4 * per) {
        const int h = pack ? lane >> 5 : 0;
        const int sl = pack ? lane & 31 : lane;
        const uint64_t half = pack ? (h ? 0xffffffff00000000ull : 0x00000000ffffffffull) : ~0ull;
        const int t = t0 + h;
        const int tx = tx0 + t % kSuper, ty = ty0 + t / kSuper;
        const bool active = tx < tx1 && ty < ty1;
        uint32_t *lst = &sm.tlst[wave][pack ? (kListCap / 2) * h : 0];
        int4 *box = &sm.tbox[wave][pack ? (kListCap / 2) * h : 0];
        const int cap = pack ? kListCap / 2 : kListCap;
        int count = 0;
        {
            const int x0 = tx * tile_w, x1 = min(x0 + tile_w, E.W);
            const int y0 = ty * tile_h, y1 = min(y0 + tile_h, E.H);
            float X0 = x0 * sxp - E.tx, X1 = x1 * sxp - E.tx;
            float Y0 = E.ty - y0 * syp, Y1 = E.ty - y1 * syp;
            const bool any = active && (E.src_view < 0 || prefilter_rect(E, g, pblk, X0, X1, Y0, Y1));
            for (int b = 0; b < ns; b += pack ? 32 : 64) {
                const int s = b + sl;
                const int v = any && s < ns ? (int)(sover ? elist[s] : sm.slist[s]) : -1;
                const EyeView &vr = eve[v >= 0 ? v : 0];
                const TileCorners C = tile_corners(vr, X0, X1, Y0, Y1);
                const bool keep = v >= 0 && tile_overlaps_disk(vr, C, X0, X1, Y0, Y1);
                const uint64_t mask = __ballot(keep) & half;
                if (keep) {
                    const int slot = count + __popcll(mask & below);
                    if (slot < cap) {
                        int4 bx = make_int4(-1, -1, -1, -1);
                        if (!tile_cell_box(vr, C, g.M, g.sM, g.cM, bx.x, bx.y, bx.z, bx.w))
                            bx.x = -1;
                        lst[slot] = (uint32_t)v;
                        box[slot] = bx;
                    }
                }
                count += __popcll(mask);
            }
        }
        // the lists are this wave's own: other lanes' LDS writes are visible
        // once they complete, no other wave takes part
        __threadfence_block();
        __builtin_amdgcn_wave_barrier();
        for (int hh = 0; hh < per; ++hh) {
            // tile t0 + hh: its count from a lane of its half
            const int th = t0 + hh;
            const int txh = tx0 + th % kSuper, tyh = ty0 + th / kSuper;
            if (!(txh < tx1 && tyh < ty1)) continue;
            const int ch = __builtin_amdgcn_readlane(count, 32 * hh);
            uint32_t *lh = &sm.tlst[wave][pack ? (kListCap / 2) * hh : 0];
            const int tile = E.tile_off + tyh * E.tiles_x + txh;
            const int m = min(ch, kListCap);
            // each listed view's start bound: the largest cell bound in its box
            // (lists longer than kListCap are never read: those tiles scan every view)
            if (ch <= kListCap) {
                list_bounds(g, lh, &sm.tbox[wave][pack ? (kListCap / 2) * hh : 0], m, lane);
                __threadfence_block();  // the entries written by other lanes are visible below
            }
            for (int q = lane; q < m; q += 64) tile_list[(int64_t)tile * kListCap + q] = lh[q];
            if (lane == 0) tile_count[tile] = ch;
        }
        // every lane has read the lists before the wave's next pass rewrites them
        __threadfence_block();
        __builtin_amdgcn_wave_barrier();
    }
}

__global__ __launch_bounds__(256) void k_cull(const EyeChunk ch, const CullGeo g, const EyeView *__restrict__ ev,
                                              int32_t n, const uint16_t *__restrict__ elist,
                                              const int32_t *__restrict__ ecount, uint32_t *__restrict__ tile_list,
                                              int32_t *__restrict__ tile_count) {
    __shared__ CullSmem sm;
    const int super = blockIdx.x;
    const int e = find_eye_super(ch, super);
    cull_super(ch.e[e], super - ch.e[e].super_off, ch.tile_w, ch.tile_h, ev + (int64_t)e * n, elist + (int64_t)e * n,
               ecount[e], g, tile_list, tile_count, sm);
}

// Eye whose range [off(e), off(e+1)) holds item t, for a device eye table
// sorted by offset (binary search; uniform across the workgroup).
__device__ __forceinline__ int find_eye_sorted(const EyeParam *__restrict__ eyes, int n_eyes, int t, bool super) {
    int lo = 0, hi = n_eyes - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const int off = super ? eyes[mid].super_off : eyes[mid].tile_off;
        if (off <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(256) void k_cull_batch(const BatchArgs b, const CullGeo g,
                                                    const EyeView *__restrict__ ev, int32_t n,
                                                    const uint16_t *__restrict__ elist,
                                                    const int32_t *__restrict__ ecount,
                                                    uint32_t *__restrict__ tile_list,
                                                    int32_t *__restrict__ tile_count) {
    __shared__ CullSmem sm;
    const int super = blockIdx.x;
    const int e = find_eye_sorted(b.eyes, b.n_eyes, super, true);
    const EyeParam E = b.eyes[e];
    cull_super(E, super - E.super_off, b.tile_w, b.tile_h, ev + (int64_t)e * n, elist + (int64_t)e * n, ecount[e],
               g, tile_list, tile_count, sm);
}

// ---------------------------------------------------------------------------------------------
// fused reproject + gather + blend

// Read-only data at a wave-uniform address, fetched by the scalar unit into
// SGPRs (a constant-address-space load). The data must not be written while
// the kernel runs; every table read this way is produced by an earlier kernel.
// Read dword by dword: the scalar unit loads 1, 2, 4, 8 or 16 dwords, and
// adjacent dword loads are merged into those widths.
template <typename T>
__device__ __forceinline__ T uniform_load(const T *p) {
    static_assert(sizeof(T) % 4 == 0 && alignof(T) >= 4, "dword-granular records only");
#if defined(__HIP_DEVICE_COMPILE__)
    union {
        T t;
        uint32_t w[sizeof(T) / 4];
    } u;
    const __attribute__((address_space(4))) uint32_t *q = (const __attribute__((address_space(4))) uint32_t *)p;
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) u.w[i] = q[i];
    return u.t;
#else
    return *p;
#endif
}

// One screen tile of eye E (index e) by one workgroup of tile_w x tile_h
// threads. Each candidate view's record (with the view's data addresses) is
// wave-uniform and lives in SGPRs; a lane holds only its own ray's state.
// DISK: DISK_CIRCLE or DISK_OVAL (the asymmetric disks of Sec. 4.4).
template <int IMG, int GEO, int MODE, int DISK>
__device__ __forceinline__ void render_tile(const EyeParam &E, int e, int tile, int tile_w, int tile_h,
                                            const RenderArgs &a) {
    tile = __builtin_amdgcn_readfirstlane(tile);
    e = __builtin_amdgcn_readfirstlane(e);
    const int local = tile - E.tile_off;
    const int tx0 = (local % E.tiles_x) * tile_w, ty0 = (local / E.tiles_x) * tile_h;
    // one 8x8 pixel block per wavefront
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int bpr = tile_w >> 3;
    const int px = tx0 + (wave % bpr) * 8 + (lane & 7);
    const int py = ty0 + (wave / bpr) * 8 + (lane >> 3);
    const bool inside_img = px < E.W && py < E.H;

    const float sub_x = MODE == MODE_SUBPIXEL ? a.sub_x : (MODE == MODE_PREFILTER ? 0.5f + E.off_x : 0.5f);
    const float sub_y = MODE == MODE_SUBPIXEL ? a.sub_y : (MODE == MODE_PREFILTER ? 0.5f + E.off_y : 0.5f);
    float X = fmaf((float)px + sub_x, E.sx, -E.tx);
    float Y = fmaf(-((float)py + sub_y), E.sy, E.ty);
    const int64_t pix = E.pix_off + (int64_t)py * E.W + px;

    const int cnt = uniform_load(a.tile_count + tile);
    const bool overflow = cnt > a.list_cap;
    const int total = overflow ? a.n_views : cnt;
    const EyeView *eve = a.ev + (int64_t)e * a.n_views;
    bool inside = inside_img;
    if (MODE == MODE_PREFILTER && inside) {
        // the ray leaves the eye (a point of the source view's disk) towards the
        // source mesh point seen at (X, Y): in the eye's image plane that is
        // (X - par_u w, Y - par_v w) with w the mesh's inverse depth there
        float w = 0.0f;
        inside = mesh_point<GEO>(uniform_load(eve + E.src_view).cells, a.M, a.sM, a.cM, X, Y, w);
        X = fmaf(-E.par_u, w, X);
        Y = fmaf(-E.par_v, w, Y);
    }
    const uint32_t *tl = a.tile_list + (int64_t)tile * kListCap;

    float accr = 0.0f, accg = 0.0f, accb = 0.0f, ws = 0.0f;
    int nc = 0, nh = 0, n_tests = 0, n_cells = 0, n_miss = 0;
    if (inside) {
        for (int c = 0; c < total; ++c) {
            int vid = c;
            uint32_t top_bits = 0;
            if (!overflow) {
                const uint32_t entry = uniform_load(tl + c);
                vid = (int)(entry & 0xffffu);
                top_bits = entry >> 16;
            }
            const EyeView v = uniform_load(eve + vid);
            if (overflow && !(v.rk > 0.0f)) continue;  // a disabled view (listed tiles never hold one)
            RayView rv;
            ++n_tests;
            const bool cand = DISK == DISK_OVAL
                                  ? disk_test_oval(v, X, Y, uniform_load(a.ext_inv + v.view), a.ext_inv_scale, rv)
                                  : disk_test(v, X, Y, a.invR, rv);
            if (!cand) continue;
            if (MODE == MODE_STATS) ++nc;
            if (MODE == MODE_DEBUG) {
                if (nc < a.dbg_cap) a.dbg_cand[pix * a.dbg_cap + nc] = v.view;
                ++nc;
            }
            // listed views: one walk from the tile's start bound; a tile that
            // scans every view walks the inverse-depth blocks instead
            float wh;
            const bool hit =
                overflow ? march<GEO>(v.cells, v.blk, a.M, a.NB, a.sM, a.cM, v.wmin, v.wmax, rv.Vx, rv.Vy, rv.Dx, rv.Dy,
                                      wh, n_cells)
                         : march_top<GEO>(v.cells, a.M, a.sM, a.cM, v.wmin, v.wmax, half_bits_to_float(top_bits), rv.Vx,
                                          rv.Vy, rv.Dx, rv.Dy, wh, n_cells);
            if (!hit) continue;
            if (MODE == MODE_DEBUG) {
                if (nh < a.dbg_cap) a.dbg_contrib[pix * a.dbg_cap + nh] = v.view;
                ++nh;
                continue;
            }
            const float Xs = fmaf(wh, rv.Dx, rv.Vx), Ys = fmaf(wh, rv.Dy, rv.Vy);
            const float tpx = fmaf(Xs, a.sW, a.cW), tpy = fmaf(-Ys, a.sH, a.cH);
            if constexpr (MODE == MODE_VISIBILITY) {
                mark_taps(a.vis + (int64_t)v.view * (a.tiles_x * a.tiles_y), a.tiles_x, a.img_w, a.img_h, tpx, tpy);
                continue;
            }
            Rgb col;
            if constexpr (IMG == 5) {
                if (!bilinear_paged(v.img, a.pool, a.tiles_x, a.img_w, a.img_h, tpx, tpy, col)) {
                    ++n_miss;
                    continue;
                }
            } else if constexpr (IMG == 3) {
                col = bilinear_yuv(v.img, v.img2, a.img_w, a.img_h, tpx, tpy);
            } else if constexpr (IMG == 4) {
                col = bilinear_rgtc(v.img, v.img2, a.img_w, a.img_h, tpx, tpy);
            } else {
                col = bilinear<IMG>(v.img, a.img_w, a.img_h, a.img_limx, a.img_limy, tpx, tpy);
            }
            accr = fmaf(rv.rho, col.r, accr);
            accg = fmaf(rv.rho, col.g, accg);
            accb = fmaf(rv.rho, col.b, accb);
            ws += rv.rho;
            ++nh;
        }
    }
    if (IMG == 5 && MODE != MODE_VISIBILITY && n_miss > 0 && a.page_miss) atomicAdd(a.page_miss, (unsigned)n_miss);
    if (MODE == MODE_VISIBILITY) return;
    if (MODE == MODE_PREFILTER) {
        // one sample of Eq. (5): out += w * L, wsum += w where L is defined,
        // w = the sample's rho sigma times the eye's aperture-area factor
        if (inside && ws > 0.0f) {
            const float k = texel_scale<IMG>() * fast_rcp(ws);
            const float sw = a.scale * E.pf_w;
            float *o = a.out_rgb + pix * 3;
            o[0] = fmaf(sw, accr * k, o[0]);
            o[1] = fmaf(sw, accg * k, o[1]);
            o[2] = fmaf(sw, accb * k, o[2]);
            a.out_wsum[pix] += sw;
        }
        return;
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
        __syncthreads();
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
    const float k = ws > 0.0f ? texel_scale<IMG>() * fast_rcp(ws) : 0.0f;
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

template <int IMG, int GEO, int MODE, int DISK>
__global__ __launch_bounds__(256) void k_render(const EyeChunk ch, const RenderArgs a) {
    const int tile = blockIdx.x;
    const int e = find_eye(ch, tile);
    render_tile<IMG, GEO, MODE, DISK>(ch.e[e], e, tile, ch.tile_w, ch.tile_h, a);
}

// Next tile of a persistent workgroup. Each eye's tile rows are cut into
// kXcds bands; the queue of XCD x (its own counter, on its own 128-byte line)
// holds one band of every eye in turn: band (x + e / 2) mod kXcds of eye e,
// so both eyes of a stereo pair give XCD x the same band and over every
// kXcds poses each XCD takes every band once (the queues cost the same and
// move through the eyes together: short frame spans). Work-group ids are
// dispatched round-robin over the XCDs, so workgroup b runs on XCD b % kXcds
// and drains that queue: each XCD works on neighbouring tiles of its current
// band, whose source texels its L2 then holds, instead of every XCD fetching
// every part of every eye into its own L2. A workgroup whose queue is empty
// takes slots from the other queues in turn (load balance). `probe` counts
// the queues found empty; once all are, the result is total_tiles (the exit).
__device__ __forceinline__ int next_tile(const BatchArgs &b, int home, int &probe) {
    while (probe < kXcds) {
        const int q = (home + probe) % kXcds;
        const int t = (int)atomicAdd(b.queue + q * kQueueStride, 1u);
        if (t < b.q_len[q]) {
            // the last eye whose band in queue q starts at or before slot t
            int lo = 0, hi = b.n_eyes - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (b.eyes[mid].band_off[q] <= t) lo = mid;
                else hi = mid - 1;
            }
            const EyeParam *E = b.eyes + lo;
            const int band = (q + lo / 2) % kXcds;
            return E->tile_off + (band * E->tiles_y) / kXcds * E->tiles_x + (t - E->band_off[q]);
        }
        ++probe;
    }
    return b.total_tiles;
}

// Persistent form for batches: a grid sized to the machine; each workgroup
// takes tiles from the queues above (all eyes of the batch, any sizes) until
// every queue is empty -- each workgroup reaches the exit after at most
// kXcds probes of empty queues. Per eye, the earliest start and latest end
// wall-clock stamps of its tiles are kept (per-frame latency).
// Seven waves per SIMD: the register budget that leaves room for a small
// spill but hides more of the mesh walk's load latency than the default five.
template <int IMG, int GEO, int DISK>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(7, 7))) void
k_render_persistent(const BatchArgs b, const RenderArgs a) {
    __shared__ int s_tile;
    const int home = blockIdx.x % kXcds;
    int probe = 0;  // used by thread 0 only
    if (threadIdx.x == 0) s_tile = next_tile(b, home, probe);
    __syncthreads();
    int tile = s_tile;
    int cur_e = -1, lo = 0, hi = 0;  // tiles [lo, hi) belong to eye cur_e
    EyeParam E;
    unsigned long long t0 = 0, t1 = 0;
    while (tile < b.total_tiles) {
        __syncthreads();  // every thread has read s_tile
        // fetch the next tile now; the atomic's round trip overlaps this tile's work
        if (threadIdx.x == 0) s_tile = next_tile(b, home, probe);
        if (tile < lo || tile >= hi) {
            const int e = find_eye_sorted(b.eyes, b.n_eyes, tile, false);
            if (threadIdx.x == 0) {
                if (cur_e >= 0 && b.frame_t) {
                    atomicMin(&b.frame_t[2 * cur_e], t0);
                    atomicMax(&b.frame_t[2 * cur_e + 1], t1);
                }
                t0 = wall_clock64();
            }
            E = uniform_load(b.eyes + e);
            cur_e = e;
            lo = E.tile_off;
            hi = lo + E.tiles_x * E.tiles_y;
        }
        render_tile<IMG, GEO, MODE_RENDER, DISK>(E, cur_e, tile, b.tile_w, b.tile_h, a);
        if (threadIdx.x == 0) t1 = wall_clock64();
        __syncthreads();  // the prefetched index is visible
        tile = s_tile;
    }
    if (threadIdx.x == 0 && cur_e >= 0 && b.frame_t) {
        atomicMin(&b.frame_t[2 * cur_e], t0);
        atomicMax(&b.frame_t[2 * cur_e + 1], t1);
    }
}

// Start-of-batch reset: empty queues, per-eye stamps at (max, 0). A kernel
// (not a memset) so the batch graph holds kernels only.
__global__ void k_batch_reset(unsigned int *queue, unsigned long long *frame_t, int n_eyes) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kXcds) queue[i * kQueueStride] = 0u;
    if (frame_t && i < n_eyes) {
        frame_t[2 * i] = ~0ull;
        frame_t[2 * i + 1] = 0ull;
    }
}

// Per (eye, view) set-up for a batch whose eye table lives in device memory.
__global__ __launch_bounds__(256) void k_prep_batch(const BatchArgs b, const double *__restrict__ vt,
                                                    const float2 *__restrict__ wr, int32_t n, const DiskBound db,
                                                    const ViewBases vb, EyeView *__restrict__ ev) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    const int e = blockIdx.y;
    if (v >= n || e >= b.n_eyes) return;
    const EyeParam E = b.eyes[e];
    ev[(int64_t)e * n + v] = eye_view(E, vt, wr, v, db, vb);
}

// Prefilter finish (Eq. (5)): divide the weighted colour sums by the weight sums.
__global__ void k_prefilter_finish(float *__restrict__ out, const float *__restrict__ wsum, int64_t n) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        const float w = wsum[p];
        const float k = w != 0.0f ? 1.0f / w : 0.0f;
        out[3 * p] *= k;
        out[3 * p + 1] *= k;
        out[3 * p + 2] *= k;
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

hipError_t launch_convert_yuv420(const uint8_t *src, uint8_t *y, uint8_t *uv, int32_t n, int32_t W, int32_t H,
                                 hipStream_t s) {
    const int g = grid_for((int64_t)n * (W / 2) * (H / 2), 256);
    hipLaunchKernelGGL(k_convert_yuv420, dim3(g), dim3(256), 0, s, (const uint32_t *)src, y, uv, n, W, H);
    return hipGetLastError();
}

hipError_t launch_convert_rgtc(const uint8_t *y, const uint8_t *uv, void *yb, void *uvb, int32_t n, int32_t W,
                               int32_t H, hipStream_t s) {
    const int64_t blocks = (int64_t)n * ((int64_t)(W / 4) * (H / 4) + (int64_t)(W / 8) * (H / 8));
    const int g = grid_for(blocks, 256);
    hipLaunchKernelGGL(k_convert_rgtc, dim3(g), dim3(256), 0, s, y, uv, (uint2 *)yb, (uint4 *)uvb, n, W, H);
    return hipGetLastError();
}

// RGBA8 images to kPage x kPage tiles: one workgroup per tile row of kPage texels (uint4 = 4 texels)
__global__ void k_tile_images(const uint4 *__restrict__ src, uint4 *__restrict__ dst, int32_t n, int32_t W, int32_t H) {
    const int tx = W / kPage, ty = H / kPage;
    const int64_t rows = (int64_t)n * H;  // one source row per (view, y)
    constexpr int q = kPage / 4;          // uint4 per tile row
    for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
        const int64_t v = r / H;
        const int y = (int)(r % H);
        for (int k = threadIdx.x; k < W / 4; k += blockDim.x) {
            const int x4 = k * 4;
            const int64_t tile = (v * ty + (y >> kPageShift)) * tx + (x4 >> kPageShift);
            dst[tile * (kPage * q) + (y & (kPage - 1)) * q + ((x4 & (kPage - 1)) >> 2)] = src[r * (W / 4) + k];
        }
    }
}

hipError_t launch_tile_images(const uint32_t *src, uint32_t *dst, int32_t n, int32_t W, int32_t H, hipStream_t s) {
    const int g = (int)std::min<int64_t>((int64_t)n * H, 65536);
    hipLaunchKernelGGL(k_tile_images, dim3(g), dim3(256), 0, s, (const uint4 *)src, (uint4 *)dst, n, W, H);
    return hipGetLastError();
}

// Tile cache update: workgroup 0 patches the page table; workgroup 1 + k
// copies staged tile k into its page (16 KB: 1024 uint4, 4 per thread).
__global__ void k_cache_apply(int32_t *__restrict__ pt, const int2 *__restrict__ patch, int32_t n_patch,
                              const uint4 *__restrict__ staged, const int32_t *__restrict__ slot, char *__restrict__ pool) {
    if (blockIdx.x == 0) {
        for (int k = threadIdx.x; k < n_patch; k += blockDim.x) pt[patch[k].x] = patch[k].y;
        return;
    }
    const int k = blockIdx.x - 1;
    constexpr int per = kPage * kPage * 4 / 16;
    uint4 *dst = reinterpret_cast<uint4 *>(pool + (int64_t)slot[k] * (kPage * kPage * 4));
    const uint4 *src = staged + (int64_t)k * per;
    for (int i = threadIdx.x; i < per; i += blockDim.x) dst[i] = src[i];
}

// Keys of the set bytes of vis[0, n) (the visible tiles of a visibility
// pass), in no particular order: one atomic per wavefront reserves the slots
// of its set lanes. keys holds room for n entries; *count starts at 0.
__global__ void k_vis_compact(const uint8_t *__restrict__ vis, int64_t n, int32_t *__restrict__ keys,
                              unsigned int *__restrict__ count) {
    const int lane = threadIdx.x & 63;
    const uint64_t below = (1ull << lane) - 1ull;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n; base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = base + threadIdx.x;
        const bool set = i < n && vis[i] != 0;
        const uint64_t mask = __ballot(set);
        unsigned int first = 0;
        if (lane == 0 && mask) first = atomicAdd(count, (unsigned int)__popcll(mask));
        first = __shfl(first, 0);
        if (set) keys[first + __popcll(mask & below)] = (int32_t)i;
    }
}

hipError_t launch_vis_compact(const uint8_t *vis, int64_t n, int32_t *keys, unsigned int *count, hipStream_t s) {
    const int g = (int)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_vis_compact, dim3(g), dim3(256), 0, s, vis, n, keys, count);
    return hipGetLastError();
}

hipError_t launch_cache_apply(int32_t *pt, const int2 *patch, int32_t n_patch, const uint4 *staged,
                              const int32_t *slot, int32_t n_tiles, char *pool, hipStream_t s) {
    hipLaunchKernelGGL(k_cache_apply, dim3(1 + n_tiles), dim3(256), 0, s, pt, patch, n_patch, staged, slot, pool);
    return hipGetLastError();
}

hipError_t launch_geo_cells(const float *z, void *cells, int geo_fmt, int32_t n, int32_t M, float2 *qr,
                            hipStream_t s) {
    const int g = grid_for((int64_t)(M - 1) * (M - 1) * n, 256);
    if (geo_fmt == 0) {
        hipLaunchKernelGGL(k_geo_cells<0>, dim3(g), dim3(256), 0, s, z, cells, n, M, qr);
    } else if (geo_fmt == 1) {
        hipLaunchKernelGGL(k_geo_cells<1>, dim3(g), dim3(256), 0, s, z, cells, n, M, qr);
    } else {
        hipLaunchKernelGGL(k_z_range, dim3(n), dim3(256), 0, s, z, M, qr);
        hipLaunchKernelGGL(k_geo_cells<2>, dim3(g), dim3(256), 0, s, z, cells, n, M, qr);
    }
    return hipGetLastError();
}

#define LF_GEO3(K, ...)                                                 \
    do {                                                                \
        if (geo_fmt == 0) hipLaunchKernelGGL(K<0>, __VA_ARGS__);        \
        else if (geo_fmt == 1) hipLaunchKernelGGL(K<1>, __VA_ARGS__);   \
        else hipLaunchKernelGGL(K<2>, __VA_ARGS__);                     \
    } while (0)

hipError_t launch_geo_range(const void *cells, int geo_fmt, int32_t n, int32_t M, float2 *wr, hipStream_t s) {
    LF_GEO3(k_geo_range, dim3(n), dim3(256), 0, s, cells, M, wr);
    return hipGetLastError();
}

hipError_t launch_geo_blocks(const void *cells, int geo_fmt, int32_t n, int32_t M, float2 *blk, hipStream_t s) {
    const int NB = num_blocks(M);
    const int g = grid_for((int64_t)n * NB * NB, 256);
    LF_GEO3(k_geo_blocks, dim3(g), dim3(256), 0, s, cells, n, M, NB, blk);
    return hipGetLastError();
}

hipError_t launch_geo_win(const void *cells, int geo_fmt, int32_t n, int32_t M, uint16_t *win, hipStream_t s) {
    const int g = grid_for((int64_t)n * (M - 1) * (M - 1), 256);
    LF_GEO3(k_geo_win, dim3(g), dim3(256), 0, s, cells, n, M, win);
    return hipGetLastError();
}
#undef LF_GEO3

hipError_t launch_prep(const EyeChunk &ch, const double *vt, const float2 *wr, int32_t n, const DiskBound &db,
                       const ViewBases &vb, EyeView *ev, hipStream_t s) {
    hipLaunchKernelGGL(k_prep, dim3((n + 255) / 256, ch.n_eyes), dim3(256), 0, s, ch, vt, wr, n, db, vb, ev);
    return hipGetLastError();
}

hipError_t launch_cull(const EyeChunk &ch, const CullGeo &g, const EyeView *ev, int32_t n, uint16_t *elist,
                       int32_t *ecount, uint32_t *tile_list, int32_t *tile_count, hipStream_t s) {
    hipLaunchKernelGGL(k_eye_list, dim3(ch.n_eyes), dim3(256), 0, s, ev, n, elist, ecount);
    hipLaunchKernelGGL(k_cull, dim3(ch.total_supers), dim3(256), 0, s, ch, g, ev, n, elist, ecount, tile_list,
                       tile_count);
    return hipGetLastError();
}

template <int MODE, int DISK>
static void launch_render_mode(const EyeChunk &ch, const RenderArgs &a, int img_fmt, int geo_fmt, hipStream_t s) {
    const dim3 grid(ch.total_tiles), block(ch.tile_w * ch.tile_h);
#define LF_R(I, G) hipLaunchKernelGGL((k_render<I, G, MODE, DISK>), grid, block, 0, s, ch, a)
#define LF_RG(G)                          \
    do {                                  \
        if (img_fmt == 0) LF_R(0, G);     \
        else if (img_fmt == 1) LF_R(1, G); \
        else if (img_fmt == 2) LF_R(2, G); \
        else if (img_fmt == 3) LF_R(3, G); \
        else if (img_fmt == 4) LF_R(4, G); \
        else LF_R(5, G);                  \
    } while (0)
    if (geo_fmt == 0) LF_RG(0);
    else if (geo_fmt == 1) LF_RG(1);
    else LF_RG(2);
#undef LF_RG
#undef LF_R
}

// the visibility pass exists for paged images only
static void launch_visibility(const EyeChunk &ch, const RenderArgs &a, int geo_fmt, hipStream_t s) {
    const dim3 grid(ch.total_tiles), block(ch.tile_w * ch.tile_h);
#define LF_V(G, D) hipLaunchKernelGGL((k_render<5, G, MODE_VISIBILITY, D>), grid, block, 0, s, ch, a)
    if (a.ext_inv) {
        if (geo_fmt == 0) LF_V(0, DISK_OVAL);
        else if (geo_fmt == 1) LF_V(1, DISK_OVAL);
        else LF_V(2, DISK_OVAL);
    } else {
        if (geo_fmt == 0) LF_V(0, DISK_CIRCLE);
        else if (geo_fmt == 1) LF_V(1, DISK_CIRCLE);
        else LF_V(2, DISK_CIRCLE);
    }
#undef LF_V
}

template <int MODE>
static void launch_render_disk(const EyeChunk &ch, const RenderArgs &a, int img_fmt, int geo_fmt, hipStream_t s) {
    if (a.ext_inv) launch_render_mode<MODE, DISK_OVAL>(ch, a, img_fmt, geo_fmt, s);
    else launch_render_mode<MODE, DISK_CIRCLE>(ch, a, img_fmt, geo_fmt, s);
}

template <int DISK>
static void launch_persistent(const BatchArgs &b, const RenderArgs &a, int img_fmt, int geo_fmt, int grid,
                              hipStream_t s) {
    const dim3 block(b.tile_w * b.tile_h);
#define LF_P(I, G) hipLaunchKernelGGL((k_render_persistent<I, G, DISK>), dim3(grid), block, 0, s, b, a)
#define LF_PG(G)                          \
    do {                                  \
        if (img_fmt == 0) LF_P(0, G);     \
        else if (img_fmt == 1) LF_P(1, G); \
        else if (img_fmt == 2) LF_P(2, G); \
        else if (img_fmt == 3) LF_P(3, G); \
        else if (img_fmt == 4) LF_P(4, G); \
        else LF_P(5, G);                  \
    } while (0)
    if (geo_fmt == 0) LF_PG(0);
    else if (geo_fmt == 1) LF_PG(1);
    else LF_PG(2);
#undef LF_PG
#undef LF_P
}

hipError_t launch_batch(const BatchArgs &b, const RenderArgs &a, const double *vt, const float2 *wr, int32_t n,
                        const DiskBound &db, const ViewBases &vb, const CullGeo &g, uint16_t *elist, int32_t *ecount,
                        int img_fmt, int geo_fmt, int grid, hipStream_t s, hipEvent_t ev_a, hipEvent_t ev_b) {
    hipLaunchKernelGGL(k_batch_reset, dim3((b.n_eyes + 255) / 256), dim3(256), 0, s, b.queue, b.frame_t, b.n_eyes);
    hipLaunchKernelGGL(k_prep_batch, dim3((n + 255) / 256, b.n_eyes), dim3(256), 0, s, b, vt, wr, n, db, vb,
                       const_cast<EyeView *>(a.ev));
    hipLaunchKernelGGL(k_eye_list, dim3(b.n_eyes), dim3(256), 0, s, a.ev, n, elist, ecount);
    hipLaunchKernelGGL(k_cull_batch, dim3(b.total_supers), dim3(256), 0, s, b, g, a.ev, n, elist, ecount,
                       const_cast<uint32_t *>(a.tile_list), const_cast<int32_t *>(a.tile_count));
    if (ev_a) {
        hipError_t e = hipEventRecordWithFlags(ev_a, s, hipEventRecordExternal);
        if (e != hipSuccess) return e;
    }
    if (a.ext_inv) launch_persistent<DISK_OVAL>(b, a, img_fmt, geo_fmt, grid, s);
    else launch_persistent<DISK_CIRCLE>(b, a, img_fmt, geo_fmt, grid, s);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && ev_b) e = hipEventRecordWithFlags(ev_b, s, hipEventRecordExternal);
    return e;
}

template <int DISK>
static const void *persistent_fn(int img_fmt, int geo_fmt) {
    const void *f0[6] = {(const void *)k_render_persistent<0, 0, DISK>, (const void *)k_render_persistent<1, 0, DISK>,
                         (const void *)k_render_persistent<2, 0, DISK>, (const void *)k_render_persistent<3, 0, DISK>,
                         (const void *)k_render_persistent<4, 0, DISK>, (const void *)k_render_persistent<5, 0, DISK>};
    const void *f1[6] = {(const void *)k_render_persistent<0, 1, DISK>, (const void *)k_render_persistent<1, 1, DISK>,
                         (const void *)k_render_persistent<2, 1, DISK>, (const void *)k_render_persistent<3, 1, DISK>,
                         (const void *)k_render_persistent<4, 1, DISK>, (const void *)k_render_persistent<5, 1, DISK>};
    const void *f2[6] = {(const void *)k_render_persistent<0, 2, DISK>, (const void *)k_render_persistent<1, 2, DISK>,
                         (const void *)k_render_persistent<2, 2, DISK>, (const void *)k_render_persistent<3, 2, DISK>,
                         (const void *)k_render_persistent<4, 2, DISK>, (const void *)k_render_persistent<5, 2, DISK>};
    return geo_fmt == 0 ? f0[img_fmt] : geo_fmt == 1 ? f1[img_fmt] : f2[img_fmt];
}

hipError_t persistent_occupancy(int img_fmt, int geo_fmt, bool oval, int block, int *per_cu) {
    const void *f = oval ? persistent_fn<DISK_OVAL>(img_fmt, geo_fmt) : persistent_fn<DISK_CIRCLE>(img_fmt, geo_fmt);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, f, block, 0);
}

hipError_t launch_prefilter_finish(float *out_rgb, const float *wsum, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_prefilter_finish, dim3(grid_for(n, 256)), dim3(256), 0, s, out_rgb, wsum, n);
    return hipGetLastError();
}

hipError_t launch_render(const EyeChunk &ch, const RenderArgs &a, int img_fmt, int geo_fmt, int mode,
                         hipStream_t s) {
    if (mode == MODE_RENDER) launch_render_disk<MODE_RENDER>(ch, a, img_fmt, geo_fmt, s);
    else if (mode == MODE_SUBPIXEL) launch_render_disk<MODE_SUBPIXEL>(ch, a, img_fmt, geo_fmt, s);
    else if (mode == MODE_STATS) launch_render_disk<MODE_STATS>(ch, a, img_fmt, geo_fmt, s);
    else if (mode == MODE_PREFILTER) launch_render_disk<MODE_PREFILTER>(ch, a, img_fmt, geo_fmt, s);
    else if (mode == MODE_VISIBILITY) launch_visibility(ch, a, geo_fmt, s);
    else launch_render_disk<MODE_DEBUG>(ch, a, img_fmt, geo_fmt, s);
    return hipGetLastError();
}

}  // namespace lf
