// Host build of the renderer's per-ray arithmetic (lf_ray.h) for CPU tests:
// the same disk test and two-level inverse-depth mesh walk the kernels run,
// evaluated ray by ray on the host. Test support only; not part of liblf.so.
#include <cmath>
#include <cstdint>
#include <algorithm>
#include <cstring>
#include <vector>

#include "lf_ray.h"

using namespace lf;

extern "C" {

// For each ray k and view i: cand[k*n+i] (disk test passed), hit[k*n+i] (mesh
// hit), and the normalised image-plane position (Xs, Ys) of the hit.
// geo_fmt 0 = FP32 cells, 1 = FP16 cells. walk 0: the two-level march over
// the inverse-depth blocks; walk 1: the single walk from the start bound that
// the culling gives a listed view (the largest per-cell bound over the cell
// box of the ray, as a one-ray tile). Returns 0, or 1 for another geo_fmt.
static int trace(int32_t n, int32_t M, const float *z, const double *centres, const double *rot, double src_fov_deg,
                 double R, int32_t geo_fmt, int32_t walk, int64_t n_rays, const double *o, const double *e,
                 int32_t *cand, int32_t *hit, float *Xs, float *Ys, int32_t *cells_visited) {
    if (geo_fmt != 0 && geo_fmt != 1) return 1;  // the trace builds FP32 or FP16 cells only
    const int Mc = M - 1, NB = num_blocks(M);
    const size_t per = (size_t)Mc * Mc;
    std::vector<float4> c32(geo_fmt == 0 ? per * n : 0);
    std::vector<uint2> c16(geo_fmt == 1 ? per * n : 0);
    std::vector<float2> wr(n), blk((size_t)n * NB * NB);
    std::vector<uint16_t> cmax(per * n);
    for (int v = 0; v < n; ++v) {
        const float *zv = z + (size_t)v * M * M;
        for (int k = 0; k < Mc; ++k)
            for (int j = 0; j < Mc; ++j) {
                const float w00 = 1.0f / zv[k * M + j], w10 = 1.0f / zv[k * M + j + 1];
                const float w01 = 1.0f / zv[(k + 1) * M + j], w11 = 1.0f / zv[(k + 1) * M + j + 1];
                const size_t idx = (size_t)v * per + (size_t)k * Mc + j;
                if (geo_fmt == 0) {
                    c32[idx] = make_float4(w00, w10, w01, w11);
                    cmax[idx] = half_up_bits(fmaxf(fmaxf(w00, w10), fmaxf(w01, w11)));
                } else {
                    __half2 a = __floats2half2_rn(w00, w10), b = __floats2half2_rn(w01, w11);
                    uint2 q;
                    std::memcpy(&q.x, &a, 4);
                    std::memcpy(&q.y, &b, 4);
                    c16[idx] = q;
                    const float4 d = load_cell<1>(&c16[idx], 0u);
                    cmax[idx] = half_up_bits(fmaxf(fmaxf(d.x, d.y), fmaxf(d.z, d.w)));
                }
            }
    }
    // the window table: per cell, the largest cell bound over the kWin x kWin cells from it
    std::vector<uint16_t> win(per * n);
    for (int v = 0; v < n; ++v)
        for (int k = 0; k < Mc; ++k)
            for (int j = 0; j < Mc; ++j) {
                uint16_t m = 0;
                for (int kk = k; kk < std::min(k + kWin, Mc); ++kk)
                    for (int jj = j; jj < std::min(j + kWin, Mc); ++jj)
                        m = std::max(m, cmax[(size_t)v * per + (size_t)kk * Mc + jj]);
                win[(size_t)v * per + (size_t)k * Mc + j] = m;
            }
    for (int v = 0; v < n; ++v) {
        float lo = INFINITY, hi = -INFINITY;
        for (int b = 0; b < NB * NB; ++b) {
            const int bk = b / NB, bi = b % NB;
            float blo = INFINITY, bhi = -INFINITY;
            for (int k = bk * kBlk; k < std::min(bk * kBlk + kBlk, Mc); ++k)
                for (int j = bi * kBlk; j < std::min(bi * kBlk + kBlk, Mc); ++j) {
                    const uint32_t idx = (uint32_t)(k * Mc + j);
                    const float4 q = geo_fmt == 0 ? load_cell<0>(c32.data() + (size_t)v * per, idx)
                                                  : load_cell<1>(c16.data() + (size_t)v * per, idx);
                    blo = fminf(blo, fminf(fminf(q.x, q.y), fminf(q.z, q.w)));
                    bhi = fmaxf(bhi, fmaxf(fmaxf(q.x, q.y), fmaxf(q.z, q.w)));
                }
            blk[(size_t)v * NB * NB + b] = make_float2(blo, bhi);
            lo = fminf(lo, blo);
            hi = fmaxf(hi, bhi);
        }
        wr[v] = make_float2(lo, hi);
    }
    const double ts = std::tan(0.5 * src_fov_deg * M_PI / 180.0);
    const float sM = (float)(M / (2.0 * ts)), cM = (float)(0.5 * (M - 1));
    const float invR = (float)(1.0 / R);
    for (int64_t k = 0; k < n_rays; ++k) {
        for (int v = 0; v < n; ++v) {
            const double *c = centres + 3 * v, *Rv = rot + 9 * v;
            EyeView ev;
            std::memset(&ev, 0, sizeof ev);
            // e' = R^T e placed in the third column: the ray is (X, Y) = (0, 0)
            for (int a = 0; a < 3; ++a) {
                double s = 0.0, t = 0.0;
                for (int r = 0; r < 3; ++r) {
                    s += Rv[3 * r + a] * e[3 * k + r];
                    t += Rv[3 * r + a] * (o[3 * k + r] - c[r]);
                }
                ev.m[3 * a + 2] = (float)s;
                ev.o[a] = (float)t;
            }
            ev.wmin = wr[v].x;
            ev.wmax = wr[v].y;
            ev.view = v;
            const size_t out = (size_t)k * n + v;
            RayView rv;
            cand[out] = disk_test(ev, 0.0f, 0.0f, invR, rv) ? 1 : 0;
            hit[out] = 0;
            Xs[out] = Ys[out] = NAN;
            cells_visited[out] = 0;
            if (!cand[out]) continue;
            float wh;
            int nc = 0;
            const float2 *b = blk.data() + (size_t)v * NB * NB;
            const void *cv = geo_fmt == 0 ? (const void *)(c32.data() + (size_t)v * per)
                                          : (const void *)(c16.data() + (size_t)v * per);
            bool h;
            if (walk == 0) {
                h = geo_fmt == 0 ? march<0>(cv, b, M, NB, sM, cM, ev.wmin, ev.wmax, rv.Vx, rv.Vy, rv.Dx, rv.Dy, wh, nc)
                                 : march<1>(cv, b, M, NB, sM, cM, ev.wmin, ev.wmax, rv.Vx, rv.Vy, rv.Dx, rv.Dy, wh, nc);
            } else {
                int4 bx = make_int4(-1, -1, -1, -1);
                if (!tile_cell_box(ev, 0.0f, 0.0f, 0.0f, 0.0f, M, sM, cM, bx.x, bx.y, bx.z, bx.w)) bx.x = -1;
                uint32_t top = 0;
                int nx, ny;
                if (box_windows(bx, nx, ny, top))
                    for (int ty = 0; ty < ny; ++ty)
                        for (int tx = 0; tx < nx; ++tx)
                            top = std::max(top, (uint32_t)win[(size_t)v * per + box_window_index(bx, tx, ty, Mc)]);
                const float wt = half_bits_to_float(top);
                h = geo_fmt == 0
                        ? march_top<0>(cv, M, sM, cM, ev.wmin, ev.wmax, wt, rv.Vx, rv.Vy, rv.Dx, rv.Dy, wh, nc)
                        : march_top<1>(cv, M, sM, cM, ev.wmin, ev.wmax, wt, rv.Vx, rv.Vy, rv.Dx, rv.Dy, wh, nc);
            }
            cells_visited[out] = nc;
            if (!h) continue;
            hit[out] = 1;
            Xs[out] = fmaf(wh, rv.Dx, rv.Vx);
            Ys[out] = fmaf(wh, rv.Dy, rv.Vy);
        }
    }
    return 0;
}

int lfh_trace(int32_t n, int32_t M, const float *z, const double *centres, const double *rot, double src_fov_deg,
              double R, int32_t geo_fmt, int64_t n_rays, const double *o, const double *e, int32_t *cand,
              int32_t *hit, float *Xs, float *Ys, int32_t *cells_visited) {
    return trace(n, M, z, centres, rot, src_fov_deg, R, geo_fmt, 0, n_rays, o, e, cand, hit, Xs, Ys, cells_visited);
}

int lfh_trace_top(int32_t n, int32_t M, const float *z, const double *centres, const double *rot, double src_fov_deg,
                  double R, int32_t geo_fmt, int64_t n_rays, const double *o, const double *e, int32_t *cand,
                  int32_t *hit, float *Xs, float *Ys, int32_t *cells_visited) {
    return trace(n, M, z, centres, rot, src_fov_deg, R, geo_fmt, 1, n_rays, o, e, cand, hit, Xs, Ys, cells_visited);
}

// The cell box of tile_cell_box for one (eye-view frame, rectangle): m, o as
// in an eye-view record, w range [wmin, wmax]; box = (j0, j1, k0, k1).
// Returns 1 with a box, 0 without one.
int lfh_tile_box(const float *m, const float *o, float wmin, float wmax, float X0, float X1, float Y0, float Y1,
                 int32_t M, float sM, float cM, int32_t *box) {
    EyeView ev;
    std::memset(&ev, 0, sizeof ev);
    std::memcpy(ev.m, m, sizeof ev.m);
    std::memcpy(ev.o, o, sizeof ev.o);
    ev.wmin = wmin;
    ev.wmax = wmax;
    return tile_cell_box(ev, X0, X1, Y0, Y1, M, sM, cM, box[0], box[1], box[2], box[3]) ? 1 : 0;
}

// FP16 round-up of the per-cell bounds, for n values.
void lfh_half_up(int64_t n, const float *x, uint16_t *bits) {
    for (int64_t k = 0; k < n; ++k) bits[k] = half_up_bits(x[k]);
}

// Corner inverse depths of cell idx of the view whose cells start at `cells`
// (for the 16-bit codes, 8 bytes after its (base, scale) header).
void lfh_load_cell(int32_t geo_fmt, const void *cells, uint32_t idx, float *out4) {
    const float4 q = geo_fmt == 0 ? load_cell<0>(cells, idx) : geo_fmt == 1 ? load_cell<1>(cells, idx)
                                                                           : load_cell<2>(cells, idx);
    out4[0] = q.x;
    out4[1] = q.y;
    out4[2] = q.z;
    out4[3] = q.w;
}

// The kernels' bilinear sample (clamp-to-edge, texel i's centre at i, result
// in stored texel units) of a W x H image of format img_fmt (0 RGBA8, 1
// RGBA16F, 2 RGBA32F) at (px, py); RGB into rgb3. Returns 0, or 1 for another
// format or an image smaller than 2 x 2.
int lfh_bilinear(int32_t img_fmt, const void *img, int32_t W, int32_t H, float px, float py, float *rgb3) {
    if (W < 2 || H < 2) return 1;
    const float limx = (float)(W - 1), limy = (float)(H - 1);
    Rgb c;
    if (img_fmt == 0)
        c = bilinear<0>(img, W, H, limx, limy, px, py);
    else if (img_fmt == 1)
        c = bilinear<1>(img, W, H, limx, limy, px, py);
    else if (img_fmt == 2)
        c = bilinear<2>(img, W, H, limx, limy, px, py);
    else
        return 1;
    rgb3[0] = c.r;
    rgb3[1] = c.g;
    rgb3[2] = c.b;
    return 0;
}

}  // extern "C"
