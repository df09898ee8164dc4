/*
 * FP64 CPU oracle for disk-blended light field reconstruction.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the slow, plain reference that the
 * GPU path is checked against. Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it. It shares no code, header,
 * table or helper with the HIP library; the only thing both consume is the
 * synthetic input data written by the seeded generator.
 *
 * What it computes (paper, Sec. 4.1, Eqs. (1)-(2)): for an eye ray (o, e)
 *
 *     L(o, e) = sum_i I_i(s_i, t_i) rho_i(u_i, v_i) / sum_i rho_i(u_i, v_i)
 *
 * where (u_i, v_i) is where the ray crosses view i's disk (centred on the
 * view's centre of projection, tangent to the capture sphere, normal along the
 * optical axis, u and v along the image axes: Sec. 4.1 and Sec. 4.4), rho_i is
 * the linear-falloff kernel (1 at the centre, 0 at the rim: Sec. 4.1), and
 * (s_i, t_i) is the image-i position of the nearest intersection of the ray
 * with view i's own triangle mesh (Sec. 4.1; intra-image occlusion only,
 * Sec. 4.2.2; the mesh is the depth map tessellated with two triangles per
 * depth pixel, Sec. 4.5). Pass 1 / pass 2 of Sec. 4.2 (accumulate numerator and
 * denominator, then divide) become two running sums and one division.
 *
 * The prefilter of Sec. 5 (Eqs. (4)-(5)) is built on the same query: see
 * orc_prefilter below.
 *
 * The geometry is deliberately evaluated in WORLD space with the published
 * watertight ray/triangle test (Woop, Benthin & Wald 2013), over either all
 * triangles ("brute") or the cells visited by an Amanatides-Woo 2-D grid walk
 * (Amanatides & Woo 1987) dilated by one cell ("traversal"); the nearest hit
 * is the minimum t over every triangle tested, with no early exit.
 *
 * Readings of points the paper leaves open (each also listed in the design
 * notes of the repository):
 *   - disk: a planar circle of radius R in the tangent plane at c_i, normal f_i;
 *     rho = 1 - r/R, a candidate iff rho > 0; a ray with e.f_i <= 0 never uses
 *     view i (back-facing disk);
 *   - asymmetric oval disk (Sec. 4.4, "Disk Shape"), when per-view extents
 *     (e+u, e-u, e+v, e-v) are given: the union of four elliptic quarters, one
 *     per quadrant of the disk plane around c_i; the linear falloff runs in the
 *     quadrant's normalised radius, rho = 1 - sqrt((u/e_u)^2 + (v/e_v)^2) with
 *     e_u = e+u for u >= 0 else e-u and e_v likewise;
 *   - mesh: vertices at depth-pixel centres, V_jk = c_i + z_jk R_i (X_j, Y_k, 1),
 *     cell (j,k) split along (j,k)-(j+1,k+1); both faces count; barycentric
 *     tests inclusive;
 *   - (s,t): exact projection of the 3-D hit into view i;
 *   - a view whose mesh the ray misses adds nothing to either sum; if both sums
 *     are empty the pixel is (0,0,0);
 *   - sampling: bilinear, texel centres at half-integers, clamp-to-edge, RGB of
 *     the RGBA8 texel divided by 255, alpha ignored.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t n, img_w, img_h, mesh_m;
    double src_fov_deg;
    const double *centres;   /* [n][3] world metres */
    const double *rot;       /* [n][9] row-major, columns (r,u,f) */
    const uint8_t *rgba8;    /* [n][img_h][img_w][4] */
    const float *zdepth;     /* [n][mesh_m][mesh_m] z along f, metres */
    const double *zrange;    /* [n][2] min,max of each depth map (orc_zrange) */
    double disk_radius;
    const double *disk_ext;  /* [n][4] oval extents e+u, e-u, e+v, e-v (metres), or NULL: circles of disk_radius */
    int32_t mode;            /* 0 = traversal, 1 = brute force over all triangles */
    int32_t threads;
    const uint8_t *yuv_y;    /* [n][img_h][img_w] luma, or NULL: sample rgba8 */
    const uint8_t *yuv_uv;   /* [n][img_h/2][img_w/2][2] chroma (Cb, Cr) at half resolution */
    const uint8_t *rgtc_y;   /* [n][img_h/4][img_w/4][8] luma as RGTC1 blocks, or NULL: sample yuv_y / rgba8 */
    const uint8_t *rgtc_uv;  /* [n][img_h/8][img_w/8][16] chroma as RGTC2 blocks (Cb block, then Cr block) */
    const uint8_t *resident; /* [n][img_h/page][img_w/page] 1 = image tile in the tile cache, or NULL: all */
    int32_t page;            /* image tile size in texels (with resident) */
} orc_views;

/* Per-ray outputs. Lists are ascending view ids padded with -1. */
typedef struct {
    int32_t cap;             /* capacity of each list (0 = no lists) */
    int32_t *cand;           /* [n_rays][cap] views with rho > 0 */
    int32_t *cand_band;      /* [n_rays][cap] views whose disk decision is ill-conditioned */
    int32_t *contrib;        /* [n_rays][cap] candidates whose mesh is hit */
    int32_t *contrib_band;   /* [n_rays][cap] contributing or not, hit/miss ill-conditioned */
    int32_t *n_cand;         /* [n_rays] number of candidates (even beyond cap) */
} orc_lists;

static inline double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static inline void cross3(const double a[3], const double b[3], double o[3]) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
static inline void sub3(const double a[3], const double b[3], double o[3]) { o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2]; }
/* column a of a row-major frame */
static inline void col3(const double *R, int a, double o[3]) { o[0] = R[a]; o[1] = R[3 + a]; o[2] = R[6 + a]; }
/* R^T x  (world vector -> view-local components along r, u, f) */
static inline void to_local(const double *R, const double x[3], double o[3]) {
    o[0] = R[0] * x[0] + R[3] * x[1] + R[6] * x[2];
    o[1] = R[1] * x[0] + R[4] * x[1] + R[7] * x[2];
    o[2] = R[2] * x[0] + R[5] * x[1] + R[8] * x[2];
}

/* Exact min / max of each depth map (the mesh cannot leave this z range). */
void orc_zrange(int32_t n, int32_t m, const float *z, double *out) {
    for (int32_t i = 0; i < n; ++i) {
        const float *zi = z + (int64_t)i * m * m;
        double lo = INFINITY, hi = -INFINITY;
        for (int64_t k = 0; k < (int64_t)m * m; ++k) {
            if (zi[k] < lo) lo = zi[k];
            if (zi[k] > hi) hi = zi[k];
        }
        out[2 * i] = lo;
        out[2 * i + 1] = hi;
    }
}

/*
 * Eye rays (Sec. 4.1, Eq. (1)): origin o = eye centre, direction through the
 * continuous pixel position (x, y), where pixel (px, py) has its centre at
 * (px + 1/2, py + 1/2). The FOV is horizontal; the vertical half-angle follows
 * from the aspect ratio (square pixels).
 */
void orc_eye_rays(const double pos[3], const double *rot, double hfov_deg, int32_t W, int32_t H,
                  int64_t n, const double *pxy, double *o, double *e) {
    double tx = tan(0.5 * hfov_deg * M_PI / 180.0), ty = tx * (double)H / (double)W;
    for (int64_t k = 0; k < n; ++k) {
        double X = (2.0 * pxy[2 * k] / W - 1.0) * tx;
        double Y = (1.0 - 2.0 * pxy[2 * k + 1] / H) * ty;
        for (int a = 0; a < 3; ++a) {
            o[3 * k + a] = pos[a];
            e[3 * k + a] = rot[3 * a + 0] * X + rot[3 * a + 1] * Y + rot[3 * a + 2];
        }
    }
}

/*
 * Disk of view i (Sec. 4.1 and Sec. 4.4): plane through c_i with normal f_i,
 * local axes r_i, u_i. Returns a = e.f_i, the local intersection (u, v) and
 * rho = 1 - |(u,v)| / R, or for an oval disk (Sec. 4.4) 1 minus the radius
 * normalised by the extents of (u, v)'s quadrant (not clamped). For a <= 0 the
 * disk faces away and u, v, rho are set to NaN.
 */
void orc_disk(const orc_views *V, int32_t i, const double o[3], const double e[3],
              double *a_out, double *u_out, double *v_out, double *rho_out) {
    const double *c = V->centres + 3 * i, *R = V->rot + 9 * i;
    double f[3], r[3], u[3];
    col3(R, 0, r); col3(R, 1, u); col3(R, 2, f);
    double a = dot3(e, f);
    *a_out = a;
    if (!(a > 0.0)) { *u_out = *v_out = *rho_out = NAN; return; }
    double co[3]; sub3(c, o, co);
    double ts = dot3(co, f) / a;
    double q[3] = {o[0] + ts * e[0] - c[0], o[1] + ts * e[1] - c[1], o[2] + ts * e[2] - c[2]};
    double uu = dot3(q, r), vv = dot3(q, u);
    *u_out = uu; *v_out = vv;
    if (V->disk_ext) {
        const double *x = V->disk_ext + 4 * i;
        const double su = uu / (uu >= 0.0 ? x[0] : x[1]), sv = vv / (vv >= 0.0 ? x[2] : x[3]);
        *rho_out = 1.0 - sqrt(su * su + sv * sv);
    } else {
        *rho_out = 1.0 - sqrt(uu * uu + vv * vv) / V->disk_radius;
    }
}

/* World-space vertex (j, k) of view i's mesh: c_i + z_jk R_i (X_j, Y_k, 1). */
static inline void mesh_vertex(const orc_views *V, int32_t i, int32_t j, int32_t k, double out[3]) {
    const int32_t M = V->mesh_m;
    const double ts = tan(0.5 * V->src_fov_deg * M_PI / 180.0);
    double X = (2.0 * (j + 0.5) / M - 1.0) * ts;
    double Y = (1.0 - 2.0 * (k + 0.5) / M) * ts;
    double z = (double)V->zdepth[((int64_t)i * M + k) * M + j];
    const double *c = V->centres + 3 * i, *R = V->rot + 9 * i;
    for (int a = 0; a < 3; ++a) out[a] = c[a] + z * (R[3 * a + 0] * X + R[3 * a + 1] * Y + R[3 * a + 2]);
}

/*
 * Watertight ray/triangle test (Woop, Benthin & Wald, JCGT 2013): the ray is
 * sheared so that it runs along the +z axis of a permuted frame, and the
 * triangle is tested by the signs of three 2-D edge functions. A shared edge or
 * vertex is evaluated from the same operands in every triangle that owns it,
 * so a ray through it hits at least one of them (no cracks). Both faces count;
 * a zero edge function is inside (inclusive).
 */
static int tri_hit(const double o[3], const double d[3], const double v0[3], const double v1[3],
                   const double v2[3], double *t_out) {
    int kz = 0;
    if (fabs(d[1]) > fabs(d[kz])) kz = 1;
    if (fabs(d[2]) > fabs(d[kz])) kz = 2;
    int kx = (kz + 1) % 3, ky = (kx + 1) % 3;
    if (d[kz] < 0.0) { int tmp = kx; kx = ky; ky = tmp; }
    const double Sx = d[kx] / d[kz], Sy = d[ky] / d[kz], Sz = 1.0 / d[kz];
    double A[3], B[3], C[3];
    sub3(v0, o, A);
    sub3(v1, o, B);
    sub3(v2, o, C);
    const double Ax = A[kx] - Sx * A[kz], Ay = A[ky] - Sy * A[kz];
    const double Bx = B[kx] - Sx * B[kz], By = B[ky] - Sy * B[kz];
    const double Cx = C[kx] - Sx * C[kz], Cy = C[ky] - Sy * C[kz];
    const double U = Cx * By - Cy * Bx;
    const double Vv = Ax * Cy - Ay * Cx;
    const double Ww = Bx * Ay - By * Ax;
    if ((U < 0.0 || Vv < 0.0 || Ww < 0.0) && (U > 0.0 || Vv > 0.0 || Ww > 0.0)) return 0;
    const double det = U + Vv + Ww;
    if (det == 0.0) return 0;
    const double T = U * (Sz * A[kz]) + Vv * (Sz * B[kz]) + Ww * (Sz * C[kz]);
    *t_out = T / det;
    return 1;
}

/* Both triangles of cell (j, k); updates *best with the smallest positive t. */
static void test_cell(const orc_views *V, int32_t i, int32_t j, int32_t k, const double o[3],
                      const double e[3], double *best) {
    const int32_t M = V->mesh_m;
    if (j < 0 || k < 0 || j > M - 2 || k > M - 2) return;
    double v00[3], v10[3], v01[3], v11[3], t;
    mesh_vertex(V, i, j, k, v00);
    mesh_vertex(V, i, j + 1, k, v10);
    mesh_vertex(V, i, j, k + 1, v01);
    mesh_vertex(V, i, j + 1, k + 1, v11);
    if (tri_hit(o, e, v00, v10, v11, &t) && t > 0.0 && t < *best) *best = t;
    if (tri_hit(o, e, v00, v11, v01, &t) && t > 0.0 && t < *best) *best = t;
}

/*
 * Nearest intersection of the ray with view i's mesh (Sec. 4.1, Sec. 4.2.2,
 * Sec. 4.5). Returns t (INFINITY when the mesh is missed).
 */
double orc_mesh_hit(const orc_views *V, int32_t i, const double o[3], const double e[3]) {
    const int32_t M = V->mesh_m;
    double best = INFINITY;
    if (V->mode == 1) {
        for (int32_t k = 0; k < M - 1; ++k)
            for (int32_t j = 0; j < M - 1; ++j) test_cell(V, i, j, k, o, e, &best);
        return best;
    }
    /* Traversal: the mesh lies within z in [zmin, zmax] in view i's frame, so the
     * hit projects onto the image-plane segment between the ray's points at
     * those two depths. Walk the grid cells that segment crosses. */
    const double *c = V->centres + 3 * i, *R = V->rot + 9 * i;
    const double ts = tan(0.5 * V->src_fov_deg * M_PI / 180.0);
    double oc[3], ol[3], el[3];
    sub3(o, c, oc);
    to_local(R, oc, ol);
    to_local(R, e, el);
    if (!(el[2] > 0.0)) {
        /* rays that never move forward along f can still meet the mesh only if
         * they start in front of the view; never the case for eyes inside the
         * capture sphere, so fall back to the brute force walk */
        for (int32_t k = 0; k < M - 1; ++k)
            for (int32_t j = 0; j < M - 1; ++j) test_cell(V, i, j, k, o, e, &best);
        return best;
    }
    double zlo = V->zrange[2 * i], zhi = V->zrange[2 * i + 1];
    double g[2][2];
    for (int s = 0; s < 2; ++s) {
        double z = s ? zhi : zlo;
        double t = (z - ol[2]) / el[2];
        double px = ol[0] + t * el[0], py = ol[1] + t * el[1];
        double X = px / z, Y = py / z;
        g[s][0] = (X / ts + 1.0) * 0.5 * M - 0.5;  /* grid coordinate: vertex j sits at j */
        g[s][1] = (1.0 - Y / ts) * 0.5 * M - 0.5;
    }
    double bx0 = fmin(g[0][0], g[1][0]), bx1 = fmax(g[0][0], g[1][0]);
    double by0 = fmin(g[0][1], g[1][1]), by1 = fmax(g[0][1], g[1][1]);
    if (bx1 < -2.0 || by1 < -2.0 || bx0 > M + 1.0 || by0 > M + 1.0) return best;
    /* clip the walk to the grid box grown by two cells (the dilation covers the rest) */
    double x0 = g[0][0], y0 = g[0][1], x1 = g[1][0], y1 = g[1][1];
    {
        double dx = x1 - x0, dy = y1 - y0, tl = 0.0, th = 1.0;
        const double lo = -2.0, hi = M + 1.0;
        double p[4] = {-dx, dx, -dy, dy}, q[4] = {x0 - lo, hi - x0, y0 - lo, hi - y0};
        for (int s = 0; s < 4; ++s) {
            if (p[s] == 0.0) { if (q[s] < 0.0) return best; continue; }
            double r = q[s] / p[s];
            if (p[s] < 0.0) { if (r > tl) tl = r; } else { if (r < th) th = r; }
        }
        if (tl > th) return best;
        double nx0 = x0 + tl * dx, ny0 = y0 + tl * dy, nx1 = x0 + th * dx, ny1 = y0 + th * dy;
        x0 = nx0; y0 = ny0; x1 = nx1; y1 = ny1;
    }
    /* Amanatides-Woo over unit cells; cell (j,k) spans [j, j+1) x [k, k+1) */
    int64_t cj = (int64_t)floor(x0), ck = (int64_t)floor(y0);
    int64_t ej = (int64_t)floor(x1), ek = (int64_t)floor(y1);
    double dx = x1 - x0, dy = y1 - y0;
    int sx = dx > 0 ? 1 : (dx < 0 ? -1 : 0), sy = dy > 0 ? 1 : (dy < 0 ? -1 : 0);
    double tmx = INFINITY, tmy = INFINITY, tdx = INFINITY, tdy = INFINITY;
    if (sx != 0) { double nb = sx > 0 ? (double)(cj + 1) : (double)cj; tmx = (nb - x0) / dx; tdx = fabs(1.0 / dx); }
    if (sy != 0) { double nb = sy > 0 ? (double)(ck + 1) : (double)ck; tmy = (nb - y0) / dy; tdy = fabs(1.0 / dy); }
    int64_t guard = 4 * (int64_t)M + 16;
    for (;;) {
        for (int64_t kk = ck - 1; kk <= ck + 1; ++kk)
            for (int64_t jj = cj - 1; jj <= cj + 1; ++jj) test_cell(V, i, (int32_t)jj, (int32_t)kk, o, e, &best);
        if ((cj == ej && ck == ek) || --guard < 0) break;
        if (tmx < tmy) { if (tmx > 1.0) break; cj += sx; tmx += tdx; }
        else { if (tmy > 1.0) break; ck += sy; tmy += tdy; }
    }
    return best;
}

/*
 * YUV420 form of the images (the paper's tile cache stores its tiles as
 * YUV420: a full-resolution luma plane and a half-resolution two-channel
 * chroma plane, sampled separately and recombined to RGB; Sec. 7.2). Full
 * range BT.601 in 8-bit fixed point: Y = (77 R + 150 G + 29 B + 128) >> 8,
 * Cb = ((-43 R - 85 G + 128 B + 128) >> 8) + 128,
 * Cr = ((128 R - 107 G - 21 B + 128) >> 8) + 128 (clamped to 255; the shifts
 * floor), each chroma sample the rounded mean (sum + 2) >> 2 of the 2x2
 * block it covers. Integer arithmetic only, so any exact implementation gives
 * the same bytes. Image sizes must be even.
 */
static inline int32_t yuv_floor_div256(int32_t v) { return (v + 256 * 256) / 256 - 256; }

void orc_yuv420_encode(int32_t n, int32_t W, int32_t H, const uint8_t *rgba8, uint8_t *y, uint8_t *uv) {
    for (int32_t i = 0; i < n; ++i) {
        const uint8_t *img = rgba8 + (int64_t)i * W * H * 4;
        uint8_t *yi = y + (int64_t)i * W * H;
        uint8_t *ci = uv + (int64_t)i * (W / 2) * (H / 2) * 2;
        for (int32_t by = 0; by < H / 2; ++by)
            for (int32_t bx = 0; bx < W / 2; ++bx) {
                int32_t sb = 0, sr = 0;
                for (int32_t dy = 0; dy < 2; ++dy)
                    for (int32_t dx = 0; dx < 2; ++dx) {
                        const int64_t p = (int64_t)(2 * by + dy) * W + 2 * bx + dx;
                        const int32_t R = img[4 * p], G = img[4 * p + 1], B = img[4 * p + 2];
                        yi[p] = (uint8_t)((77 * R + 150 * G + 29 * B + 128) >> 8);
                        int32_t cb = yuv_floor_div256(-43 * R - 85 * G + 128 * B + 128) + 128;
                        int32_t cr = yuv_floor_div256(128 * R - 107 * G - 21 * B + 128) + 128;
                        sb += cb > 255 ? 255 : cb;
                        sr += cr > 255 ? 255 : cr;
                    }
                ci[2 * ((int64_t)by * (W / 2) + bx)] = (uint8_t)((sb + 2) >> 2);
                ci[2 * ((int64_t)by * (W / 2) + bx) + 1] = (uint8_t)((sr + 2) >> 2);
            }
    }
}

/*
 * RGTC form of the YUV420 planes (the paper's renderer can transcode its
 * cached YUV420 tiles to RGTC for a 4x smaller tile cache, Sec. 7.2). The
 * block format is the published RGTC1 (BC4, unsigned) one: a 4x4 block of one
 * 8-bit channel is 8 bytes, two endpoints e0 = byte 0 and e1 = byte 1, then a
 * 48-bit little-endian field holding a 3-bit code per texel, texel (x, y) of
 * the block at bits 3 (4 y + x). Code 0 stands for e0 and code 1 for e1; if
 * e0 > e1, codes 2..7 stand for the six points that split [e1, e0] into
 * sevenths, code c at ((8 - c) e0 + (c - 1) e1) / 7; otherwise codes 2..5
 * split it into fifths, ((6 - c) e0 + (c - 1) e1) / 5, code 6 is 0 and code 7
 * is 255. RGTC2 (BC5) is two such blocks, one per channel, first channel
 * first. Luma is coded in RGTC1 blocks of the full-resolution plane and the
 * chroma pair in RGTC2 blocks of the half-resolution plane, both row-major
 * over blocks, so the image sizes must be multiples of 8.
 *
 * The encoder (any encoder yields a valid block; this one is fixed so that
 * every implementation writes the same bytes, with integer arithmetic only):
 * e0 = the block maximum, e1 = the block minimum; a constant block takes code
 * 0 everywhere; otherwise each texel takes the nearest of the eight points,
 * the one at p = round(7 (e0 - x) / (e0 - e1)) sevenths from e0, halves
 * rounded up, coded 0 for p = 0, 1 for p = 7 and p + 1 in between.
 */
static void rgtc1_block(const uint8_t *src, int64_t stride, int32_t step, uint8_t out[8]) {
    int32_t v[16], hi = 0, lo = 255;
    for (int32_t t = 0; t < 16; ++t) {
        v[t] = src[(t / 4) * stride + (t % 4) * step];
        if (v[t] > hi) hi = v[t];
        if (v[t] < lo) lo = v[t];
    }
    uint64_t bits = 0;
    if (hi > lo) {
        const int32_t d = hi - lo;
        for (int32_t t = 0; t < 16; ++t) {
            const int32_t p = (14 * (hi - v[t]) + d) / (2 * d);
            const uint64_t code = p == 0 ? 0 : (p == 7 ? 1 : (uint64_t)(p + 1));
            bits |= code << (3 * t);
        }
    }
    out[0] = (uint8_t)hi;
    out[1] = (uint8_t)lo;
    for (int32_t b = 0; b < 6; ++b) out[2 + b] = (uint8_t)(bits >> (8 * b));
}

void orc_rgtc_encode(int32_t n, int32_t W, int32_t H, const uint8_t *y, const uint8_t *uv, uint8_t *yb,
                     uint8_t *uvb) {
    const int32_t Wc = W / 2, Hc = H / 2;
    for (int32_t i = 0; i < n; ++i) {
        const uint8_t *yi = y + (int64_t)i * W * H;
        const uint8_t *ci = uv + (int64_t)i * Wc * Hc * 2;
        uint8_t *ybi = yb + (int64_t)i * (W / 4) * (H / 4) * 8;
        uint8_t *cbi = uvb + (int64_t)i * (Wc / 4) * (Hc / 4) * 16;
        for (int32_t by = 0; by < H / 4; ++by)
            for (int32_t bx = 0; bx < W / 4; ++bx)
                rgtc1_block(yi + (int64_t)4 * by * W + 4 * bx, W, 1, ybi + 8 * ((int64_t)by * (W / 4) + bx));
        for (int32_t by = 0; by < Hc / 4; ++by)
            for (int32_t bx = 0; bx < Wc / 4; ++bx) {
                uint8_t *o = cbi + 16 * ((int64_t)by * (Wc / 4) + bx);
                const uint8_t *s0 = ci + 2 * ((int64_t)4 * by * Wc + 4 * bx);
                rgtc1_block(s0, 2 * (int64_t)Wc, 2, o);
                rgtc1_block(s0 + 1, 2 * (int64_t)Wc, 2, o + 8);
            }
    }
}

/* Texel t (= 4 y + x) of an RGTC1 block, decoded to a real value in 0..255. */
static double rgtc1_texel(const uint8_t *blk, int32_t t) {
    uint64_t bits = 0;
    for (int32_t b = 0; b < 6; ++b) bits |= (uint64_t)blk[2 + b] << (8 * b);
    const int32_t c = (int32_t)((bits >> (3 * t)) & 7u);
    const double e0 = blk[0], e1 = blk[1];
    if (c == 0) return e0;
    if (c == 1) return e1;
    if (blk[0] > blk[1]) return ((8 - c) * e0 + (c - 1) * e1) / 7.0;
    if (c == 6) return 0.0;
    if (c == 7) return 255.0;
    return ((6 - c) * e0 + (c - 1) * e1) / 5.0;
}

/* Texel (x, y) of channel ch of a plane of W x H texels stored as RGTC blocks
 * of bpb bytes (8: RGTC1; 16: RGTC2, channel ch's block at byte 8 ch). */
static double rgtc_plane_texel(const uint8_t *blocks, int32_t W, int32_t bpb, int32_t ch, int64_t x, int64_t y) {
    const uint8_t *blk = blocks + bpb * ((y / 4) * (W / 4) + x / 4) + 8 * ch;
    return rgtc1_texel(blk, (int32_t)(4 * (y % 4) + x % 4));
}

/* Decoded planes (luma [n][H][W], chroma [n][H/2][W/2][2]) in 0..255 units. */
void orc_rgtc_decode(int32_t n, int32_t W, int32_t H, const uint8_t *yb, const uint8_t *uvb, double *y, double *uv) {
    const int32_t Wc = W / 2, Hc = H / 2;
    for (int32_t i = 0; i < n; ++i) {
        const uint8_t *ybi = yb + (int64_t)i * (W / 4) * (H / 4) * 8;
        const uint8_t *cbi = uvb + (int64_t)i * (Wc / 4) * (Hc / 4) * 16;
        for (int64_t r = 0; r < H; ++r)
            for (int64_t c = 0; c < W; ++c) y[((int64_t)i * H + r) * W + c] = rgtc_plane_texel(ybi, W, 8, 0, c, r);
        for (int64_t r = 0; r < Hc; ++r)
            for (int64_t c = 0; c < Wc; ++c)
                for (int32_t ch = 0; ch < 2; ++ch)
                    uv[(((int64_t)i * Hc + r) * Wc + c) * 2 + ch] = rgtc_plane_texel(cbi, Wc, 16, ch, c, r);
    }
}

/* Bilinear sample of channel ch of an RGTC-coded plane, as plane_bilinear. */
static double rgtc_bilinear(const uint8_t *blocks, int32_t W, int32_t H, int32_t bpb, int32_t ch, double px, double py) {
    double fx0 = floor(px), fy0 = floor(py);
    double fx = px - fx0, fy = py - fy0;
    int64_t x0 = (int64_t)fx0, y0 = (int64_t)fy0, x1 = x0 + 1, y1 = y0 + 1;
    if (x0 < 0) x0 = 0; if (x0 > W - 1) x0 = W - 1;
    if (x1 < 0) x1 = 0; if (x1 > W - 1) x1 = W - 1;
    if (y0 < 0) y0 = 0; if (y0 > H - 1) y0 = H - 1;
    if (y1 < 0) y1 = 0; if (y1 > H - 1) y1 = H - 1;
    const double a = rgtc_plane_texel(blocks, W, bpb, ch, x0, y0), b = rgtc_plane_texel(blocks, W, bpb, ch, x1, y0);
    const double d = rgtc_plane_texel(blocks, W, bpb, ch, x0, y1), e = rgtc_plane_texel(blocks, W, bpb, ch, x1, y1);
    const double top = a + fx * (b - a), bot = d + fx * (e - d);
    return top + fy * (bot - top);
}

/* Bilinear sample of a one- or two-channel 8-bit plane at texel-centre
 * coordinate (px, py), clamp-to-edge; channel c of nc. */
static double plane_bilinear(const uint8_t *pl, int32_t W, int32_t H, int32_t nc, int32_t c, double px, double py) {
    double fx0 = floor(px), fy0 = floor(py);
    double fx = px - fx0, fy = py - fy0;
    int64_t x0 = (int64_t)fx0, y0 = (int64_t)fy0, x1 = x0 + 1, y1 = y0 + 1;
    if (x0 < 0) x0 = 0; if (x0 > W - 1) x0 = W - 1;
    if (x1 < 0) x1 = 0; if (x1 > W - 1) x1 = W - 1;
    if (y0 < 0) y0 = 0; if (y0 > H - 1) y0 = H - 1;
    if (y1 < 0) y1 = 0; if (y1 > H - 1) y1 = H - 1;
    const double a = pl[(y0 * W + x0) * nc + c], b = pl[(y0 * W + x1) * nc + c];
    const double d = pl[(y1 * W + x0) * nc + c], e = pl[(y1 * W + x1) * nc + c];
    const double top = a + fx * (b - a), bot = d + fx * (e - d);
    return top + fy * (bot - top);
}

/* Continuous sample of view i's image at normalised image-plane point (Xs, Ys):
 * bilinear over texel centres, clamp-to-edge, RGB/255. With YUV420 planes the
 * luma is sampled at full resolution and the chroma at half resolution (a
 * chroma sample sits at the centre of its 2x2 luma block), then recombined
 * with the full-range BT.601 inverse; no clamping of the result. With RGTC
 * blocks the planes' texels are the decoded block values, sampled the same
 * way. */
void orc_sample(const orc_views *V, int32_t i, double Xs, double Ys, double rgb[3]) {
    const double ts = tan(0.5 * V->src_fov_deg * M_PI / 180.0);
    const int32_t W = V->img_w, H = V->img_h;
    double px = (Xs / ts + 1.0) * 0.5 * W - 0.5;
    double py = (1.0 - Ys / ts) * 0.5 * H - 0.5;
    if (V->rgtc_y) {
        const uint8_t *yb = V->rgtc_y + (int64_t)i * (W / 4) * (H / 4) * 8;
        const uint8_t *cb_blocks = V->rgtc_uv + (int64_t)i * (W / 8) * (H / 8) * 16;
        const double Y = rgtc_bilinear(yb, W, H, 8, 0, px, py);
        const double cx = 0.5 * (px - 0.5), cy = 0.5 * (py - 0.5);
        const double cb = rgtc_bilinear(cb_blocks, W / 2, H / 2, 16, 0, cx, cy) - 128.0;
        const double cr = rgtc_bilinear(cb_blocks, W / 2, H / 2, 16, 1, cx, cy) - 128.0;
        rgb[0] = (Y + 1.402 * cr) / 255.0;
        rgb[1] = (Y - 0.344136 * cb - 0.714136 * cr) / 255.0;
        rgb[2] = (Y + 1.772 * cb) / 255.0;
        return;
    }
    if (V->yuv_y) {
        const double Y = plane_bilinear(V->yuv_y + (int64_t)i * W * H, W, H, 1, 0, px, py);
        const uint8_t *uv = V->yuv_uv + (int64_t)i * (W / 2) * (H / 2) * 2;
        const double cx = 0.5 * (px - 0.5), cy = 0.5 * (py - 0.5);
        const double cb = plane_bilinear(uv, W / 2, H / 2, 2, 0, cx, cy) - 128.0;
        const double cr = plane_bilinear(uv, W / 2, H / 2, 2, 1, cx, cy) - 128.0;
        rgb[0] = (Y + 1.402 * cr) / 255.0;
        rgb[1] = (Y - 0.344136 * cb - 0.714136 * cr) / 255.0;
        rgb[2] = (Y + 1.772 * cb) / 255.0;
        return;
    }
    double fx0 = floor(px), fy0 = floor(py);
    double fx = px - fx0, fy = py - fy0;
    int64_t x0 = (int64_t)fx0, y0 = (int64_t)fy0, x1 = x0 + 1, y1 = y0 + 1;
    if (x0 < 0) x0 = 0; if (x0 > W - 1) x0 = W - 1;
    if (x1 < 0) x1 = 0; if (x1 > W - 1) x1 = W - 1;
    if (y0 < 0) y0 = 0; if (y0 > H - 1) y0 = H - 1;
    if (y1 < 0) y1 = 0; if (y1 > H - 1) y1 = H - 1;
    const uint8_t *img = V->rgba8 + (int64_t)i * W * H * 4;
    const uint8_t *p00 = img + (y0 * W + x0) * 4, *p10 = img + (y0 * W + x1) * 4;
    const uint8_t *p01 = img + (y1 * W + x0) * 4, *p11 = img + (y1 * W + x1) * 4;
    for (int a = 0; a < 3; ++a) {
        double top = p00[a] + fx * ((double)p10[a] - p00[a]);
        double bot = p01[a] + fx * ((double)p11[a] - p01[a]);
        rgb[a] = (top + fy * (bot - top)) / 255.0;
    }
}

/*
 * Tile streaming (Sec. 4.2, tile streaming and caching; Sec. 7.2): the images
 * are cut into page x page tiles and only the tiles in the cache can be
 * sampled. Reading: a view whose bilinear sample for a ray needs a tile that
 * is not in the cache contributes nothing to that ray (left out of both sums
 * of Eq. 2, like a missed mesh). The taps of a sample are the four texels
 * orc_sample interpolates (clamped to the image), so a tile is needed iff one
 * of them lies in it, whatever its weight.
 */
static void sample_tap_tiles(const orc_views *V, double Xs, double Ys, int64_t tiles[4]) {
    const double ts = tan(0.5 * V->src_fov_deg * M_PI / 180.0);
    const int32_t W = V->img_w, H = V->img_h, P = V->page;
    const double px = (Xs / ts + 1.0) * 0.5 * W - 0.5, py = (1.0 - Ys / ts) * 0.5 * H - 0.5;
    int64_t x0 = (int64_t)floor(px), y0 = (int64_t)floor(py), x1 = x0 + 1, y1 = y0 + 1;
    if (x0 < 0) x0 = 0; if (x0 > W - 1) x0 = W - 1;
    if (x1 < 0) x1 = 0; if (x1 > W - 1) x1 = W - 1;
    if (y0 < 0) y0 = 0; if (y0 > H - 1) y0 = H - 1;
    if (y1 < 0) y1 = 0; if (y1 > H - 1) y1 = H - 1;
    const int64_t tw = W / P;
    tiles[0] = (y0 / P) * tw + x0 / P;
    tiles[1] = (y0 / P) * tw + x1 / P;
    tiles[2] = (y1 / P) * tw + x0 / P;
    tiles[3] = (y1 / P) * tw + x1 / P;
}

/* One view's full record for one ray (used by the per-ray loop and by tests). */
typedef struct {
    double a, u, v, rho, t_hit, Xs, Ys, rgb[3];
    int32_t cand, hit;
} orc_rec;

void orc_view_ray(const orc_views *V, int32_t i, const double o[3], const double e[3], orc_rec *r) {
    memset(r, 0, sizeof(*r));
    orc_disk(V, i, o, e, &r->a, &r->u, &r->v, &r->rho);
    r->t_hit = INFINITY;
    r->Xs = r->Ys = NAN;
    r->cand = (r->a > 0.0 && r->rho > 0.0);
    if (!r->cand) return;
    double t = orc_mesh_hit(V, i, o, e);
    if (!isfinite(t)) return;
    r->hit = 1;
    r->t_hit = t;
    /* reproject the 3-D hit into view i */
    const double *c = V->centres + 3 * i, *R = V->rot + 9 * i;
    double P[3] = {o[0] + t * e[0] - c[0], o[1] + t * e[1] - c[1], o[2] + t * e[2] - c[2]};
    double Pl[3];
    to_local(R, P, Pl);
    r->Xs = Pl[0] / Pl[2];
    r->Ys = Pl[1] / Pl[2];
    if (V->resident) {
        int64_t tl[4];
        sample_tap_tiles(V, r->Xs, r->Ys, tl);
        const int64_t tpv = (int64_t)(V->img_w / V->page) * (V->img_h / V->page);
        for (int k = 0; k < 4; ++k)
            if (!V->resident[(int64_t)i * tpv + tl[k]]) {
                r->hit = 0; /* the view is left out for this ray */
                return;
            }
    }
    orc_sample(V, i, r->Xs, r->Ys, r->rgb);
}

/*
 * The image tiles a set of rays samples: vis[i][tile] = 1 for every tile
 * holding a tap of a sample that view i contributes to one of the rays
 * (ignoring any residency table), else left as it is.
 */
void orc_visible_tiles(const orc_views *V, int64_t n_rays, const double *o, const double *e, int32_t page,
                       uint8_t *vis) {
    orc_views A = *V;
    A.resident = NULL;
    A.page = page;
    const int64_t tpv = (int64_t)(V->img_w / page) * (V->img_h / page);
#ifdef _OPENMP
    if (V->threads > 0) omp_set_num_threads(V->threads);
#endif
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < n_rays; ++k)
        for (int32_t i = 0; i < A.n; ++i) {
            orc_rec r;
            orc_view_ray(&A, i, o + 3 * k, e + 3 * k, &r);
            if (!r.hit) continue;
            int64_t tl[4];
            sample_tap_tiles(&A, r.Xs, r.Ys, tl);
            for (int q = 0; q < 4; ++q) {
#pragma omp atomic write
                vis[(int64_t)i * tpv + tl[q]] = 1;
            }
        }
}

/*
 * The visible tiles of a set of rays split by how firmly the oracle decides
 * them, for comparisons with a float implementation: must[i][tile] = 1 where a
 * ray shows the tile through decisions that are all well-conditioned (disk
 * margin |rho| > 1e-5 and a > 1e-9 |e|, hit more than 1e-6 inside the mesh
 * domain, and both tap coordinates more than `margin` texels away from a
 * texel boundary, so the tap columns and rows cannot change); may[i][tile] = 1
 * for every tile some ray could show under a decision within those bands
 * (both tap choices at a boundary, the hit of a view whose disk decision is
 * ill-conditioned either way). must is within the plain visible set and that
 * set within may. margin is below one texel (a position is then near at most
 * one boundary per axis). Arrays are OR-ed into (the caller clears them).
 */
void orc_visible_tiles_band(const orc_views *V, int64_t n_rays, const double *o, const double *e, int32_t page,
                            double margin, uint8_t *must, uint8_t *may) {
    const double md_band = 1e-5, a_band = 1e-9, edge_band = 1e-6;
    const double ts = tan(0.5 * V->src_fov_deg * M_PI / 180.0);
    const double dom = 1.0 - 1.0 / V->mesh_m;
    const int32_t W = V->img_w, H = V->img_h;
    const int64_t tw = W / page, tpv = (int64_t)tw * (H / page);
#ifdef _OPENMP
    if (V->threads > 0) omp_set_num_threads(V->threads);
#endif
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < n_rays; ++k) {
        const double *ok = o + 3 * k, *ek = e + 3 * k;
        const double en = sqrt(dot3(ek, ek));
        for (int32_t i = 0; i < V->n; ++i) {
            double a, u, v, rho;
            orc_disk(V, i, ok, ek, &a, &u, &v, &rho);
            const double md = isnan(rho) ? INFINITY : fabs(rho);
            const int band_c = md <= md_band || fabs(a) <= a_band * en;
            const int cand = a > 0.0 && rho > 0.0;
            if (!cand && !band_c) continue;
            const double t = orc_mesh_hit(V, i, ok, ek);
            if (!isfinite(t)) continue;
            const double *c = V->centres + 3 * i, *R = V->rot + 9 * i;
            double P[3] = {ok[0] + t * ek[0] - c[0], ok[1] + t * ek[1] - c[1], ok[2] + t * ek[2] - c[2]}, Pl[3];
            to_local(R, P, Pl);
            const double Xs = Pl[0] / Pl[2], Ys = Pl[1] / Pl[2];
            const int band_h = fmin(dom - fabs(Xs / ts), dom - fabs(Ys / ts)) < edge_band;
            const double px = (Xs / ts + 1.0) * 0.5 * W - 0.5, py = (1.0 - Ys / ts) * 0.5 * H - 0.5;
            /* the first tap column / row for the position and for positions within the margin */
            const double fx[2] = {floor(px - margin), floor(px + margin)};
            const double fy[2] = {floor(py - margin), floor(py + margin)};
            const int firm = cand && !band_c && !band_h && fx[0] == fx[1] && fy[0] == fy[1];
            for (int sy = 0; sy < 2; ++sy)
                for (int sx = 0; sx < 2; ++sx)
                    for (int dy = 0; dy < 2; ++dy)
                        for (int dx = 0; dx < 2; ++dx) {
                            int64_t x = (int64_t)fx[sx] + dx, y = (int64_t)fy[sy] + dy;
                            if (x < 0) x = 0; if (x > W - 1) x = W - 1;
                            if (y < 0) y = 0; if (y > H - 1) y = H - 1;
                            const int64_t q = (int64_t)i * tpv + (y / page) * tw + x / page;
#pragma omp atomic write
                            may[q] = 1;
                            if (firm) {
#pragma omp atomic write
                                must[q] = 1;
                            }
                        }
        }
    }
}

static void list_put(int32_t *list, int32_t cap, int32_t *cnt, int32_t id) {
    if (list && *cnt < cap) list[*cnt] = id;
    (*cnt)++;
}

/*
 * Eq. (2) for a batch of rays over ALL views (no culling). Outputs colour
 * (n,3), weight sum W (n), contributing-view count (n); lists optional.
 */
void orc_render_rays(const orc_views *V, int64_t n_rays, const double *o, const double *e,
                     double *rgb, double *wsum, int32_t *count, const orc_lists *L) {
#ifdef _OPENMP
    if (V->threads > 0) omp_set_num_threads(V->threads);
#endif
    const double md_band = 1e-5, a_band = 1e-9, edge_band = 1e-6;
    const double ts = tan(0.5 * V->src_fov_deg * M_PI / 180.0);
    const double dom = 1.0 - 1.0 / V->mesh_m; /* mesh domain in normalised image units */
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < n_rays; ++k) {
        const double *ok = o + 3 * k, *ek = e + 3 * k;
        double acc[3] = {0, 0, 0}, ws = 0.0;
        int32_t cnt = 0, nc = 0, nb = 0, nh = 0, nhb = 0;
        int32_t cap = L ? L->cap : 0;
        int32_t *lc = L && L->cand ? L->cand + k * cap : NULL;
        int32_t *lb = L && L->cand_band ? L->cand_band + k * cap : NULL;
        int32_t *lh = L && L->contrib ? L->contrib + k * cap : NULL;
        int32_t *lhb = L && L->contrib_band ? L->contrib_band + k * cap : NULL;
        double en = sqrt(dot3(ek, ek));
        for (int32_t i = 0; i < V->n; ++i) {
            orc_rec r;
            orc_view_ray(V, i, ok, ek, &r);
            if (L) {
                double md = isnan(r.rho) ? INFINITY : fabs(r.rho);
                if (md <= md_band || fabs(r.a) <= a_band * en) list_put(lb, cap, &nb, i);
            }
            if (!r.cand) continue;
            list_put(lc, cap, &nc, i);
            if (!r.hit) continue;
            if (L) {
                double m = fmin(dom - fabs(r.Xs / ts), dom - fabs(r.Ys / ts));
                if (m < edge_band) list_put(lhb, cap, &nhb, i);
            }
            list_put(lh, cap, &nh, i);
            for (int a = 0; a < 3; ++a) acc[a] += r.rho * r.rgb[a];
            ws += r.rho;
            cnt++;
        }
        if (L) {
            if (L->n_cand) L->n_cand[k] = nc;
            for (int32_t s = nc; s < cap; ++s) if (lc) lc[s] = -1;
            for (int32_t s = nb; s < cap; ++s) if (lb) lb[s] = -1;
            for (int32_t s = nh; s < cap; ++s) if (lh) lh[s] = -1;
            for (int32_t s = nhb; s < cap; ++s) if (lhb) lhb[s] = -1;
        }
        for (int a = 0; a < 3; ++a) rgb[3 * k + a] = ws > 0.0 ? acc[a] / ws : 0.0;
        if (wsum) wsum[k] = ws;
        if (count) count[k] = cnt;
    }
}

/*
 * Light field prefilter (Sec. 5, Eqs. (4)-(5)). The prefiltered value of pixel
 * (x', y') of view i of the real-time model T is the ratio estimate
 *
 *     sum_j rho_i(u_j, v_j) sigma(s_j, t_j) Lbar(o_j, e_j) / sum_j rho_i(u_j, v_j) sigma(s_j, t_j)
 *
 * over J sample pairs: (u_j, v_j) a point of view i's disk (the synthetic
 * aperture, the real-time disk of Sec. 4.1 or Sec. 4.4; disk_pts are points
 * (du, dv) of the unit disk, scaled by the target disk radius, or for an oval
 * aperture with extents ext = (e+u, e-u, e+v, e-v) by the extents of their
 * quadrant: u = du e+u for du >= 0, du e-u otherwise, v likewise), (s_j, t_j)
 * a point of the pixel basis' support around the pixel centre (pix_offs, in
 * pixels). The ray origin o_j is the disk point in 3-D
 * (c_i + u_j r_i + v_j u_i); the ray passes through the 3-D point of view i's
 * mesh that projects to image position (s_j, t_j) (the nearest hit of the ray
 * from c_i through that image point). Lbar is Eq. (2) over the offline model
 * (its own views, meshes and disks).
 *
 * Readings: rho is the linear falloff of Sec. 4.1 (1 - |(du, dv)| for a unit
 * disk point, which is also the oval kernel of Sec. 4.4 at the mapped point);
 * Eq. (4) integrates over the disk's area, and a uniform point of the unit
 * disk lands in an oval quadrant with density 1 / (e_u e_v), so an oval
 * sample's weight also carries the factor e_u e_v of its quadrant (a circle's
 * factor is the same for every sample and cancels); sigma is separable, box (1 on |d| <= 1/2) or Lanczos-2
 * (sinc(d) sinc(d/2) on |d| < 2); a sample whose image point has no mesh
 * point (outside the mesh domain), or whose ray no disk of the offline model
 * covers (Lbar undefined), is left out of both sums; a pixel whose
 * denominator is 0 is (0, 0, 0).
 */
static double lanczos2(double x) {
    x = fabs(x);
    if (x >= 2.0) return 0.0;
    if (x == 0.0) return 1.0;
    const double px = M_PI * x;
    return 2.0 * sin(px) * sin(0.5 * px) / (px * px);
}

double orc_basis(int32_t basis, double d) {
    if (basis == 1) return lanczos2(d);
    return fabs(d) <= 0.5 ? 1.0 : 0.0;
}

void orc_prefilter(const orc_views *Lbar, const orc_views *T, int32_t i, double radius, const double *ext, int32_t J,
                   const double *disk_pts, const double *pix_offs, int32_t basis, int64_t n_pix,
                   const int64_t *pix, double *rgb, double *wsum) {
#ifdef _OPENMP
    if (Lbar->threads > 0) omp_set_num_threads(Lbar->threads);
#endif
    const double *c = T->centres + 3 * i, *R = T->rot + 9 * i;
    const double ts = tan(0.5 * T->src_fov_deg * M_PI / 180.0);
    const int32_t W = T->img_w, H = T->img_h;
    double r[3], u[3];
    col3(R, 0, r);
    col3(R, 1, u);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < n_pix; ++q) {
        const double xc = (double)(pix[q] % W) + 0.5, yc = (double)(pix[q] / W) + 0.5;
        double num[3] = {0, 0, 0}, den = 0.0;
        for (int32_t j = 0; j < J; ++j) {
            const double du = disk_pts[2 * j], dv = disk_pts[2 * j + 1];
            const double rho = 1.0 - sqrt(du * du + dv * dv);
            const double sigma = orc_basis(basis, pix_offs[2 * j]) * orc_basis(basis, pix_offs[2 * j + 1]);
            /* the aperture point in metres along r and u: the circle of the
             * given radius, or the oval whose quadrant holds (du, dv) */
            const double su = ext ? (du >= 0.0 ? ext[0] : ext[1]) : radius;
            const double sv = ext ? (dv >= 0.0 ? ext[2] : ext[3]) : radius;
            /* uniform points of the unit disk land in an oval quadrant with
             * density 1 / (su sv): the area factor restores the uniform
             * measure du dv of Eq. (4) (constant for a circle, so left out) */
            const double wgt = ext ? rho * sigma * su * sv : rho * sigma;
            if (!(rho > 0.0) || wgt == 0.0) continue;
            /* the 3-D point of view i's mesh seen at image position (s, t) */
            const double s = xc + pix_offs[2 * j], t = yc + pix_offs[2 * j + 1];
            const double X = (2.0 * s / W - 1.0) * ts, Y = (1.0 - 2.0 * t / H) * ts;
            double dir[3];
            for (int a = 0; a < 3; ++a) dir[a] = R[3 * a + 0] * X + R[3 * a + 1] * Y + R[3 * a + 2];
            const double th = orc_mesh_hit(T, i, c, dir);
            if (!isfinite(th)) continue;
            double o[3], e[3];
            for (int a = 0; a < 3; ++a) {
                o[a] = c[a] + su * du * r[a] + sv * dv * u[a];
                e[a] = c[a] + th * dir[a] - o[a];
            }
            double L[3], ws;
            int32_t cnt;
            orc_render_rays(Lbar, 1, o, e, L, &ws, &cnt, NULL);
            if (!(ws > 0.0)) continue;
            for (int a = 0; a < 3; ++a) num[a] += wgt * L[a];
            den += wgt;
        }
        for (int a = 0; a < 3; ++a) rgb[3 * q + a] = den != 0.0 ? num[a] / den : 0.0;
        if (wsum) wsum[q] = den;
    }
}

/* Per-view records for a single ray (tests and diagnostics). */
void orc_ray_records(const orc_views *V, const double o[3], const double e[3], orc_rec *recs) {
    for (int32_t i = 0; i < V->n; ++i) orc_view_ray(V, i, o, e, &recs[i]);
}

int32_t orc_views_size(void) { return (int32_t)sizeof(orc_views); }
int32_t orc_rec_size(void) { return (int32_t)sizeof(orc_rec); }
int32_t orc_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
