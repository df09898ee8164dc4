/*
 * lfsynth — seeded synthetic inputs for the spherical light field renderer.
 *
 * This module produces INPUTS only: a capture rig on a sphere, an analytic
 * scene (spheres inside a box, or a single plane), the RGBA8 source images and
 * per-view z-depth maps obtained by ray casting that scene, and random head
 * poses. It contains none of the reconstruction arithmetic (disk selection,
 * mesh intersection, reprojection, sampling, blending); both the FP64 oracle
 * and the HIP path consume the bytes it writes.
 *
 * Shapes follow the paper's capture setup (Sec. 3: a 70 cm capture sphere;
 * Sec. 6: about a thousand views of about a megapixel; Sec. 7.1: 120-degree
 * source views; Sec. 4.5: per-view meshes from per-view depth maps).
 *
 * Camera convention shared by every consumer (a convention, not code):
 *   a camera frame is an orthonormal 3x3 matrix R, row-major, whose columns
 *   are (r, u, f): image +x, image up, optical axis. The camera-local point
 *   (X*z, Y*z, z) maps to world c + R (X*z, Y*z, z). Pixel (j, k) of a W x H
 *   image with half-FOV tangents (tx, ty) has its centre at
 *   X = (2(j+1/2)/W - 1) tx, Y = (1 - 2(k+1/2)/H) ty (row 0 at the top).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define SYN_MAX_SPHERES 64

typedef struct {
    int32_t kind;          /* 0 = spheres inside an axis-aligned box, 1 = single plane */
    int32_t texture;       /* 0 = checker x value noise, 1 = smooth sinusoid, 2 = constant */
    int32_t n_spheres;
    int32_t pad;
    double  sphere_c[SYN_MAX_SPHERES][3];
    double  sphere_r[SYN_MAX_SPHERES];
    double  sphere_rgb[SYN_MAX_SPHERES][3];
    double  box_half;      /* half side of the enclosing box (m) */
    double  box_rgb[6][3]; /* faces -x,+x,-y,+y,-z,+z */
    double  plane_n[3];    /* kind 1: points p with n.p = d */
    double  plane_d;
    double  const_rgb[3];  /* texture 2 */
    double  checker;       /* checker cell size (m) */
    double  noise_cell;    /* value-noise lattice spacing (m) */
    double  smooth_period; /* texture 1 period (m) */
    uint64_t noise_seed;
} syn_scene;

/* ---------------- deterministic random numbers (splitmix64) ---------------- */
static uint64_t sm_next(uint64_t *s) {
    uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static double sm_unif(uint64_t *s) { return (double)(sm_next(s) >> 11) * (1.0 / 9007199254740992.0); }
static double sm_gauss(uint64_t *s) {
    double u1 = sm_unif(s), u2 = sm_unif(s);
    if (u1 < 1e-300) u1 = 1e-300;
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}
static uint64_t hash3(int64_t i, int64_t j, int64_t k, uint64_t seed) {
    uint64_t s = seed ^ ((uint64_t)i * 0x8DA6B343ull) ^ ((uint64_t)j * 0xD8163841ull) ^ ((uint64_t)k * 0xCB1AB31Full);
    return sm_next(&s);
}

/* ---------------- rig ---------------- */
/* Fibonacci lattice of n points on a sphere of the given radius; outward frames. */
void syn_rig(int32_t n, double radius, double *centres, double *rot) {
    const double ga = M_PI * (3.0 - sqrt(5.0));
    for (int32_t k = 0; k < n; ++k) {
        double z = 1.0 - (2.0 * k + 1.0) / n;
        double s = sqrt(fmax(0.0, 1.0 - z * z));
        double phi = ga * k;
        double f[3] = {s * cos(phi), s * sin(phi), z};
        centres[3 * k + 0] = radius * f[0];
        centres[3 * k + 1] = radius * f[1];
        centres[3 * k + 2] = radius * f[2];
        /* r = normalise(f x z_hat), fallback f x y_hat; u = r x f */
        double r[3] = {f[1], -f[0], 0.0};
        double rn = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
        if (rn < 1e-9) { r[0] = -f[2]; r[1] = 0.0; r[2] = f[0]; rn = sqrt(r[0] * r[0] + r[2] * r[2]); }
        r[0] /= rn; r[1] /= rn; r[2] /= rn;
        double u[3] = {r[1] * f[2] - r[2] * f[1], r[2] * f[0] - r[0] * f[2], r[0] * f[1] - r[1] * f[0]};
        double *R = rot + 9 * k;
        for (int a = 0; a < 3; ++a) { R[3 * a + 0] = r[a]; R[3 * a + 1] = u[a]; R[3 * a + 2] = f[a]; }
    }
}

/* Mean over views of the distance (chord) to the nearest other view. */
double syn_mean_nn(int32_t n, const double *c) {
    double acc = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        double best = INFINITY;
        for (int32_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = c[3 * i] - c[3 * j], dy = c[3 * i + 1] - c[3 * j + 1], dz = c[3 * i + 2] - c[3 * j + 2];
            double d = sqrt(dx * dx + dy * dy + dz * dz);
            if (d < best) best = d;
        }
        acc += best;
    }
    return acc / n;
}
double syn_min_nn(int32_t n, const double *c) {
    double best = INFINITY;
    for (int32_t i = 0; i < n; ++i)
        for (int32_t j = i + 1; j < n; ++j) {
            double dx = c[3 * i] - c[3 * j], dy = c[3 * i + 1] - c[3 * j + 1], dz = c[3 * i + 2] - c[3 * j + 2];
            double d = sqrt(dx * dx + dy * dy + dz * dz);
            if (d < best) best = d;
        }
    return best;
}

/* ---------------- scenes ---------------- */
static void unit_dir(uint64_t *s, double d[3]) {
    double x, y, z, n;
    do { x = sm_gauss(s); y = sm_gauss(s); z = sm_gauss(s); n = sqrt(x * x + y * y + z * z); } while (n < 1e-12);
    d[0] = x / n; d[1] = y / n; d[2] = z / n;
}

/* K spheres: radius U[0.3,1] m, centre = uniform direction x U[1.5,4] m; plus a box. */
void syn_scene_spheres(syn_scene *sc, uint64_t seed, int32_t n_spheres, double box_half) {
    memset(sc, 0, sizeof(*sc));
    uint64_t s = seed * 0x2545F4914F6CDD1Dull + 17u;
    if (n_spheres > SYN_MAX_SPHERES) n_spheres = SYN_MAX_SPHERES;
    sc->kind = 0; sc->texture = 0; sc->n_spheres = n_spheres; sc->box_half = box_half;
    for (int32_t k = 0; k < n_spheres; ++k) {
        double rad = 0.3 + 0.7 * sm_unif(&s);
        double d[3]; unit_dir(&s, d);
        double dist = 1.5 + 2.5 * sm_unif(&s);
        for (int a = 0; a < 3; ++a) sc->sphere_c[k][a] = d[a] * dist;
        sc->sphere_r[k] = rad;
        for (int a = 0; a < 3; ++a) sc->sphere_rgb[k][a] = 0.25 + 0.75 * sm_unif(&s);
    }
    for (int f = 0; f < 6; ++f)
        for (int a = 0; a < 3; ++a) sc->box_rgb[f][a] = 0.3 + 0.7 * sm_unif(&s);
    sc->checker = 0.2; sc->noise_cell = 0.09; sc->smooth_period = 1.0;
    sc->noise_seed = sm_next(&s);
}

/* A single plane n.p = d; texture 1 (smooth) or 2 (constant). */
void syn_scene_plane(syn_scene *sc, const double n[3], double d, int32_t texture, double period, const double rgb[3]) {
    memset(sc, 0, sizeof(*sc));
    sc->kind = 1; sc->texture = texture;
    double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    for (int a = 0; a < 3; ++a) sc->plane_n[a] = n[a] / nn;
    sc->plane_d = d / nn;
    sc->smooth_period = period; sc->checker = 0.2; sc->noise_cell = 0.09;
    for (int a = 0; a < 3; ++a) sc->const_rgb[a] = rgb[a];
}

static double smooth5(double t) { return t * t * t * (t * (t * 6.0 - 15.0) + 10.0); }

static double value_noise(const syn_scene *sc, const double p[3]) {
    double x = p[0] / sc->noise_cell, y = p[1] / sc->noise_cell, z = p[2] / sc->noise_cell;
    double fx = floor(x), fy = floor(y), fz = floor(z);
    int64_t i = (int64_t)fx, j = (int64_t)fy, k = (int64_t)fz;
    double tx = smooth5(x - fx), ty = smooth5(y - fy), tz = smooth5(z - fz);
    double v[8];
    for (int c = 0; c < 8; ++c)
        v[c] = (double)(hash3(i + (c & 1), j + ((c >> 1) & 1), k + ((c >> 2) & 1), sc->noise_seed) >> 11) * (1.0 / 9007199254740992.0);
    double x00 = v[0] + tx * (v[1] - v[0]), x10 = v[2] + tx * (v[3] - v[2]);
    double x01 = v[4] + tx * (v[5] - v[4]), x11 = v[6] + tx * (v[7] - v[6]);
    double y0 = x00 + ty * (x10 - x00), y1 = x01 + ty * (x11 - x01);
    return y0 + tz * (y1 - y0);
}

/* Surface colour at world point p on object obj (sphere index, or 100+face for the box, 200 for the plane). */
void syn_texture(const syn_scene *sc, int32_t obj, const double p[3], double rgb[3]) {
    if (sc->texture == 2) { for (int a = 0; a < 3; ++a) rgb[a] = sc->const_rgb[a]; return; }
    if (sc->texture == 1) {
        const double w = 6.283185307179586 / sc->smooth_period;
        rgb[0] = 0.5 + 0.3 * sin(w * p[1] + 0.3) * cos(w * p[2] - 0.2);
        rgb[1] = 0.5 + 0.3 * cos(w * p[1] - 0.7) * sin(w * p[2] + 0.4);
        rgb[2] = 0.5 + 0.25 * sin(w * (p[1] + p[2]) + 1.1);
        return;
    }
    const double *base;
    if (obj < 100) base = sc->sphere_rgb[obj];
    else if (obj < 200) base = sc->box_rgb[obj - 100];
    else base = sc->const_rgb;
    int64_t cx = (int64_t)floor(p[0] / sc->checker), cy = (int64_t)floor(p[1] / sc->checker), cz = (int64_t)floor(p[2] / sc->checker);
    double chk = (double)((cx + cy + cz) & 1);
    double nz = value_noise(sc, p);
    double m = (0.55 + 0.45 * chk) * (0.7 + 0.3 * nz);
    for (int a = 0; a < 3; ++a) rgb[a] = base[a] * m;
}

/* Nearest positive hit of the ray o + t d with the scene; returns t (INFINITY if none). */
double syn_cast(const syn_scene *sc, const double o[3], const double d[3], int32_t *obj) {
    double best = INFINITY; int32_t bo = -1;
    if (sc->kind == 1) {
        double den = sc->plane_n[0] * d[0] + sc->plane_n[1] * d[1] + sc->plane_n[2] * d[2];
        if (fabs(den) > 1e-300) {
            double t = (sc->plane_d - (sc->plane_n[0] * o[0] + sc->plane_n[1] * o[1] + sc->plane_n[2] * o[2])) / den;
            if (t > 0) { best = t; bo = 200; }
        }
        if (obj) *obj = bo;
        return best;
    }
    double dd = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    for (int32_t k = 0; k < sc->n_spheres; ++k) {
        double oc[3] = {o[0] - sc->sphere_c[k][0], o[1] - sc->sphere_c[k][1], o[2] - sc->sphere_c[k][2]};
        double b = oc[0] * d[0] + oc[1] * d[1] + oc[2] * d[2];
        double c = oc[0] * oc[0] + oc[1] * oc[1] + oc[2] * oc[2] - sc->sphere_r[k] * sc->sphere_r[k];
        double disc = b * b - dd * c;
        if (disc < 0) continue;
        double sq = sqrt(disc);
        double t = (-b - sq) / dd;
        if (t <= 0) t = (-b + sq) / dd;
        if (t > 0 && t < best) { best = t; bo = k; }
    }
    if (sc->box_half > 0) {
        /* exit distance from inside the box */
        for (int a = 0; a < 3; ++a) {
            if (d[a] == 0.0) continue;
            double wall = d[a] > 0 ? sc->box_half : -sc->box_half;
            double t = (wall - o[a]) / d[a];
            if (t > 0 && t < best) { best = t; bo = 100 + 2 * a + (d[a] > 0 ? 1 : 0); }
        }
    }
    if (obj) *obj = bo;
    return best;
}

/*
 * Ray-cast n views: RGBA8 images (img_w x img_h, one ray per pixel centre) and
 * z-depth maps (mesh_m x mesh_m, one ray per depth-pixel centre; z along f).
 * Either output may be NULL. Depth of a ray that escapes the scene is written as
 * +inf (never happens for the box scenes). Returns the number of escaped rays.
 */
int64_t syn_render_views(const syn_scene *sc, int32_t n, const double *centres, const double *rot,
                         double fov_deg, int32_t img_w, int32_t img_h, uint8_t *rgba8,
                         int32_t mesh_m, float *zdepth, int32_t threads) {
    const double tf = tan(0.5 * fov_deg * M_PI / 180.0);
    int64_t escaped = 0;
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#endif
    if (rgba8) {
        const int64_t total = (int64_t)n * img_h;
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : escaped)
        for (int64_t vr = 0; vr < total; ++vr) {
            int32_t v = (int32_t)(vr / img_h), k = (int32_t)(vr % img_h);
            const double *c = centres + 3 * v, *R = rot + 9 * v;
            double Y = (1.0 - 2.0 * (k + 0.5) / img_h) * tf;
            uint8_t *row = rgba8 + ((int64_t)v * img_h + k) * (int64_t)img_w * 4;
            for (int32_t j = 0; j < img_w; ++j) {
                double X = (2.0 * (j + 0.5) / img_w - 1.0) * tf;
                double d[3] = {R[0] * X + R[1] * Y + R[2], R[3] * X + R[4] * Y + R[5], R[6] * X + R[7] * Y + R[8]};
                int32_t obj;
                double t = syn_cast(sc, c, d, &obj);
                double rgb[3] = {0, 0, 0};
                if (isfinite(t)) {
                    double p[3] = {c[0] + t * d[0], c[1] + t * d[1], c[2] + t * d[2]};
                    syn_texture(sc, obj, p, rgb);
                } else {
                    escaped++;
                }
                for (int a = 0; a < 3; ++a) {
                    double q = floor(fmin(fmax(rgb[a], 0.0), 1.0) * 255.0 + 0.5);
                    row[4 * j + a] = (uint8_t)q;
                }
                row[4 * j + 3] = 255;
            }
        }
    }
    if (zdepth) {
        const int64_t total = (int64_t)n * mesh_m;
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : escaped)
        for (int64_t vr = 0; vr < total; ++vr) {
            int32_t v = (int32_t)(vr / mesh_m), k = (int32_t)(vr % mesh_m);
            const double *c = centres + 3 * v, *R = rot + 9 * v;
            double Y = (1.0 - 2.0 * (k + 0.5) / mesh_m) * tf;
            float *row = zdepth + ((int64_t)v * mesh_m + k) * (int64_t)mesh_m;
            for (int32_t j = 0; j < mesh_m; ++j) {
                double X = (2.0 * (j + 0.5) / mesh_m - 1.0) * tf;
                double d[3] = {R[0] * X + R[1] * Y + R[2], R[3] * X + R[4] * Y + R[5], R[6] * X + R[7] * Y + R[8]};
                double t = syn_cast(sc, c, d, NULL);
                /* d has unit component along f, so the ray parameter is the z-depth */
                if (!isfinite(t)) escaped++;
                row[j] = (float)t;
            }
        }
    }
    return escaped;
}

/*
 * Head poses: position uniform in a ball (radius * U^(1/3) * direction),
 * orientation uniform on SO(3) from a normalised 4-D Gaussian quaternion q.
 * The frame written is (r, u, f) = (Q e_x, Q e_y, -Q e_z) so that image +x,
 * image up and the optical axis follow the same handedness as the rig frames.
 */
void syn_poses(uint64_t seed, int32_t count, double ball_radius, double *pos, double *rot) {
    uint64_t s = seed * 0x9E3779B97F4A7C15ull + 0x1234567ull;
    for (int32_t p = 0; p < count; ++p) {
        double d[3]; unit_dir(&s, d);
        double rr = ball_radius * cbrt(sm_unif(&s));
        for (int a = 0; a < 3; ++a) pos[3 * p + a] = rr * d[a];
        double w, x, y, z, n;
        do { w = sm_gauss(&s); x = sm_gauss(&s); y = sm_gauss(&s); z = sm_gauss(&s); n = sqrt(w * w + x * x + y * y + z * z); } while (n < 1e-12);
        w /= n; x /= n; y /= n; z /= n;
        double Q[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                       2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                       2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
        double *R = rot + 9 * p;
        for (int a = 0; a < 3; ++a) { R[3 * a + 0] = Q[3 * a + 0]; R[3 * a + 1] = Q[3 * a + 1]; R[3 * a + 2] = -Q[3 * a + 2]; }
    }
}

/* Uniform doubles in [0,1) from a seed (for test sampling that both sides share). */
void syn_uniform(uint64_t seed, int64_t count, double *out) {
    uint64_t s = seed ^ 0xA0761D6478BD642Full;
    for (int64_t i = 0; i < count; ++i) out[i] = sm_unif(&s);
}

int32_t syn_scene_size(void) { return (int32_t)sizeof(syn_scene); }
