/*
 * lf.h -- C ABI of the MI355X light field renderer (liblf.so).
 *
 * The library answers the disk-blended light field query of Overbeck et al.
 * 2018 (Sec. 4.1, Eq. (2)) for every pixel of one or more eye views:
 *
 *   L(o, e) = sum_i I_i(s_i, t_i) rho_i(u_i, v_i) / sum_i rho_i(u_i, v_i)
 *
 * over a set of source views captured on a sphere. Each view i has a centre of
 * projection c_i, an orthonormal frame R_i (columns r_i, u_i, f_i: image +x,
 * image up, optical axis), an RGBA8 image and a z-depth map that defines the
 * view's own triangle mesh (Sec. 4.5: two triangles per depth pixel, vertices
 * at depth-pixel centres, cell (j,k) split along its (j,k)-(j+1,k+1) diagonal).
 * The disk of view i lies in the plane through c_i with normal f_i, with local
 * axes r_i, u_i, and weights rays by rho = 1 - r/R (Sec. 4.1 linear falloff),
 * or, for an asymmetric oval disk (Sec. 4.4) with extents (e+u, e-u, e+v,
 * e-v), by rho = 1 - sqrt((u/e_u)^2 + (v/e_v)^2) where e_u is e+u for u >= 0
 * and e-u otherwise (e_v likewise).
 * (s_i, t_i) is the image-i position of the nearest intersection of the ray
 * with view i's mesh (intra-image occlusion only, Sec. 4.2.2); a view whose
 * disk or mesh the ray misses contributes to neither sum. A pixel no view
 * contributes to is (0,0,0).
 *
 * Conventions
 *  - Every function returns LF_OK (0) or a negative LF_E* code; the message of
 *    the last failure on the calling thread is returned by lf_last_error().
 *    No C++ exception crosses this boundary.
 *  - Frames are 3x3 row-major doubles whose COLUMNS are (r, u, f). The
 *    camera-local point (X z, Y z, z) is the world point c + R (X z, Y z, z).
 *  - Pixel (x, y) of a W x H image with horizontal half-FOV tangent tx has its
 *    centre ray through X = (2(x+1/2)/W - 1) tx, Y = (1 - 2(y+1/2)/H) ty,
 *    ty = tx H / W (row 0 at the top, square pixels). Source views are square
 *    with the same FOV on both axes.
 *  - Render calls are asynchronous on the given HIP stream (NULL = the null
 *    stream). Argument errors are returned at once; a device fault surfaces as
 *    LF_EHIP from a later call or synchronisation.
 *  - A context owns all device memory it allocates and is not thread-safe; use
 *    one context per host thread / stream. Separate contexts are independent.
 */
#ifndef LF_H
#define LF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lf_ctx lf_ctx;

enum {
    LF_OK = 0,
    LF_EINVAL = -1, /* invalid argument (null pointer, bad size, non-orthonormal frame, ...) */
    LF_ENOMEM = -2, /* device allocation failed */
    LF_EHIP = -3,   /* HIP runtime error (launch failure, asynchronous fault) */
    LF_ESTATE = -4  /* call not valid in the context's current state */
};

/* Storage format of the source images on the device. RGBA32F is the plain
 * FP32 form; RGBA16F and RGBA8 (UNORM) are the compact forms. YUV420 is the
 * form of the paper's tile cache (Sec. 7.2): a full-resolution 8-bit luma
 * plane and a half-resolution two-channel 8-bit chroma plane (1.5 bytes per
 * texel), converted on load with full-range BT.601 in 8-bit fixed point
 * (Y = (77 R + 150 G + 29 B + 128) >> 8, Cb = ((-43 R - 85 G + 128 B + 128)
 * >> 8) + 128, Cr = ((128 R - 107 G - 21 B + 128) >> 8) + 128, clamped to 255,
 * each chroma sample the rounded mean of its 2x2 block), sampled bilinearly
 * per plane (a chroma sample sits at the centre of its block) and recombined
 * with the BT.601 inverse; it needs even image sizes. YUV420_RGTC is the
 * same two planes transcoded to RGTC blocks, the paper's 4x smaller tile
 * cache (Sec. 7.2): luma as RGTC1 (BC4) blocks of 4 x 4 texels, 8 bytes
 * each, chroma as RGTC2 (BC5) blocks of 4 x 4 chroma samples, 16 bytes each
 * (the Cb block, then the Cr block), 0.75 bytes per texel in all. Each block
 * takes e0 = its maximum and e1 = its minimum and every value the nearest of
 * the eight points that split [e1, e0] into sevenths (halves rounded towards
 * e1; a constant block takes code 0 everywhere, so the five-point form is
 * never used); the render decodes the texels it reads from their blocks and
 * samples as for YUV420. It needs image sizes that are multiples of 8. All sampling
 * and blending arithmetic is FP32 in every format. */
enum {
    LF_IMG_RGBA8 = 0,
    LF_IMG_RGBA16F = 1,
    LF_IMG_RGBA32F = 2,
    LF_IMG_YUV420 = 3,
    LF_IMG_YUV420_RGTC = 4,
    LF_IMG_PAGED_RGBA8 = 5  /* RGBA8 tiles streamed into a device tile cache: see lf_cache_config */
};

/* Storage of the per-view geometry: inverse depth 1/z of each mesh vertex,
 * packed per mesh cell (its four corners): FP32 (16 bytes a cell), FP16 (8
 * bytes), or 16-bit codes spread linearly over the view's inverse-depth range
 * (8 bytes; w = min + code * (max - min) / 65535, an error of at most half a
 * step, 1/131070 of the range, where FP16 errs by up to 2^-11 of w).
 * Intersection arithmetic is FP32. */
enum { LF_GEO_F32 = 0, LF_GEO_F16 = 1, LF_GEO_U16 = 2 };

/* lf_views_desc.flags: the rgba8 / zdepth pointers are device pointers. */
enum { LF_SRC_DEVICE = 1 };

typedef struct {
    int32_t n_views;          /* N >= 1 (at most 65535) */
    int32_t img_w, img_h;     /* source image size, pixels (square FOV: img_w == img_h) */
    int32_t mesh_m;           /* depth map is mesh_m x mesh_m, mesh_m >= 2 */
    double src_fov_deg;       /* full FOV of the source views, in (0, 180) */
    const double *centres;    /* [N][3] view centres c_i, world metres (host memory) */
    const double *rot;        /* [N][9] frames R_i, row-major, columns (r,u,f) (host memory) */
    const uint8_t *rgba8;     /* [N][img_h][img_w][4] images, UNORM8; alpha is ignored */
    const float *zdepth;      /* [N][mesh_m][mesh_m] z along f_i at depth-pixel centres, metres, > 0 */
    double disk_radius;       /* R, metres, > 0: circular disks (and the unit of lf_render_reference's scale) */
    const double *disk_ext;   /* NULL for circular disks of radius R, else [N][4] oval extents e+u, e-u, e+v,
                                 e-v in metres, each finite and > 0 (host memory; see lf_disk_extents) */
    int32_t img_fmt;          /* LF_IMG_* */
    int32_t geo_fmt;          /* LF_GEO_* */
    int32_t flags;            /* LF_SRC_DEVICE or 0 */
} lf_views_desc;

/*
 * Extents of asymmetric oval disks (Sec. 4.4): every disk reaches the centres
 * of its 1-ring neighbours in a Delaunay triangulation of the disk centres;
 * its extent towards +u, -u, +v and -v (the frame's r and u axes) is the
 * furthest 1-ring neighbour on that side, measured as the neighbour's centre
 * offset projected on the axis. The views are taken to lie on a capture sphere
 * about the origin, whose Delaunay triangulation is the convex hull of the
 * centres' directions. centres [N][3], rot [N][9] as in lf_views_desc (host);
 * out_ext [N][4] (host) receives scale * (e+u, e-u, e+v, e-v) in metres. Where
 * four centres are (nearly) co-circular both diagonals are Delaunay and either
 * may be chosen. Host computation, synchronous, no device use.
 * LF_EINVAL: NULL pointer, N outside [4, 65535], scale not finite and > 0, a
 * centre at the origin, directions that do not close a sphere (coplanar,
 * duplicated), or a view with no neighbour on one side of an axis.
 */
int lf_disk_extents(int32_t n_views, const double *centres, const double *rot, double scale, double *out_ext);

/* One eye: centre of projection and frame (columns r, u, f). */
typedef struct {
    double pos[3];
    double rot[9];
} lf_eye;

/* Launch shape: screen tile of tile_w x tile_h pixels (both multiples of 8,
 * tile_w * tile_h <= 256); one workgroup renders one tile, one wavefront one
 * 8 x 8 pixel block of it. cap: capacity of a tile's candidate-view list
 * (1..64; 0 = 64): the culling lists the views whose disk may reach the tile,
 * each with an upper bound of the inverse depth its rays can meet (where
 * their mesh walks start), and a tile with more than cap of them is rendered
 * by the exact scan over every view instead, whose walks start from the
 * inverse-depth blocks (the same views in the same order, and a mesh cell's
 * root does not depend on where a walk entered the cell, so shapes and caps
 * give the same image: bit for bit in the tests; a root within rounding of a
 * cell edge may come from either cell). A smaller cap sends more tiles to the
 * scan. */
typedef struct {
    int32_t tile_w, tile_h;
    int32_t cap;
} lf_tune;

/*
 * Copy a light field to the device and prepare it for rendering: convert the
 * images to img_fmt, turn each depth map into per-cell inverse-depth corners
 * (the vertex set of the view's mesh, Sec. 4.5) and record each view's
 * inverse-depth range. The caller may free every input on return.
 * Errors: LF_EINVAL for a null pointer, non-positive size, an image side
 * below 2, mesh_m < 2,
 * img_w != img_h, FOV outside (0,180), a frame not orthonormal to 1e-6, a
 * depth that is not finite and positive, or R <= 0; LF_EINVAL also when an
 * image dimension reaches 2^24 or one view's share of any per-view array
 * (the image in img_fmt or its second plane, the RGBA8 source image, the
 * mesh cells in geo_fmt) reaches 2^32 bytes: the kernels address within a
 * view with 32-bit offsets (e.g. RGBA32F views must be below 16384^2,
 * RGBA8 below 32768^2). These size checks come before any device use.
 * LF_ENOMEM; LF_EHIP.
 * On success *out owns the device data until lf_free.
 */
int lf_load_views(const lf_views_desc *d, lf_ctx **out);

/* Stereo pair from a head pose: eyes at pos -/+ (ipd/2) r_head with the head's
 * frame (parallel optical axes). out[0] is the left eye. */
int lf_stereo_eyes(const double head_pos[3], const double head_rot[9], double ipd_m, lf_eye out[2]);

/* Set the launch shape used by lf_render (NULL restores the default: 16 x 16
 * tiles, candidate lists of 64). */
int lf_set_tune(lf_ctx *c, const lf_tune *t);

/*
 * Render n_eyes eye views (Sec. 4.1, Eqs. (1)-(2)). res[2k], res[2k+1] are the
 * width and height of eye k; hfov_deg is the horizontal FOV of every eye.
 * out_rgb is a DEVICE buffer of sum_k W_k H_k RGB float triples, eyes
 * concatenated in order, each eye row-major from the top row. out_wsum
 * (device, one float per pixel: sum of rho over contributing views) and
 * out_count (device, one byte per pixel: number of contributing views,
 * saturating at 255) may be NULL. Every eye must lie behind every view's disk
 * plane (inside the capture surface), else LF_EINVAL.
 */
int lf_render(lf_ctx *c, const lf_eye *eyes, int32_t n_eyes, double hfov_deg, const int32_t *res,
              float *out_rgb, float *out_wsum, uint8_t *out_count, void *hip_stream);

/*
 * lf_render for callers that cannot allocate device memory: code under HIP
 * stream capture, tight serving loops, harnesses that forbid hipMalloc. Same
 * arguments, results and asynchrony as lf_render (bit for bit the same
 * image), but the per-launch scratch (per eye-view records, per-tile
 * candidate lists and counts) lives in a fixed device array of 16 MiB that
 * the library holds on each GPU until the process ends, instead of in the
 * context's buffer. The call allocates nothing and records no timing events
 * (lf_profile does not see it). Nothing in the scratch needs clearing: the
 * set-up and culling kernels write every entry the render reads.
 * Limit: each launch of at most 16 eyes must fit in 16 MiB (a stereo pair of
 * 2160 x 2160 eyes over 1024 views needs about 9.2 MiB at the default
 * 16 x 16 tiles); a call
 * with a larger launch returns LF_EINVAL before launching anything.
 * Every call on one GPU shares that GPU's array: calls whose work overlaps on
 * one GPU (different streams, or host threads, without ordering) race and
 * must not be made. The current device must be the context's device.
 */
int lf_render_noalloc(lf_ctx *c, const lf_eye *eyes, int32_t n_eyes, double hfov_deg, const int32_t *res,
                      float *out_rgb, float *out_wsum, uint8_t *out_count, void *hip_stream);

/*
 * Views taking part in renders. enabled: host uint8 [n_views], non-zero =
 * enabled, or NULL to enable every view (the state after lf_load_views). A
 * disabled view is left out of every later query (render, batch, reference,
 * prefilter, candidate lists): Eq. (2) sums over the enabled views only.
 * Synchronous: waits for the device to be idle, then applies to later calls.
 */
int lf_set_view_mask(lf_ctx *c, const uint8_t *enabled);

/*
 * Two-level progressive rendering (Sec. 7.2): the context holds a fine level
 * (views [0, n_fine)) and a coarse level (views [n_fine, n_views), typically
 * a subset of the same captures with larger disks given through per-view
 * extents); each level alone is a complete light field. Given which fine
 * views are available this frame (fine_available, host uint8 [n_fine], e.g.
 * the ones a decode budget allowed), writes the view mask for
 * lf_set_view_mask: every available fine view, plus every coarse view whose
 * disk reaches the centre of an unavailable fine view (the coarse disk is
 * drawn in the region the missing fine disks leave); both levels then blend
 * in Eq. (2). mask_out: host uint8 [n_views].
 */
int lf_two_level_mask(const lf_ctx *c, int32_t n_fine, const uint8_t *fine_available, uint8_t *mask_out);

/*
 * Tile streaming and caching (Sec. 4.2, tile streaming and caching; Sec. 7.2).
 * A context loaded with LF_IMG_PAGED_RGBA8 (image sizes multiples of 64) keeps
 * every image cut into 64 x 64-texel tiles in pinned host memory (the store
 * the paper decodes its tiles from) and samples them only from a device cache
 * of pages, one tile per 16 KB page, found through a per-view page table. A
 * view whose bilinear sample for a ray needs a tile that is not in the cache
 * contributes nothing to that ray (left out of both sums of Eq. 2); such
 * samples are counted (lf_cache_page_misses).
 *
 * lf_cache_config: (re)creates the cache with `pages` pages, emptying it.
 * Views [first_resident, n_views) (the coarse level of lf_two_level_mask;
 * n_views for none) are loaded into the first pages at once and never
 * evicted, so pages must exceed their tile count. Synchronous.
 * Errors: LF_ESTATE if the images are not paged; LF_EINVAL for sizes.
 */
int lf_cache_config(lf_ctx *c, int64_t pages, int32_t first_resident);

/*
 * One frame of tile streaming for the given eyes (arguments as lf_render):
 *   1. a visibility pass (the render's own disk tests and mesh walks over the
 *      fine views [0, first_resident), no sampling) marks every image tile
 *      holding one of the four taps of a sample;
 *   2. visible tiles not in the cache are copied in from host memory, view
 *      by view in index order, at most `budget` tiles per call (the paper's
 *      per-frame decode budget), each into the next page in FIFO order,
 *      evicting that page's tile; a page filled by this call is not reused
 *      by it;
 *   3. a fine view is available iff every tile it showed is in the cache,
 *      and the view mask (lf_set_view_mask) becomes the available fine views
 *      plus, with a coarse level, lf_two_level_mask's coarse fill-in (without
 *      one, the available views).
 * A following render of the same eyes then samples only cached tiles.
 * fine_available: host uint8 [first_resident] or NULL; visible_out: host uint8
 * [n_views][tiles] (the visibility pass, 1 = shown) or NULL; stats: host
 * int64 [5] or NULL = visible tiles, of them already cached, tiles copied in,
 * tiles evicted, fine views unavailable. Synchronous on hip_stream (waits for
 * the copies); it rewrites the view mask in stream order, so renders of this
 * context on other streams must not be in flight. Errors: LF_ESTATE without lf_cache_config or paged images;
 * LF_EINVAL as lf_render or for budget < 0.
 */
int lf_cache_update(lf_ctx *c, const lf_eye *eyes, int32_t n_eyes, double hfov_deg, const int32_t *res,
                    int32_t budget, uint8_t *fine_available, uint8_t *visible_out, int64_t *stats,
                    void *hip_stream);

/* Which image tiles are in the cache: host uint8 [n_views][tiles], 1 = cached. */
int lf_cache_resident(const lf_ctx *c, uint8_t *resident_out);

/* Samples left out since the last call because a tap's tile was not in the
 * cache (then resets the count). Synchronous. */
int lf_cache_page_misses(lf_ctx *c, uint64_t *misses);

/* Pixel reconstruction basis of the prefilter (one axis; the 2-D basis is the
 * product of two): box, 1 on |d| <= 1/2; Lanczos-2, sinc(d) sinc(d/2) on
 * |d| < 2 with sinc(x) = sin(pi x) / (pi x). */
enum { LF_BASIS_BOX = 0, LF_BASIS_LANCZOS2 = 1 };

/*
 * Light field prefilter (Sec. 5, Eqs. (4)-(5)). For every pixel (x, y) of each
 * listed view i the result is the Monte Carlo ratio estimate
 *
 *   sum_j a_j rho(du_j, dv_j) sigma(ds_j) sigma(dt_j) Lbar(o_j, e_j) / sum_j (same weights)
 *
 * with rho = 1 - |(du, dv)| the linear disk falloff and sigma the basis. The
 * ray of sample j starts at the point o_j = c_i + su_j du_j r_i + sv_j dv_j u_i
 * of view i's disk, the synthetic aperture of the real-time model (metres):
 * for the circle of radius `radius` su = sv = radius and a_j = 1; for an oval
 * disk (Sec. 4.4) with extents aperture_ext[k] = (e+u, e-u, e+v, e-v) of the
 * k-th listed view, su = e+u for du >= 0 and e-u otherwise, sv = e+v for
 * dv >= 0 and e-v otherwise, and a_j = su sv (a uniform point of the unit
 * disk lands in an oval quadrant with density 1 / (su sv); the factor keeps
 * the disk-area measure of Eq. (4)). The ray passes through the point of view i's mesh that view i sees at
 * image position (x + 1/2 + ds_j, y + 1/2 + dt_j) (pixel units). Lbar is the
 * query of Eq. (2) over the context's views, meshes and disks (the offline
 * model). A sample whose image position has no mesh point (outside the mesh
 * domain) or whose ray no disk of the context covers is left out of both
 * sums; a pixel with an empty denominator is (0, 0, 0). The same J samples
 * serve every pixel.
 *
 *   views      host int32 [n_views], indices of the views to prefilter (any order,
 *              repeats allowed); each is rendered at the context's image size
 *   radius     circle aperture radius in metres (> 0); unused with aperture_ext
 *   aperture_ext  host float64 [n_views][4] oval extents of the listed views
 *              (each finite and > 0, e.g. from lf_disk_extents), or NULL for circles
 *   disk_pts   host float64 [J][2], points of the unit disk (|p| <= 1)
 *   pix_offs   host float64 [J][2], offsets from the pixel centre in pixels (|.| <= 64)
 *   basis      LF_BASIS_BOX or LF_BASIS_LANCZOS2
 *   out_rgb    DEVICE float [n_views][img_h][img_w][3], overwritten
 *   out_wsum   DEVICE float [n_views][img_h][img_w], receives the denominator
 *
 * Source images must be square. Asynchronous on hip_stream; LF_EINVAL for a
 * NULL pointer, an empty list, a view index out of range, a non-positive
 * radius (circles) or extent (ovals), a disk point outside the unit disk or an
 * unknown basis.
 */
int lf_prefilter(lf_ctx *c, const int32_t *views, int32_t n_views, double radius, const double *aperture_ext,
                 const double *disk_pts, const double *pix_offs, int32_t n_samples, int32_t basis, float *out_rgb,
                 float *out_wsum, void *hip_stream);

/*
 * Offline reference render (the analogue of the high-quality offline query of
 * Sec. 5.1): ss x ss regular sub-pixel rays per pixel, disks of radius
 * disk_scale * R, box-averaged; a sub-ray no view covers counts as 0.
 * Same buffers and layout as lf_render (out_rgb only).
 */
int lf_render_reference(lf_ctx *c, const lf_eye *eyes, int32_t n_eyes, double hfov_deg, const int32_t *res,
                        int32_t ss, double disk_scale, float *out_rgb, void *hip_stream);

/*
 * Per-pixel view sets of one eye, for parity checks: out_cand[p][cap] lists
 * the views whose disk covers pixel p's centre ray (rho > 0), out_contrib[p][cap]
 * those of them whose mesh the ray hits, both ascending and padded with -1
 * (device int32 buffers of W*H*cap entries). out_ncand (device int32, may be
 * NULL) receives the full candidate count even when it exceeds cap.
 * The decisions are exactly the ones lf_render takes.
 */
int lf_debug_candidates(lf_ctx *c, const lf_eye *eye, double hfov_deg, int32_t W, int32_t H, int32_t cap,
                        int32_t *out_cand, int32_t *out_contrib, int32_t *out_ncand, void *hip_stream);

/*
 * Batched render: the same images as lf_render for n_eyes eyes of any sizes,
 * produced by ONE persistent launch in which every workgroup takes screen
 * tiles of all eyes from a global queue. The launch sequence (queue reset,
 * per-eye set-up, culling, persistent render) is captured once in a HIP graph
 * per batch shape (eye count, sizes, FOV, output buffers, tune) and replayed;
 * each call uploads only the eye poses. tune NULL = the context's tune (the
 * autotuned one after lf_autotune_batch, else 16x16 tiles).
 * Output layout as lf_render. Per-eye start / end stamps of the last batch are
 * read with lf_batch_frame_times.
 */
int lf_render_batch(lf_ctx *c, const lf_eye *eyes, int32_t n_eyes, double hfov_deg, const int32_t *res,
                    float *out_rgb, float *out_wsum, uint8_t *out_count, const lf_tune *tune, void *hip_stream);

/*
 * Autotuner of the batched path: times lf_render_batch on the given batch for
 * tiles {8x8, 16x16, 32x8} x candidate caps {8, 16, 32, 64} (median of reps
 * runs each, after a capture and warm-up run), stores the fastest in the
 * context and returns it in *best (may be NULL); ms[12] (may be NULL)
 * receives the medians, shape-major in that order. Synchronous.
 */
int lf_autotune_batch(lf_ctx *c, const lf_eye *eyes, int32_t n_eyes, double hfov_deg, const int32_t *res,
                      float *out_rgb, int32_t reps, lf_tune *best, float *ms, void *hip_stream);

/*
 * Device wall-clock stamps of the last batch: out_us[2k] / out_us[2k+1] are the
 * start of eye k's first tile and the end of its last tile, in microseconds
 * from the batch's first stamp. Synchronises the device. LF_ESTATE if the last
 * batch did not have n_eyes eyes.
 */
int lf_batch_frame_times(lf_ctx *c, double *out_us, int32_t n_eyes);

/*
 * Count the work one lf_render call with the same arguments performs (it runs
 * the same decisions without writing an image): counters[0] pixels,
 * [1] per-ray disk tests, [2] candidate (ray, view) pairs with rho > 0,
 * [3] mesh cells visited by the intersection walk, [4] contributing
 * (ray, view) pairs (bilinear samples). Synchronous on hip_stream.
 */
int lf_render_stats(lf_ctx *c, const lf_eye *eyes, int32_t n_eyes, double hfov_deg, const int32_t *res,
                    uint64_t counters[5], void *hip_stream);

/*
 * Per-kernel timing. lf_profile(c, 1) clears the totals and starts bracketing
 * every kernel the context launches with HIP events on the launch stream;
 * lf_profile(c, 0) stops. lf_profile_read waits for the recorded events and
 * returns the accumulated milliseconds of the set-up, cull and render kernels
 * in out[0..2] and their launch counts in out[3..5]. For lf_render_batch the
 * render entry is the persistent render kernel inside the batch graph (event
 * nodes around it, retargeted at every replay).
 */
int lf_profile(lf_ctx *c, int32_t enable);
int lf_profile_read(lf_ctx *c, double out[6]);

/*
 * Plain streaming copy of `bytes` from src to dst (both DEVICE, 16-byte
 * aligned, bytes a positive multiple of 16, not overlapping), 16-byte loads
 * and stores in a grid-stride loop; asynchronous on hip_stream. It reads and
 * writes every byte once, so timing it gives the achievable HBM bandwidth
 * that the render's measured traffic is compared with (not part of the
 * paper's method). Errors: LF_EINVAL for the conditions above.
 */
int lf_stream_copy(const void *src, void *dst, int64_t bytes, void *hip_stream);

/*
 * Vector FMA yardstick: `blocks` workgroups of 256 threads (four wavefronts);
 * the first `active` lanes of every wavefront run `iters` steps of eight
 * independent FP32 FMA chains (x = x * 0.999 + 0.001, chain k starting at
 * lane + k), the other lanes skip them; every thread writes the sum of its
 * eight values to out[block * 256 + thread] (DEVICE, blocks * 256 floats).
 * Asynchronous on hip_stream. Timing it gives the achievable rate of
 * wave-level FP32 FMA instructions with that many live lanes, which the
 * render kernel's vector instruction rate is compared with (not part of the
 * paper's method). Errors: LF_EINVAL for a NULL out, blocks < 1, iters < 1 or
 * active outside [1, 64].
 */
int lf_fma_rate(float *out, int32_t blocks, int32_t iters, int32_t active, void *hip_stream);

/* ---------------------------------------------------------------------------
 * Learned residual corrector (a post-process of the render; not in the paper,
 * whose learning-based methods are related work only, Sec. 2).
 *
 * Network: four 3x3 convolutions with zero padding, 5 -> 32 -> 32 -> 32 -> 3
 * channels, ReLU after the first three. Input per pixel: (R, G, B, W/4, n/8)
 * from lf_render's colour, weight sum W and view count n. Output: the
 * residual r; corrected pixel = render + r, except where max_c |r_c| >
 * fallback_thresh, which keep the render. Parameters: 20,835 FP32 values,
 * layer after layer, each layer w[ky][kx][ci][co] then b[co]. Kernels use
 * BF16 weights and activations with FP32 accumulation (MFMA); the master
 * parameters and Adam state are FP32.
 * Images: n_images equally sized images, eyes concatenated as lf_render
 * writes them (rgb [P][3] FP32, wsum [P] FP32, count [P] u8, all device).
 * ------------------------------------------------------------------------- */
typedef struct lf_corrector lf_corrector;

/* Create with the given parameters (host, 20,835 floats) or zeros (NULL). */
int lf_corrector_create(const float *params, lf_corrector **out);
/* Replace the parameters (host) and reset the optimiser state. */
int lf_corrector_set_params(lf_corrector *c, const float *params);
/* Copy the current FP32 parameters to host memory; *step (may be NULL) = optimiser steps taken. Synchronous. */
int lf_corrector_get_params(lf_corrector *c, float *params, int64_t *step);
/* Optimiser state for checkpoints: the FP32 master parameters, Adam's first
 * and second moments (20,835 floats each, host) and the number of steps
 * taken. get: synchronous copy out. set: replaces all of it (after the device
 * is idle), so training resumes exactly where the saved run was: the same
 * later steps on the same batches give the same parameters bit for bit.
 * LF_EINVAL for NULL pointers, a negative step, a value that is not finite or
 * a negative second moment. */
int lf_corrector_get_state(lf_corrector *c, float *params, float *adam_m, float *adam_v, int64_t *step);
int lf_corrector_set_state(lf_corrector *c, const float *params, const float *adam_m, const float *adam_v,
                           int64_t step);
/* Corrected images (device out_rgb [P][3]); out_fallback (device [P] u8, 1 =
 * kept the render) and out_resid (device [P][3] FP32) may be NULL. A
 * threshold of 0 returns the render exactly. Asynchronous on hip_stream.
 * The outputs must not overlap the inputs (rgb, wsum, count) or each other:
 * the kernel reads each tile's neighbourhood while other tiles are written
 * (no in-place correction); LF_EINVAL otherwise. */
int lf_corrector_apply(lf_corrector *c, const float *rgb, const float *wsum, const uint8_t *count, int32_t n_images,
                       int32_t W, int32_t H, float fallback_thresh, float *out_rgb, uint8_t *out_fallback,
                       float *out_resid, void *hip_stream);
/* One training step on a batch: loss = mean over pixels and channels of
 * (render + r - ref)^2 (ref device [P][3]); gradients by the backward kernels;
 * Adam (beta 0.9 / 0.999, eps 1e-8) with learning rate lr (lr = 0: gradients
 * only, no update). loss_out / grad_out (host, 20,835 floats) may be NULL;
 * when given the call synchronises. */
int lf_corrector_train_step(lf_corrector *c, const float *rgb, const float *wsum, const uint8_t *count,
                            const float *ref, int32_t n_images, int32_t W, int32_t H, float lr, float *loss_out,
                            float *grad_out, void *hip_stream);
/* Release (NULL is a no-op). */
void lf_corrector_free(lf_corrector *c);

/* Number of views, image and mesh sizes and formats of a context. */
int lf_query(const lf_ctx *c, int32_t *n_views, int32_t *img_w, int32_t *mesh_m, int32_t *img_fmt,
             int32_t *geo_fmt);

/* Thread-local message describing the last failure ("" if none). */
const char *lf_last_error(void);

/* Release a context and all its device memory (NULL is a no-op). */
void lf_free(lf_ctx *c);

#ifdef __cplusplus
}
#endif
#endif /* LF_H */
