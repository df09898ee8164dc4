// Internal interface between the C-ABI runtime (lf_api.cpp) and the HIP
// kernels (lf_kernels.hip). Not installed; not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lf.h"

namespace lf {

constexpr int kMaxEyesPerLaunch = 16;  // eye parameters travel in kernel arguments
constexpr int kListCap = 64;           // per-tile candidate list capacity (exact beyond: full scan)
constexpr int kBlk = 16;               // mesh cells per side of an inverse-depth bounds block
constexpr int kWin = 4;                // mesh cells per side of a window of the start-bound table
constexpr int kXcds = 8;               // XCDs of an MI355X (one L2 each)
constexpr int kQueueStride = 32;       // batch queue counters: one per XCD, 128 bytes apart
constexpr int kSuper = 4;              // screen tiles per side of a culling super-tile
constexpr int kSuperCap = 256;         // super-tile survivor list capacity (exact beyond: every view)
constexpr int kPage = 64;              // image tile (cache page) side in texels, paged images
constexpr int kPageShift = 6;

inline int num_blocks(int M) { return (M - 1 + kBlk - 1) / kBlk; }

// One eye of a launch. pos/rot feed the per-(eye, view) setup in FP64.
struct EyeParam {
    double pos[3];
    double rot[9];   // row-major, columns (r, u, f)
    float tx, ty;    // half-FOV tangents
    float sx, sy;    // image-plane pitch of one pixel: 2 tx / W, 2 ty / H
    int32_t W, H;
    int32_t tiles_x, tiles_y;
    int32_t tile_off;  // first tile of this eye within the launch
    int32_t supers_x, supers_y;
    int32_t super_off; // first culling super-tile of this eye within the launch
    int64_t pix_off;   // first output pixel of this eye
    // prefilter eyes (MODE_PREFILTER; src_view = -1 otherwise): the eye sits at a
    // point of view src_view's disk, displaced by (par_u, par_v) metres along the
    // view's r and u axes, with the view's frame and camera; the ray of pixel
    // (x, y) passes through the view's mesh point seen at (x + off_x, y + off_y)
    int32_t src_view;
    float off_x, off_y;
    float par_u, par_v;
    float pf_w;        // prefilter eyes: weight factor of the eye's sample (an oval quadrant's area; 1 for circles)
    // batches: first slot of this eye's band in each XCD's tile queue (band k
    // = tile rows [k tiles_y / kXcds, (k + 1) tiles_y / kXcds); queue x holds
    // band (x + e / 2) mod kXcds of eye e)
    int32_t band_off[kXcds];
};

struct EyeChunk {
    int32_t n_eyes;
    int32_t total_tiles;
    int32_t total_supers;
    int32_t pad;
    int32_t tile_w, tile_h;
    EyeParam e[kMaxEyesPerLaunch];
};

// Per (eye, view) record, 96 bytes: e' = M (X, Y, 1) is the eye ray in the
// view's frame, o' the eye centre in the view's frame; the view's mesh cells,
// image and inverse-depth blocks are addressed through the pointers here, so
// the render loop needs no per-view address arithmetic of its own.
struct alignas(16) EyeView {
    float m[9];
    float o[3];
    float wmin, wmax;  // inverse-depth range of the view's mesh
    int32_t view;
    float rk;          // radius bounding the view's disk, padded for the conservative tile test; < 0: view disabled
    const void *cells;  // this view's mesh cells
    const void *img;    // this view's image (YUV420: its luma plane)
    const float2 *blk;  // this view's inverse-depth blocks
    const void *img2;   // YUV420: this view's chroma plane (else unused)
};

// Where each view's data starts: base + view * stride (bytes; blocks in elements).
struct ViewBases {
    const char *geo, *img, *img2;
    const float2 *blk;
    int64_t geo_bytes, img_bytes, img2_bytes, blk_per_view;
    int64_t geo_head;  // bytes before each view's cells (its dequantisation constants)
};

// Mesh grid of the light field as the culling kernels need it: the grid
// transform, the inverse-depth blocks (prefilter eyes) and the window table
// from which each listed view of a tile gets the bound its rays' mesh walks
// start from: per mesh cell (j, k), an upper bound of the inverse depth over
// the cells [j, j + kWin) x [k, k + kWin) (FP16 bits, rounded up).
struct CullGeo {
    int32_t M, NB;
    float sM, cM;
    const uint16_t *win;   // [n][M-1][M-1]
    int64_t win_per_view;  // (M-1)^2
};

// Bound of every disk for culling: the radius of view v's disk is
// vrad[v] * vscale (oval disks: the largest of the four extents) or R
// (circles); both already include the disk scale of the call.
struct DiskBound {
    const float *vrad;  // [n] or null
    double R, vscale;
    const uint8_t *vmask;  // [n]: 0 = the view takes no part in renders (its record gets rk = -1); or null
};

// A batch: eye table in device memory (sorted by tile_off / super_off), the
// tile queues (kXcds counters, kQueueStride apart) and per-eye wall-clock
// stamps.
struct BatchArgs {
    const EyeParam *eyes;
    int32_t n_eyes, total_tiles, total_supers;
    int32_t tile_w, tile_h;
    unsigned int *queue;
    unsigned long long *frame_t;  // [n_eyes][2]: earliest tile start, latest tile end
    int32_t q_len[kXcds];         // slots of each XCD's queue (one band of every eye)
};

enum { MODE_RENDER = 0, MODE_SUBPIXEL = 1, MODE_DEBUG = 2, MODE_STATS = 3, MODE_PREFILTER = 4, MODE_VISIBILITY = 5 };
enum { DISK_CIRCLE = 0, DISK_OVAL = 1 };

struct RenderArgs {
    const EyeView *ev;          // [n_eyes][n_views]
    int32_t n_views;
    // [tiles][kListCap]: view index (low 16 bits) and the FP16 bits of an upper
    // bound of the view's mesh inverse depth over every cell a ray of the tile
    // can reach (high 16 bits; +inf: no bound)
    const uint32_t *tile_list;
    const int32_t *tile_count;  // [tiles]
    int32_t list_cap;           // a tile with more candidates than this takes the scan over every view
    int32_t NB;                 // inverse-depth blocks per side of a view's mesh
    int32_t M, img_w, img_h;
    float img_limx, img_limy;   // img_w - 1, img_h - 1 (clamp-to-edge limits of the texel coordinate)
    float sM, cM;               // grid coordinate g = X sM + cM (and cM - Y sM)
    float sW, cW, sH, cH;       // texel coordinate px = Xs sW + cW, py = cH - Ys sH
    float invR;                 // circular disks: 1 / radius
    const float4 *ext_inv;      // oval disks (null: circles): [n] 1/e+u, 1/e-u, 1/e+v, 1/e-v
    float ext_inv_scale;        // multiplies ext_inv (1 / disk scale)
    float *out_rgb;
    float *out_wsum;
    uint8_t *out_count;
    // sub-pixel (reference) passes: ray through (x + sub_x, y + sub_y); out += scale * L
    // prefilter passes: out += scale * L and out_wsum += scale where L is defined
    float sub_x, sub_y, scale;
    int32_t accumulate;
    // debug lists
    int32_t *dbg_cand, *dbg_contrib, *dbg_ncand;
    int32_t dbg_cap;
    // work counters: pixels, disk tests, candidates, mesh cells visited, samples
    unsigned long long *stats;
    // paged images: kPage x kPage-texel RGBA8 tiles in a cache of pages (pool,
    // 16 KB each); a view's record points at its row of the page table (page
    // of each image tile, row-major, -1 = not in the cache)
    const char *pool;
    int32_t tiles_x, tiles_y;       // image tiles per row / column
    uint8_t *vis;                   // visibility pass: [n_views][tiles] set to 1 where a tap lies
    unsigned int *page_miss;        // paged renders: samples left out for a tile not in the cache
};

// Record an error message for lf_last_error and return code (lf_api.cpp).
int fail_msg(int code, const char *msg);

// The device a context's data lives on (current when it was loaded).
int ctx_device(const lf_ctx *c);

// lf_render with the per-launch scratch (eye-view records, tile lists and
// counts) in the caller's device region [scratch, scratch + scratch_bytes)
// instead of the context's buffer: no device allocation. Every launch chunk
// is checked against scratch_bytes before the first launch (LF_EINVAL).
int render_fixed_scratch(lf_ctx *c, const lf_eye *eyes, int32_t n_eyes, double hfov_deg, const int32_t *res,
                         float *out_rgb, float *out_wsum, uint8_t *out_count, void *scratch, size_t scratch_bytes,
                         hipStream_t s);

// Launchers (lf_kernels.hip). All are asynchronous on `s` and return the
// launch status.
hipError_t launch_convert_images(const uint8_t *src, void *dst, int img_fmt, int64_t n_texels, hipStream_t s);
// RGBA8 [n][H][W] -> luma [n][H][W] and chroma [n][H/2][W/2][2] (H, W even)
hipError_t launch_convert_yuv420(const uint8_t *src, uint8_t *y, uint8_t *uv, int32_t n, int32_t W, int32_t H,
                                 hipStream_t s);
hipError_t launch_convert_rgtc(const uint8_t *y, const uint8_t *uv, void *yb, void *uvb, int32_t n, int32_t W,
                               int32_t H, hipStream_t s);
hipError_t launch_geo_cells(const float *z, void *cells, int geo_fmt, int32_t n, int32_t M, float2 *qr,
                            hipStream_t s);
hipError_t launch_geo_range(const void *cells, int geo_fmt, int32_t n, int32_t M, float2 *wr, hipStream_t s);
hipError_t launch_geo_blocks(const void *cells, int geo_fmt, int32_t n, int32_t M, float2 *blk, hipStream_t s);
// per mesh cell: the largest corner inverse depth of the kWin x kWin cells from it, FP16 rounded up
hipError_t launch_geo_win(const void *cells, int geo_fmt, int32_t n, int32_t M, uint16_t *win, hipStream_t s);
hipError_t launch_prep(const EyeChunk &ch, const double *vt, const float2 *wr, int32_t n, const DiskBound &db,
                       const ViewBases &vb, EyeView *ev, hipStream_t s);
// per-eye lists of the views the eye-level cull keeps (elist [n_eyes][n], ecount [n_eyes]), then the tile lists
hipError_t launch_cull(const EyeChunk &ch, const CullGeo &g, const EyeView *ev, int32_t n, uint16_t *elist,
                       int32_t *ecount, uint32_t *tile_list, int32_t *tile_count, hipStream_t s);
hipError_t launch_render(const EyeChunk &ch, const RenderArgs &a, int img_fmt, int geo_fmt, int mode,
                         hipStream_t s);
// reset + prep + cull + persistent render of a batch (a.ev / tile lists are the batch's buffers)
// ev_a / ev_b (may be null) are recorded just before / after the persistent render kernel
hipError_t launch_batch(const BatchArgs &b, const RenderArgs &a, const double *vt, const float2 *wr, int32_t n,
                        const DiskBound &db, const ViewBases &vb, const CullGeo &g, uint16_t *elist, int32_t *ecount,
                        int img_fmt, int geo_fmt, int grid, hipStream_t s, hipEvent_t ev_a, hipEvent_t ev_b);
// occupancy of the persistent render kernel (oval: the oval-disk form)
hipError_t persistent_occupancy(int img_fmt, int geo_fmt, bool oval, int block, int *per_cu);
// RGBA8 [n][H][W] device images -> kPage x kPage tiles, [n][tiles_y][tiles_x][kPage][kPage]
hipError_t launch_tile_images(const uint32_t *src, uint32_t *dst, int32_t n, int32_t W, int32_t H, hipStream_t s);
// keys[0, *count) = indices of the set bytes of vis[0, n), any order (*count must start at 0)
hipError_t launch_vis_compact(const uint8_t *vis, int64_t n, int32_t *keys, unsigned int *count, hipStream_t s);
// tile cache update: pt[patch[k].x] = patch[k].y for k < n_patch, then staged tile k (16 KB) -> page slot[k]
hipError_t launch_cache_apply(int32_t *pt, const int2 *patch, int32_t n_patch, const uint4 *staged,
                              const int32_t *slot, int32_t n_tiles, char *pool, hipStream_t s);
// out[p] /= wsum[p] (0 where wsum[p] == 0), p < n pixels of RGB
hipError_t launch_prefilter_finish(float *out_rgb, const float *wsum, int64_t n, hipStream_t s);

}  // namespace lf
