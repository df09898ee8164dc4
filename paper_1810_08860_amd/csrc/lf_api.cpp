// Host runtime of liblf.so: argument validation, device memory, eye set-up and
// kernel launches behind the C ABI declared in include/lf.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/lf.h"
#include "lf_internal.h"

using namespace lf;

thread_local std::string g_err;

namespace lf {
int fail_msg(int code, const char *msg) {
    g_err = msg;
    return code;
}
}  // namespace lf

namespace {

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(e == hipErrorOutOfMemory ? LF_ENOMEM : LF_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define LF_HIP(call, what)                          \
    do {                                            \
        hipError_t _e = (call);                     \
        if (_e != hipSuccess) return hip_fail(_e, what); \
    } while (0)

bool frame_ok(const double *R) {
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double s = 0.0;
            for (int r = 0; r < 3; ++r) s += R[3 * r + a] * R[3 * r + b];
            if (!std::isfinite(s) || std::fabs(s - (a == b ? 1.0 : 0.0)) > 1e-6) return false;
        }
    return true;
}

// bytes of one view's first image plane (YUV420: luma; RGTC: luma blocks)
// and of its second (the chroma plane or its blocks; none for RGBA)
int64_t img_view_bytes(int fmt, int64_t W, int64_t H) {
    switch (fmt) {
    case LF_IMG_RGBA8: return 4 * W * H;
    case LF_IMG_RGBA16F: return 8 * W * H;
    case LF_IMG_RGBA32F: return 16 * W * H;
    case LF_IMG_YUV420: return W * H;
    case LF_IMG_PAGED_RGBA8: return (W / kPage) * (H / kPage) * 4;  // the view's page-table row
    default: return (W / 4) * (H / 4) * 8;
    }
}
int64_t img2_view_bytes(int fmt, int64_t W, int64_t H) {
    if (fmt == LF_IMG_YUV420) return (W / 2) * (H / 2) * 2;
    if (fmt == LF_IMG_YUV420_RGTC) return (W / 8) * (H / 8) * 16;
    return 0;
}
size_t geo_bytes_per_cell(int fmt) { return fmt == LF_GEO_F32 ? 16 : 8; }
// bytes before each view's cells: the (base, scale) of its 16-bit codes
size_t geo_head_bytes(int fmt) { return fmt == LF_GEO_U16 ? 8 : 0; }

// Limits of the per-view addressing of the kernels (at<T>, mul24 in lf_ray.h).
constexpr int64_t kMaxViewBytes = (int64_t)1 << 32;
constexpr int64_t kMaxDim = (int64_t)1 << 24;

}  // namespace

struct lf_ctx {
    int device = 0;
    int32_t n = 0, img_w = 0, img_h = 0, M = 0;
    double src_fov_deg = 0.0, tan_s = 0.0, R = 0.0;
    int32_t img_fmt = 0, geo_fmt = 0;
    void *img = nullptr;     // device images in img_fmt (YUV420: the luma planes)
    void *img2 = nullptr;    // YUV420: the chroma planes
    void *geo = nullptr;     // device mesh cells in geo_fmt
    double *vt = nullptr;    // device [n][12]: centre, frame
    float2 *wr = nullptr;    // device [n]: inverse-depth range
    float2 *blk = nullptr;   // device [n][NB][NB]: inverse-depth range per block of cells
    uint16_t *win = nullptr;  // device [n][M-1][M-1]: per cell, FP16 bound over the kWin x kWin cells from it
    float4 *ext_inv = nullptr;  // device [n]: oval disks' inverse extents (null: circles of radius R)
    float *vrad = nullptr;      // device [n]: oval disks' largest extent (culling bound)
    uint8_t *vmask = nullptr;   // device [n]: views taking part in renders (lf_set_view_mask)
    // paged images (tile streaming): every image tile in pinned host memory,
    // a cache of device pages filled on demand (lf_cache_config / lf_cache_update);
    // img is then the device page table [n][tiles]
    struct Cache {
        uint32_t *host = nullptr;           // pinned [n][tiles][kPage * kPage] RGBA8
        int32_t tiles_x = 0, tiles_y = 0, tpv = 0;
        char *pool = nullptr;               // device pages, 16 KB each
        int64_t pages = 0, fixed = 0;       // pages; the first `fixed` hold the resident views
        int64_t next = 0;                   // FIFO position in [fixed, pages)
        int32_t first_resident = 0;         // views [first_resident, n) stay in the cache
        std::vector<int32_t> pt;            // host mirror of the page table
        std::vector<int64_t> owner;         // page -> tile key (view * tpv + tile), -1 = free
        std::vector<int64_t> stamp;         // page -> update call that filled it
        int64_t calls = 0;
        uint8_t *vis_dev = nullptr;         // visibility pass output [n][tiles]
        int32_t *keys_dev = nullptr;        // its set entries, compacted [n * tiles]
        unsigned int *count_host = nullptr; // pinned: number of keys (device-written count in count_host[0])
        unsigned int *count_dev = nullptr;
        uint8_t *mask_host = nullptr;       // pinned: view mask staging [n]
        std::vector<int32_t> vis_keys;      // visible tiles of the last update, ascending
        char *stage_host = nullptr, *stage_dev = nullptr;  // patches, pages, tiles of one update
        size_t stage_bytes = 0;
        unsigned int *miss_dev = nullptr;   // samples left out for a missing page
    } cache;
    std::vector<double> h_rad;  // host [n]: each disk's largest extent (R for circles)
    std::vector<double> h_vt;  // host copy of the view table (eye validation)
    // per-render scratch: eye-view table and tile lists, grown on demand
    void *scratch = nullptr;
    size_t scratch_bytes = 0;
    lf_tune tune{16, 16, kListCap};
    // optional per-kernel timing (lf_profile): event pairs around each launch
    struct Timed {
        int kind;
        hipEvent_t a, b;
    };
    bool profiling = false;
    std::vector<Timed> timed;
    double prof_ms[3] = {0, 0, 0};
    double prof_n[3] = {0, 0, 0};
    // batched path: one persistent launch per batch, captured in a HIP graph
    struct Batch {
        hipStream_t cap_stream = nullptr;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        std::string key;
        EyeParam *eyes_dev = nullptr;
        EyeParam *eyes_host = nullptr;  // pinned staging of the eye table
        int32_t eyes_cap = 0;
        hipEvent_t copied = nullptr;    // recorded after the last eye-table upload
        void *buf = nullptr;
        size_t buf_bytes = 0;
        unsigned long long *frame_t = nullptr;
        int32_t n_eyes = 0;
        // with profiling on, the graph holds event-record nodes around the
        // persistent render kernel; each replay points them at fresh events
        hipEvent_t ph_a = nullptr, ph_b = nullptr;
        hipGraphNode_t node_a = nullptr, node_b = nullptr;
        lf_tune tune{16, 16, kListCap};
        bool tuned = false;
    } batch;
};

namespace {

// Run `launch` on stream s, bracketed by events when profiling is on.
// kind: 0 = prep, 1 = cull, 2 = render.
template <class F>
hipError_t timed_launch(lf_ctx *c, int kind, hipStream_t s, F launch) {
    if (!c->profiling) return launch();
    lf_ctx::Timed t{kind, nullptr, nullptr};
    hipError_t e = hipEventCreate(&t.a);
    if (e == hipSuccess) e = hipEventCreate(&t.b);
    if (e == hipSuccess) e = hipEventRecord(t.a, s);
    if (e != hipSuccess) return e;
    e = launch();
    if (e != hipSuccess) return e;
    e = hipEventRecord(t.b, s);
    c->timed.push_back(t);
    return e;
}

int ensure_scratch(lf_ctx *c, size_t bytes) {
    if (bytes <= c->scratch_bytes) return LF_OK;
    if (c->scratch) {
        LF_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
        LF_HIP(hipFree(c->scratch), "hipFree");
        c->scratch = nullptr;
        c->scratch_bytes = 0;
    }
    size_t want = std::max(bytes, (size_t)1 << 20);
    LF_HIP(hipMalloc(&c->scratch, want), "hipMalloc(scratch)");
    c->scratch_bytes = want;
    return LF_OK;
}

int check_eyes(const lf_ctx *c, const lf_eye *eyes, int32_t n_eyes, double hfov_deg, const int32_t *res) {
    if (!eyes || !res) return fail(LF_EINVAL, "eyes and res must not be NULL");
    if (n_eyes <= 0) return fail(LF_EINVAL, "n_eyes must be positive (got %d)", n_eyes);
    if (!(hfov_deg > 0.0 && hfov_deg < 180.0)) return fail(LF_EINVAL, "hfov_deg must be in (0,180) (got %g)", hfov_deg);
    for (int32_t k = 0; k < n_eyes; ++k) {
        if (res[2 * k] <= 0 || res[2 * k + 1] <= 0 || res[2 * k] > 32768 || res[2 * k + 1] > 32768)
            return fail(LF_EINVAL, "eye %d: resolution %dx%d out of range", k, res[2 * k], res[2 * k + 1]);
        const lf_eye &E = eyes[k];
        for (int a = 0; a < 3; ++a)
            if (!std::isfinite(E.pos[a])) return fail(LF_EINVAL, "eye %d: position is not finite", k);
        if (!frame_ok(E.rot)) return fail(LF_EINVAL, "eye %d: frame is not orthonormal to 1e-6", k);
        // the eye must lie behind every disk plane (inside the capture surface)
        for (int32_t v = 0; v < c->n; ++v) {
            const double *vc = &c->h_vt[12 * (size_t)v];
            const double *R = vc + 3;
            double s = 0.0;
            for (int r = 0; r < 3; ++r) s += R[3 * r + 2] * (E.pos[r] - vc[r]);
            if (!(s < 0.0))
                return fail(LF_EINVAL, "eye %d lies on or in front of the disk plane of view %d", k, v);
        }
    }
    return LF_OK;
}

void fill_chunk(const lf_ctx *c, EyeChunk &ch, const lf_eye *eyes, int32_t n, double hfov_deg, const int32_t *res,
                int64_t pix_off, int tw, int th) {
    std::memset(&ch, 0, sizeof ch);
    ch.n_eyes = n;
    ch.tile_w = tw;
    ch.tile_h = th;
    const double tx = std::tan(0.5 * hfov_deg * M_PI / 180.0);
    int32_t tiles = 0, supers = 0;
    for (int32_t k = 0; k < n; ++k) {
        EyeParam &E = ch.e[k];
        std::memcpy(E.pos, eyes[k].pos, sizeof E.pos);
        std::memcpy(E.rot, eyes[k].rot, sizeof E.rot);
        E.W = res[2 * k];
        E.H = res[2 * k + 1];
        E.tx = (float)tx;
        E.ty = (float)(tx * E.H / E.W);
        E.sx = (float)(2.0 * tx / E.W);
        E.sy = (float)(2.0 * tx / E.W);  // square pixels: 2 ty / H = 2 tx / W
        E.tiles_x = (E.W + tw - 1) / tw;
        E.tiles_y = (E.H + th - 1) / th;
        E.tile_off = tiles;
        E.supers_x = (E.tiles_x + kSuper - 1) / kSuper;
        E.supers_y = (E.tiles_y + kSuper - 1) / kSuper;
        E.super_off = supers;
        E.pix_off = pix_off;
        E.src_view = -1;
        E.pf_w = 1.0f;
        tiles += E.tiles_x * E.tiles_y;
        supers += E.supers_x * E.supers_y;
        pix_off += (int64_t)E.W * E.H;
    }
    ch.total_tiles = tiles;
    ch.total_supers = supers;
}

RenderArgs base_args(const lf_ctx *c, double R) {
    RenderArgs a;
    std::memset(&a, 0, sizeof a);
    a.n_views = c->n;
    a.NB = num_blocks(c->M);
    a.M = c->M;
    a.img_w = c->img_w;
    a.img_h = c->img_h;
    a.img_limx = (float)(c->img_w - 1);
    a.img_limy = (float)(c->img_h - 1);
    a.sM = (float)(c->M / (2.0 * c->tan_s));
    a.cM = (float)(0.5 * (c->M - 1));
    a.sW = (float)(c->img_w / (2.0 * c->tan_s));
    a.cW = (float)(0.5 * (c->img_w - 1));
    a.sH = (float)(c->img_h / (2.0 * c->tan_s));
    a.cH = (float)(0.5 * (c->img_h - 1));
    a.invR = (float)(1.0 / R);
    // R is the context's radius times the call's disk scale; oval extents scale alike
    a.ext_inv = c->ext_inv;
    a.pool = c->cache.pool;
    a.tiles_x = c->cache.tiles_x;
    a.tiles_y = c->cache.tiles_y;
    a.vis = c->cache.vis_dev;
    a.page_miss = c->cache.miss_dev;
    a.ext_inv_scale = (float)(c->R / R);
    a.scale = 1.0f;
    a.list_cap = c->tune.cap;
    return a;
}

// Where each view's mesh cells, image and inverse-depth blocks start.
ViewBases view_bases(const lf_ctx *c) {
    ViewBases vb;
    vb.geo = static_cast<const char *>(c->geo);
    vb.img = static_cast<const char *>(c->img);
    vb.img2 = static_cast<const char *>(c->img2);
    vb.blk = c->blk;
    vb.geo_head = (int64_t)geo_head_bytes(c->geo_fmt);
    vb.geo_bytes = (int64_t)(c->M - 1) * (c->M - 1) * (int64_t)geo_bytes_per_cell(c->geo_fmt) + vb.geo_head;
    vb.img_bytes = img_view_bytes(c->img_fmt, c->img_w, c->img_h);
    vb.img2_bytes = img2_view_bytes(c->img_fmt, c->img_w, c->img_h);
    vb.blk_per_view = (int64_t)num_blocks(c->M) * num_blocks(c->M);
    return vb;
}

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

// Mesh grid and per-cell bounds for the culling kernels.
CullGeo cull_geo(const lf_ctx *c) {
    CullGeo g;
    g.M = c->M;
    g.NB = num_blocks(c->M);
    g.sM = (float)(c->M / (2.0 * c->tan_s));
    g.cM = (float)(0.5 * (c->M - 1));
    g.win = c->win;
    g.win_per_view = (int64_t)(c->M - 1) * (c->M - 1);
    return g;
}

// Device scratch of one launch chunk: eye-view records, per-eye view lists and
// counts, tile lists, tile counts.
size_t chunk_scratch_bytes(const lf_ctx *c, const EyeChunk &ch) {
    return al256(sizeof(EyeView) * (size_t)ch.n_eyes * c->n) + al256(sizeof(uint16_t) * (size_t)ch.n_eyes * c->n) +
           al256(sizeof(int32_t) * (size_t)ch.n_eyes) + al256(sizeof(uint32_t) * (size_t)kListCap * ch.total_tiles) +
           al256(sizeof(int32_t) * (size_t)ch.total_tiles);
}

// Prep + cull for one chunk of eyes; fills the table/list pointers of `a`.
// The chunk's scratch is the context's buffer (grown on demand), or the
// caller's region `fixed` (large enough: checked by the caller).
int prep_and_cull(lf_ctx *c, EyeChunk &ch, RenderArgs &a, double R, hipStream_t s, void *fixed = nullptr) {
    const size_t ev_bytes = sizeof(EyeView) * (size_t)ch.n_eyes * c->n;
    const size_t list_bytes = sizeof(uint32_t) * (size_t)kListCap * ch.total_tiles;
    auto al = al256;
    if (!fixed) {
        int rc = ensure_scratch(c, chunk_scratch_bytes(c, ch));
        if (rc) return rc;
    }
    char *p = fixed ? (char *)fixed : (char *)c->scratch;
    EyeView *ev = (EyeView *)p;
    p += al(ev_bytes);
    uint16_t *el = (uint16_t *)p;
    p += al(sizeof(uint16_t) * (size_t)ch.n_eyes * c->n);
    int32_t *ec = (int32_t *)p;
    p += al(sizeof(int32_t) * (size_t)ch.n_eyes);
    uint32_t *tl = (uint32_t *)p;
    int32_t *tc = (int32_t *)(p + al(list_bytes));
    // conservative disk bounds for the tile test; the exact per-ray test decides in k_render
    const DiskBound db{c->vrad, R, R / c->R, c->vmask};
    LF_HIP(timed_launch(c, 0, s, [&] { return launch_prep(ch, c->vt, c->wr, c->n, db, view_bases(c), ev, s); }), "k_prep launch");
    LF_HIP(timed_launch(c, 1, s, [&] { return launch_cull(ch, cull_geo(c), ev, c->n, el, ec, tl, tc, s); }), "k_cull launch");
    a.ev = ev;
    a.tile_list = tl;
    a.tile_count = tc;
    return LF_OK;
}

}  // namespace

extern "C" {

const char *lf_last_error(void) { return g_err.c_str(); }

int lf_stereo_eyes(const double head_pos[3], const double head_rot[9], double ipd_m, lf_eye out[2]) {
    if (!head_pos || !head_rot || !out) return fail(LF_EINVAL, "NULL argument");
    if (!std::isfinite(ipd_m) || ipd_m < 0.0) return fail(LF_EINVAL, "ipd must be finite and >= 0");
    if (!frame_ok(head_rot)) return fail(LF_EINVAL, "head frame is not orthonormal to 1e-6");
    for (int k = 0; k < 2; ++k) {
        const double sgn = k == 0 ? -0.5 : 0.5;
        for (int a = 0; a < 3; ++a) out[k].pos[a] = head_pos[a] + sgn * ipd_m * head_rot[3 * a + 0];
        std::memcpy(out[k].rot, head_rot, sizeof(double) * 9);
    }
    return LF_OK;
}

int lf_load_views(const lf_views_desc *d, lf_ctx **out) {
    if (!d || !out) return fail(LF_EINVAL, "NULL argument");
    *out = nullptr;
    if (d->n_views <= 0 || d->n_views > 65535) return fail(LF_EINVAL, "n_views must be in [1, 65535] (got %d)", d->n_views);
    if (d->img_w < 2 || d->img_h < 2) return fail(LF_EINVAL, "image size must be at least 2 x 2");
    if (d->img_w != d->img_h) return fail(LF_EINVAL, "source views must be square (got %dx%d)", d->img_w, d->img_h);
    if (d->mesh_m < 2 || d->mesh_m > 8192) return fail(LF_EINVAL, "mesh_m must be in [2, 8192] (got %d)", d->mesh_m);
    if (!(d->src_fov_deg > 0.0 && d->src_fov_deg < 180.0)) return fail(LF_EINVAL, "src_fov_deg must be in (0,180)");
    if (!(d->disk_radius > 0.0) || !std::isfinite(d->disk_radius)) return fail(LF_EINVAL, "disk_radius must be > 0");
    if (!d->centres || !d->rot || !d->rgba8 || !d->zdepth) return fail(LF_EINVAL, "NULL data pointer");
    if (d->img_fmt < LF_IMG_RGBA8 || d->img_fmt > LF_IMG_PAGED_RGBA8)
        return fail(LF_EINVAL, "unknown img_fmt %d", d->img_fmt);
    if (d->img_fmt == LF_IMG_PAGED_RGBA8 && (d->img_w % kPage || d->img_h % kPage))
        return fail(LF_EINVAL, "paged images need sizes that are multiples of %d (got %dx%d)", kPage, d->img_w,
                    d->img_h);
    if (d->img_fmt == LF_IMG_PAGED_RGBA8 &&
        (int64_t)d->n_views * (d->img_w / kPage) * (d->img_h / kPage) > INT32_MAX)
        return fail(LF_EINVAL, "paged images: more than 2^31 tiles in all");
    if (d->img_fmt == LF_IMG_YUV420 && (d->img_w % 2 || d->img_h % 2))
        return fail(LF_EINVAL, "YUV420 needs even image sizes (got %dx%d)", d->img_w, d->img_h);
    if (d->img_fmt == LF_IMG_YUV420_RGTC && (d->img_w % 8 || d->img_h % 8))
        return fail(LF_EINVAL, "RGTC needs image sizes that are multiples of 8 (got %dx%d)", d->img_w, d->img_h);
    if (d->geo_fmt < LF_GEO_F32 || d->geo_fmt > LF_GEO_U16) return fail(LF_EINVAL, "unknown geo_fmt %d", d->geo_fmt);
    if (d->flags & ~LF_SRC_DEVICE) return fail(LF_EINVAL, "unknown flags 0x%x", d->flags);
    {
        // the kernels address each view's share of an array with a 32-bit byte
        // offset and form texel indices with 24-bit products
        const int64_t W = d->img_w, H = d->img_h, Mc = d->mesh_m - 1;
        if (W >= kMaxDim || H >= kMaxDim)
            return fail(LF_EINVAL, "image size %lldx%lld: each dimension must be below 2^24", (long long)W,
                        (long long)H);
        const int64_t per_view[4] = {img_view_bytes(d->img_fmt, W, H), img2_view_bytes(d->img_fmt, W, H), 4 * W * H,
                                     Mc * Mc * (int64_t)geo_bytes_per_cell(d->geo_fmt) + (int64_t)geo_head_bytes(d->geo_fmt)};
        static const char *what[4] = {"image", "second image plane", "RGBA8 source image", "mesh"};
        for (int k = 0; k < 4; ++k)
            if (per_view[k] >= kMaxViewBytes)
                return fail(LF_EINVAL, "one view's %s takes %lld bytes; each view's share of an array must stay below 2^32 bytes",
                            what[k], (long long)per_view[k]);
    }
    const int32_t n = d->n_views, M = d->mesh_m;
    if (d->disk_ext)
        for (int64_t k = 0; k < 4 * (int64_t)n; ++k)
            if (!(d->disk_ext[k] > 0.0) || !std::isfinite(d->disk_ext[k]))
                return fail(LF_EINVAL, "view %d: oval disk extent %d is not finite and positive", (int)(k / 4),
                            (int)(k % 4));
    for (int32_t v = 0; v < n; ++v) {
        for (int a = 0; a < 3; ++a)
            if (!std::isfinite(d->centres[3 * v + a])) return fail(LF_EINVAL, "view %d: centre not finite", v);
        if (!frame_ok(d->rot + 9 * (size_t)v)) return fail(LF_EINVAL, "view %d: frame is not orthonormal to 1e-6", v);
    }
    const bool dev_src = d->flags & LF_SRC_DEVICE;
    const size_t n_z = (size_t)n * M * M;
    if (!dev_src) {
        for (size_t k = 0; k < n_z; ++k)
            if (!(d->zdepth[k] > 0.0f) || !std::isfinite(d->zdepth[k]))
                return fail(LF_EINVAL, "depth %zu (view %zu) is not finite and positive", k, k / ((size_t)M * M));
    }

    lf_ctx *c = new lf_ctx();
    auto bail = [&](int rc) {
        lf_free(c);
        return rc;
    };
    (void)hipGetDevice(&c->device);
    c->n = n;
    c->img_w = d->img_w;
    c->img_h = d->img_h;
    c->M = M;
    c->src_fov_deg = d->src_fov_deg;
    c->tan_s = std::tan(0.5 * d->src_fov_deg * M_PI / 180.0);
    c->R = d->disk_radius;
    c->img_fmt = d->img_fmt;
    c->geo_fmt = d->geo_fmt;
    c->h_vt.resize(12 * (size_t)n);
    for (int32_t v = 0; v < n; ++v) {
        std::memcpy(&c->h_vt[12 * (size_t)v], d->centres + 3 * (size_t)v, 3 * sizeof(double));
        std::memcpy(&c->h_vt[12 * (size_t)v + 3], d->rot + 9 * (size_t)v, 9 * sizeof(double));
    }
    hipError_t e;
    const size_t n_tex = (size_t)n * d->img_w * d->img_h;
    if ((e = hipMalloc(&c->vt, c->h_vt.size() * sizeof(double))) != hipSuccess) return bail(hip_fail(e, "hipMalloc(view table)"));
    if ((e = hipMalloc(&c->wr, sizeof(float2) * n)) != hipSuccess) return bail(hip_fail(e, "hipMalloc(w range)"));
    if ((e = hipMemcpy(c->vt, c->h_vt.data(), c->h_vt.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess)
        return bail(hip_fail(e, "copy view table"));
    c->h_rad.assign(n, d->disk_radius);
    if ((e = hipMalloc(&c->vmask, n)) != hipSuccess) return bail(hip_fail(e, "hipMalloc(view mask)"));
    if ((e = hipMemset(c->vmask, 1, n)) != hipSuccess) return bail(hip_fail(e, "hipMemset(view mask)"));
    if (d->disk_ext) {
        std::vector<float4> inv(n);
        std::vector<float> big(n);
        for (int32_t v = 0; v < n; ++v) {
            const double *x = d->disk_ext + 4 * (size_t)v;
            inv[v] = make_float4((float)(1.0 / x[0]), (float)(1.0 / x[1]), (float)(1.0 / x[2]), (float)(1.0 / x[3]));
            big[v] = (float)std::max(std::max(x[0], x[1]), std::max(x[2], x[3]));
            c->h_rad[v] = std::max(std::max(x[0], x[1]), std::max(x[2], x[3]));
        }
        if ((e = hipMalloc(&c->ext_inv, sizeof(float4) * n)) != hipSuccess) return bail(hip_fail(e, "hipMalloc(disks)"));
        if ((e = hipMalloc(&c->vrad, sizeof(float) * n)) != hipSuccess) return bail(hip_fail(e, "hipMalloc(disks)"));
        if ((e = hipMemcpy(c->ext_inv, inv.data(), sizeof(float4) * n, hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(c->vrad, big.data(), sizeof(float) * n, hipMemcpyHostToDevice)) != hipSuccess)
            return bail(hip_fail(e, "copy disks"));
    }

    // images: RGBA8 upload, converted on the device when another format is asked for
    void *rgba_dev = nullptr;
    bool rgba_owned = false;
    if (dev_src) {
        rgba_dev = (void *)d->rgba8;
    } else {
        if ((e = hipMalloc(&rgba_dev, n_tex * 4)) != hipSuccess) return bail(hip_fail(e, "hipMalloc(images)"));
        rgba_owned = true;
        if ((e = hipMemcpy(rgba_dev, d->rgba8, n_tex * 4, hipMemcpyHostToDevice)) != hipSuccess) {
            (void)hipFree(rgba_dev);
            return bail(hip_fail(e, "copy images"));
        }
    }
    if (d->img_fmt == LF_IMG_RGBA8) {
        if (rgba_owned) {
            c->img = rgba_dev;
        } else {
            if ((e = hipMalloc(&c->img, n_tex * 4)) != hipSuccess) return bail(hip_fail(e, "hipMalloc(images)"));
            if ((e = hipMemcpy(c->img, rgba_dev, n_tex * 4, hipMemcpyDeviceToDevice)) != hipSuccess)
                return bail(hip_fail(e, "copy images"));
        }
    } else if (d->img_fmt == LF_IMG_YUV420) {
        if ((e = hipMalloc(&c->img, n_tex)) != hipSuccess || (e = hipMalloc(&c->img2, n_tex / 2)) != hipSuccess) {
            if (rgba_owned) (void)hipFree(rgba_dev);
            return bail(hip_fail(e, "hipMalloc(YUV420 planes)"));
        }
        e = launch_convert_yuv420((const uint8_t *)rgba_dev, (uint8_t *)c->img, (uint8_t *)c->img2, n, d->img_w,
                                  d->img_h, 0);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (rgba_owned) (void)hipFree(rgba_dev);
        if (e != hipSuccess) return bail(hip_fail(e, "YUV420 conversion"));
    } else if (d->img_fmt == LF_IMG_PAGED_RGBA8) {
        // tiles cut on the device, kept in pinned host memory; the device holds
        // the page table (every tile absent until lf_cache_config / lf_cache_update)
        if (((uintptr_t)rgba_dev & 15) != 0) {
            if (rgba_owned) (void)hipFree(rgba_dev);
            return bail(fail(LF_EINVAL, "paged images: the device RGBA8 source must be 16-byte aligned"));
        }
        lf_ctx::Cache &K = c->cache;
        K.tiles_x = d->img_w / kPage;
        K.tiles_y = d->img_h / kPage;
        K.tpv = K.tiles_x * K.tiles_y;
        void *tiled = nullptr;
        if ((e = hipMalloc(&tiled, n_tex * 4)) != hipSuccess ||
            (e = hipHostMalloc((void **)&K.host, n_tex * 4, hipHostMallocDefault)) != hipSuccess ||
            (e = hipMalloc(&c->img, sizeof(int32_t) * (size_t)n * K.tpv)) != hipSuccess) {
            if (tiled) (void)hipFree(tiled);
            if (rgba_owned) (void)hipFree(rgba_dev);
            return bail(hip_fail(e, "allocating paged images"));
        }
        e = launch_tile_images((const uint32_t *)rgba_dev, (uint32_t *)tiled, n, d->img_w, d->img_h, 0);
        if (e == hipSuccess) e = hipMemcpy(K.host, tiled, n_tex * 4, hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = hipMemset(c->img, 0xff, sizeof(int32_t) * (size_t)n * K.tpv);
        (void)hipFree(tiled);
        if (rgba_owned) (void)hipFree(rgba_dev);
        if (e != hipSuccess) return bail(hip_fail(e, "tiling paged images"));
        K.pt.assign((size_t)n * K.tpv, -1);
    } else if (d->img_fmt == LF_IMG_YUV420_RGTC) {
        // RGBA8 -> YUV420 planes (scratch) -> RGTC blocks
        uint8_t *yp = nullptr, *uvp = nullptr;
        if ((e = hipMalloc(&c->img, (size_t)n * img_view_bytes(d->img_fmt, d->img_w, d->img_h))) != hipSuccess ||
            (e = hipMalloc(&c->img2, (size_t)n * img2_view_bytes(d->img_fmt, d->img_w, d->img_h))) != hipSuccess ||
            (e = hipMalloc(&yp, n_tex)) != hipSuccess || (e = hipMalloc(&uvp, n_tex / 2)) != hipSuccess) {
            if (yp) (void)hipFree(yp);
            if (rgba_owned) (void)hipFree(rgba_dev);
            return bail(hip_fail(e, "hipMalloc(RGTC planes)"));
        }
        e = launch_convert_yuv420((const uint8_t *)rgba_dev, yp, uvp, n, d->img_w, d->img_h, 0);
        if (e == hipSuccess) e = launch_convert_rgtc(yp, uvp, c->img, c->img2, n, d->img_w, d->img_h, 0);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        (void)hipFree(yp);
        (void)hipFree(uvp);
        if (rgba_owned) (void)hipFree(rgba_dev);
        if (e != hipSuccess) return bail(hip_fail(e, "RGTC conversion"));
    } else {
        if ((e = hipMalloc(&c->img, n_tex * (size_t)img_view_bytes(d->img_fmt, 1, 1))) != hipSuccess) {
            if (rgba_owned) (void)hipFree(rgba_dev);
            return bail(hip_fail(e, "hipMalloc(converted images)"));
        }
        e = launch_convert_images((const uint8_t *)rgba_dev, c->img, d->img_fmt, (int64_t)n_tex, 0);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (rgba_owned) (void)hipFree(rgba_dev);
        if (e != hipSuccess) return bail(hip_fail(e, "image conversion"));
    }

    // geometry: z -> per-cell inverse-depth corners, then per-view range
    float *z_dev = nullptr;
    bool z_owned = false;
    if (dev_src) {
        z_dev = (float *)d->zdepth;
    } else {
        if ((e = hipMalloc(&z_dev, n_z * sizeof(float))) != hipSuccess) return bail(hip_fail(e, "hipMalloc(depth)"));
        z_owned = true;
        if ((e = hipMemcpy(z_dev, d->zdepth, n_z * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess) {
            (void)hipFree(z_dev);
            return bail(hip_fail(e, "copy depth"));
        }
    }
    const size_t n_cells = (size_t)n * (M - 1) * (M - 1);
    if ((e = hipMalloc(&c->geo, n_cells * geo_bytes_per_cell(d->geo_fmt) + (size_t)n * geo_head_bytes(d->geo_fmt))) !=
        hipSuccess) {
        if (z_owned) (void)hipFree(z_dev);
        return bail(hip_fail(e, "hipMalloc(mesh cells)"));
    }
    const int NB = num_blocks(M);
    if ((e = hipMalloc(&c->blk, sizeof(float2) * (size_t)n * NB * NB)) != hipSuccess) {
        if (z_owned) (void)hipFree(z_dev);
        return bail(hip_fail(e, "hipMalloc(block bounds)"));
    }
    if ((e = hipMalloc(&c->win, sizeof(uint16_t) * n_cells)) != hipSuccess) {
        if (z_owned) (void)hipFree(z_dev);
        return bail(hip_fail(e, "hipMalloc(cell bounds)"));
    }
    // (c->wr first holds the FP32 inverse-depth range the 16-bit codes span)
    e = launch_geo_cells(z_dev, c->geo, d->geo_fmt, n, M, c->wr, 0);
    if (e == hipSuccess) e = launch_geo_range(c->geo, d->geo_fmt, n, M, c->wr, 0);
    if (e == hipSuccess) e = launch_geo_blocks(c->geo, d->geo_fmt, n, M, c->blk, 0);
    if (e == hipSuccess) e = launch_geo_win(c->geo, d->geo_fmt, n, M, c->win, 0);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (z_owned) (void)hipFree(z_dev);
    if (e != hipSuccess) return bail(hip_fail(e, "geometry conversion"));
    *out = c;
    return LF_OK;
}

// A launch shape with its cap resolved (0 = kListCap); false if invalid.
static bool tune_ok(const lf_tune &t, lf_tune &out) {
    if (t.tile_w <= 0 || t.tile_h <= 0 || t.tile_w % 8 || t.tile_h % 8 || t.tile_w * t.tile_h > 256) return false;
    if (t.cap < 0 || t.cap > kListCap) return false;
    out = t;
    if (out.cap == 0) out.cap = kListCap;
    return true;
}

int lf_set_tune(lf_ctx *c, const lf_tune *t) {
    if (!c) return fail(LF_EINVAL, "NULL context");
    if (!t) {
        c->tune = lf_tune{16, 16, kListCap};
        return LF_OK;
    }
    lf_tune r;
    if (!tune_ok(*t, r))
        return fail(LF_EINVAL, "tile must be multiples of 8 with at most 256 pixels and cap in [0, %d] (got %dx%d, %d)",
                    kListCap, t->tile_w, t->tile_h, t->cap);
    c->tune = r;
    return LF_OK;
}

int lf_query(const lf_ctx *c, int32_t *n_views, int32_t *img_w, int32_t *mesh_m, int32_t *img_fmt, int32_t *geo_fmt) {
    if (!c) return fail(LF_EINVAL, "NULL context");
    if (n_views) *n_views = c->n;
    if (img_w) *img_w = c->img_w;
    if (mesh_m) *mesh_m = c->M;
    if (img_fmt) *img_fmt = c->img_fmt;
    if (geo_fmt) *geo_fmt = c->geo_fmt;
    return LF_OK;
}

static int render_impl(lf_ctx *c, const lf_eye *eyes, int32_t n_eyes, double hfov_deg, const int32_t *res,
                       float *out_rgb, float *out_wsum, uint8_t *out_count, int mode, double R, float sub_x,
                       float sub_y, float scale, int accumulate, hipStream_t s,
                       unsigned long long *stats = nullptr, void *fixed = nullptr) {
    int64_t pix_off = 0;
    for (int32_t k0 = 0; k0 < n_eyes; k0 += kMaxEyesPerLaunch) {
        const int32_t nk = std::min(kMaxEyesPerLaunch, n_eyes - k0);
        EyeChunk ch;
        fill_chunk(c, ch, eyes + k0, nk, hfov_deg, res + 2 * k0, pix_off, c->tune.tile_w, c->tune.tile_h);
        RenderArgs a = base_args(c, R);
        a.list_cap = c->tune.cap;
        int rc = prep_and_cull(c, ch, a, R, s, fixed);
        if (rc) return rc;
        a.out_rgb = out_rgb;
        a.out_wsum = out_wsum;
        a.out_count = out_count;
        a.sub_x = sub_x;
        a.sub_y = sub_y;
        a.scale = scale;
        a.accumulate = accumulate;
        a.stats = stats;
        LF_HIP(timed_launch(c, 2, s, [&] { return launch_render(ch, a, c->img_fmt, c->geo_fmt, mode, s); }),
               "k_render launch");
        for (int32_t k = 0; k < nk; ++k) pix_off += (int64_t)res[2 * (k0 + k)] * res[2 * (k0 + k) + 1];
    }
    return LF_OK;
}

int lf_render(lf_ctx *c, const lf_eye *eyes, int32_t n_eyes, double hfov_deg, const int32_t *res, float *out_rgb,
              float *out_wsum, uint8_t *out_count, void *hip_stream) {
    if (!c) return fail(LF_EINVAL, "NULL context");
    if (!out_rgb) return fail(LF_EINVAL, "out_rgb must not be NULL");
    int rc = check_eyes(c, eyes, n_eyes, hfov_deg, res);
    if (rc) return rc;
    return render_impl(c, eyes, n_eyes, hfov_deg, res, out_rgb, out_wsum, out_count, MODE_RENDER, c->R, 0.5f, 0.5f,
                       1.0f, 0, (hipStream_t)hip_stream);
}

}  // extern "C"

namespace lf {

int ctx_device(const lf_ctx *c) { return c->device; }

int render_fixed_scratch(lf_ctx *c, const lf_eye *eyes, int32_t n_eyes, double hfov_deg, const int32_t *res,
                         float *out_rgb, float *out_wsum, uint8_t *out_count, void *scratch, size_t scratch_bytes,
                         hipStream_t s) {
    if (!c) return fail(LF_EINVAL, "NULL context");
    if (!out_rgb) return fail(LF_EINVAL, "out_rgb must not be NULL");
    int rc = check_eyes(c, eyes, n_eyes, hfov_deg, res);
    if (rc) return rc;
    // every launch chunk must fit before anything is launched
    int64_t pix_off = 0;
    for (int32_t k0 = 0; k0 < n_eyes; k0 += kMaxEyesPerLaunch) {
        const int32_t nk = std::min(kMaxEyesPerLaunch, n_eyes - k0);
        EyeChunk ch;
        fill_chunk(c, ch, eyes + k0, nk, hfov_deg, res + 2 * k0, pix_off, c->tune.tile_w, c->tune.tile_h);
        const size_t need = chunk_scratch_bytes(c, ch);
        if (need > scratch_bytes)
            return fail(LF_EINVAL,
                        "eyes %d..%d need %zu bytes of scratch (eye-view records and tile lists); the fixed scratch "
                        "holds %zu bytes: render fewer or smaller eyes per call",
                        k0, k0 + nk - 1, need, scratch_bytes);
        for (int32_t k = 0; k < nk; ++k) pix_off += (int64_t)res[2 * (k0 + k)] * res[2 * (k0 + k) + 1];
    }
    // kernel launches only (no per-kernel timing events)
    const bool prof = c->profiling;
    c->profiling = false;
    rc = render_impl(c, eyes, n_eyes, hfov_deg, res, out_rgb, out_wsum, out_count, MODE_RENDER, c->R, 0.5f, 0.5f,
                     1.0f, 0, s, nullptr, scratch);
    c->profiling = prof;
    return rc;
}

}  // namespace lf

extern "C" {

int lf_render_reference(lf_ctx *c, const lf_eye *eyes, int32_t n_eyes, double hfov_deg, const int32_t *res,
                        int32_t ss, double disk_scale, float *out_rgb, void *hip_stream) {
    if (!c) return fail(LF_EINVAL, "NULL context");
    if (!out_rgb) return fail(LF_EINVAL, "out_rgb must not be NULL");
    if (ss < 1 || ss > 16) return fail(LF_EINVAL, "ss must be in [1,16] (got %d)", ss);
    if (!(disk_scale > 0.0) || !std::isfinite(disk_scale)) return fail(LF_EINVAL, "disk_scale must be > 0");
    int rc = check_eyes(c, eyes, n_eyes, hfov_deg, res);
    if (rc) return rc;
    const float scale = 1.0f / (float)(ss * ss);
    for (int32_t sy = 0; sy < ss; ++sy)
        for (int32_t sx = 0; sx < ss; ++sx) {
            rc = render_impl(c, eyes, n_eyes, hfov_deg, res, out_rgb, nullptr, nullptr, MODE_SUBPIXEL,
                             c->R * disk_scale, (sx + 0.5f) / ss, (sy + 0.5f) / ss, scale, (sx | sy) != 0,
                             (hipStream_t)hip_stream);
            if (rc) return rc;
        }
    return LF_OK;
}

// One axis of the prefilter's pixel reconstruction basis (Sec. 5.1): box or
// Lanczos-2, sinc(x) sinc(x / 2) on |x| < 2.
static double basis_weight(int32_t basis, double x) {
    x = std::fabs(x);
    if (basis == LF_BASIS_BOX) return x <= 0.5 ? 1.0 : 0.0;
    if (x >= 2.0) return 0.0;
    if (x == 0.0) return 1.0;
    const double px = M_PI * x;
    return std::sin(px) / px * (std::sin(0.5 * px) / (0.5 * px));
}

int lf_set_view_mask(lf_ctx *c, const uint8_t *enabled) {
    if (!c) return fail(LF_EINVAL, "NULL context");
    std::vector<uint8_t> m(c->n, 1);
    if (enabled)
        for (int32_t v = 0; v < c->n; ++v) m[v] = enabled[v] ? 1 : 0;
    // renders already queued on other streams may still read the mask
    LF_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
    LF_HIP(hipMemcpy(c->vmask, m.data(), c->n, hipMemcpyHostToDevice), "copy view mask");
    return LF_OK;
}

int lf_two_level_mask(const lf_ctx *c, int32_t n_fine, const uint8_t *fine_available, uint8_t *mask_out) {
    if (!c) return fail(LF_EINVAL, "NULL context");
    if (!fine_available || !mask_out) return fail(LF_EINVAL, "fine_available and mask_out must not be NULL");
    if (n_fine <= 0 || n_fine > c->n) return fail(LF_EINVAL, "n_fine must be in [1, n_views] (got %d)", n_fine);
    std::vector<int32_t> missing;  // unavailable fine views (usually few or none)
    for (int32_t v = 0; v < n_fine; ++v) {
        mask_out[v] = fine_available[v] ? 1 : 0;
        if (!fine_available[v]) missing.push_back(v);
    }
    for (int32_t j = n_fine; j < c->n; ++j) {
        const double *cj = &c->h_vt[12 * (size_t)j];
        uint8_t need = 0;
        for (size_t q = 0; q < missing.size() && !need; ++q) {
            const int32_t i = missing[q];
            const double *ci = &c->h_vt[12 * (size_t)i];
            const double dx = ci[0] - cj[0], dy = ci[1] - cj[1], dz = ci[2] - cj[2];
            need = dx * dx + dy * dy + dz * dz < c->h_rad[j] * c->h_rad[j];
        }
        mask_out[j] = need;
    }
    return LF_OK;
}

int lf_cache_config(lf_ctx *c, int64_t pages, int32_t first_resident) {
    if (!c) return fail(LF_EINVAL, "NULL context");
    if (c->img_fmt != LF_IMG_PAGED_RGBA8) return fail(LF_ESTATE, "the context's images are not paged");
    lf_ctx::Cache &K = c->cache;
    if (first_resident < 0 || first_resident > c->n)
        return fail(LF_EINVAL, "first_resident must be in [0, n_views] (got %d)", first_resident);
    const int64_t fixed = (int64_t)(c->n - first_resident) * K.tpv;
    if (pages <= fixed || pages > ((int64_t)1 << 26))
        return fail(LF_EINVAL, "pages must exceed the %lld pages of the resident views and be at most 2^26 (got %lld)",
                    (long long)fixed, (long long)pages);
    LF_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
    if (K.pool) {
        LF_HIP(hipFree(K.pool), "hipFree");
        K.pool = nullptr;
    }
    const size_t page_bytes = (size_t)kPage * kPage * 4;
    LF_HIP(hipMalloc((void **)&K.pool, page_bytes * pages), "hipMalloc(tile cache)");
    if (!K.vis_dev) LF_HIP(hipMalloc((void **)&K.vis_dev, (size_t)c->n * K.tpv), "hipMalloc(visibility)");
    if (!K.keys_dev)
        LF_HIP(hipMalloc((void **)&K.keys_dev, sizeof(int32_t) * ((size_t)c->n * K.tpv)), "hipMalloc(visible keys)");
    if (!K.count_dev) LF_HIP(hipMalloc((void **)&K.count_dev, sizeof(unsigned int)), "hipMalloc(key count)");
    if (!K.count_host)
        LF_HIP(hipHostMalloc((void **)&K.count_host, sizeof(unsigned int), hipHostMallocDefault), "hipHostMalloc(key count)");
    if (!K.mask_host)
        LF_HIP(hipHostMalloc((void **)&K.mask_host, (size_t)c->n, hipHostMallocDefault), "hipHostMalloc(mask)");
    if (!K.miss_dev) {
        LF_HIP(hipMalloc((void **)&K.miss_dev, sizeof(unsigned int)), "hipMalloc(page misses)");
        LF_HIP(hipMemset(K.miss_dev, 0, sizeof(unsigned int)), "hipMemset");
    }
    K.pages = pages;
    K.fixed = fixed;
    K.next = fixed;
    K.first_resident = first_resident;
    K.owner.assign((size_t)pages, -1);
    K.stamp.assign((size_t)pages, -1);
    std::fill(K.pt.begin(), K.pt.end(), -1);
    // the resident views' tiles take the first pages, in order (contiguous in the host store)
    for (int64_t k = 0; k < fixed; ++k) {
        const int64_t key = (int64_t)first_resident * K.tpv + k;
        K.pt[(size_t)key] = (int32_t)k;
        K.owner[(size_t)k] = key;
    }
    if (fixed > 0)
        LF_HIP(hipMemcpy(K.pool, K.host + (size_t)first_resident * K.tpv * kPage * kPage, page_bytes * fixed,
                         hipMemcpyHostToDevice),
               "copy resident tiles");
    LF_HIP(hipMemcpy(c->img, K.pt.data(), sizeof(int32_t) * K.pt.size(), hipMemcpyHostToDevice), "copy page table");
    return LF_OK;
}

int lf_cache_update(lf_ctx *c, const lf_eye *eyes, int32_t n_eyes, double hfov_deg, const int32_t *res,
                    int32_t budget, uint8_t *fine_available, uint8_t *visible_out, int64_t *stats,
                    void *hip_stream) {
    if (!c) return fail(LF_EINVAL, "NULL context");
    if (c->img_fmt != LF_IMG_PAGED_RGBA8) return fail(LF_ESTATE, "the context's images are not paged");
    lf_ctx::Cache &K = c->cache;
    if (!K.pool) return fail(LF_ESTATE, "lf_cache_config has not been called");
    if (budget < 0) return fail(LF_EINVAL, "budget must be >= 0 (got %d)", budget);
    int rc = check_eyes(c, eyes, n_eyes, hfov_deg, res);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)hip_stream;
    const int32_t n = c->n, nf = K.first_resident;
    const size_t page_bytes = (size_t)kPage * kPage * 4;
    ++K.calls;

    // 1. visibility pass over the fine views (the resident ones need nothing);
    // its set bytes come back as a compacted list of tile keys
    uint8_t *m = K.mask_host;
    for (int32_t v = 0; v < n; ++v) m[v] = v < nf ? 1 : 0;
    LF_HIP(hipMemcpyAsync(c->vmask, m, (size_t)n, hipMemcpyHostToDevice, s), "copy view mask");
    LF_HIP(hipMemsetAsync(K.vis_dev, 0, (size_t)n * K.tpv, s), "hipMemsetAsync");
    LF_HIP(hipMemsetAsync(K.count_dev, 0, sizeof(unsigned int), s), "hipMemsetAsync");
    rc = render_impl(c, eyes, n_eyes, hfov_deg, res, nullptr, nullptr, nullptr, MODE_VISIBILITY, c->R, 0.5f, 0.5f,
                     1.0f, 0, s);
    if (rc) return rc;
    LF_HIP(launch_vis_compact(K.vis_dev, (int64_t)n * K.tpv, K.keys_dev, K.count_dev, s), "k_vis_compact launch");
    LF_HIP(hipMemcpyAsync(K.count_host, K.count_dev, sizeof(unsigned int), hipMemcpyDeviceToHost, s), "copy key count");
    LF_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
    K.vis_keys.resize(*K.count_host);
    if (!K.vis_keys.empty()) {
        LF_HIP(hipMemcpyAsync(K.vis_keys.data(), K.keys_dev, sizeof(int32_t) * K.vis_keys.size(),
                              hipMemcpyDeviceToHost, s),
               "copy visible keys");
        LF_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
    }
    std::sort(K.vis_keys.begin(), K.vis_keys.end());  // view by view, tile by tile

    // 2. FIFO: fill pages with visible tiles not in the cache, view by view, up
    // to the budget; a page filled by this call is never taken again by it
    int64_t hits = 0, evicted = 0;
    const int64_t visible = (int64_t)K.vis_keys.size();
    std::vector<int64_t> touched;  // page-table entries changed by this call
    std::vector<int32_t> slots;
    std::vector<int64_t> keys;
    const int64_t ring = K.pages - K.fixed;
    for (const int32_t k32 : K.vis_keys) {
        const int64_t key = k32;
        if (K.pt[(size_t)key] >= 0) {
            ++hits;
            continue;
        }
        if ((int64_t)slots.size() >= budget || (int64_t)slots.size() >= ring) continue;
        const int64_t pg = K.next;
        if (K.stamp[(size_t)pg] == K.calls) continue;  // the ring is full of this call's tiles
        K.next = K.next + 1 < K.pages ? K.next + 1 : K.fixed;
        const int64_t old = K.owner[(size_t)pg];
        if (old >= 0) {
            K.pt[(size_t)old] = -1;
            touched.push_back(old);
            ++evicted;
        }
        K.owner[(size_t)pg] = key;
        K.stamp[(size_t)pg] = K.calls;
        K.pt[(size_t)key] = (int32_t)pg;
        touched.push_back(key);
        slots.push_back((int32_t)pg);
        keys.push_back(key);
    }
    // each changed entry once, with its final value (an entry evicted and
    // filled again by this call appears twice in `touched`)
    std::sort(touched.begin(), touched.end());
    touched.erase(std::unique(touched.begin(), touched.end()), touched.end());
    std::vector<int2> patch(touched.size());
    for (size_t k = 0; k < touched.size(); ++k) patch[k] = make_int2((int)touched[k], K.pt[(size_t)touched[k]]);

    // 3. one upload: patches, pages, then the tiles; applied by one kernel
    const size_t off_slot = ((patch.size() * sizeof(int2)) + 15) & ~(size_t)15;
    const size_t off_tiles = (off_slot + slots.size() * sizeof(int32_t) + 255) & ~(size_t)255;
    const size_t need = off_tiles + slots.size() * page_bytes;
    if (need > K.stage_bytes) {
        if (K.stage_host) (void)hipHostFree(K.stage_host);
        if (K.stage_dev) (void)hipFree(K.stage_dev);
        K.stage_host = K.stage_dev = nullptr;
        K.stage_bytes = 0;
        const size_t want = std::max(need, (size_t)1 << 20);
        LF_HIP(hipHostMalloc((void **)&K.stage_host, want, hipHostMallocDefault), "hipHostMalloc(tile staging)");
        LF_HIP(hipMalloc((void **)&K.stage_dev, want), "hipMalloc(tile staging)");
        K.stage_bytes = want;
    }
    if (!patch.empty()) {
        std::memcpy(K.stage_host, patch.data(), patch.size() * sizeof(int2));
        std::memcpy(K.stage_host + off_slot, slots.data(), slots.size() * sizeof(int32_t));
        for (size_t k = 0; k < keys.size(); ++k)
            std::memcpy(K.stage_host + off_tiles + k * page_bytes, K.host + (size_t)keys[k] * kPage * kPage, page_bytes);
        LF_HIP(hipMemcpyAsync(K.stage_dev, K.stage_host, need, hipMemcpyHostToDevice, s), "copy tiles");
        LF_HIP(launch_cache_apply((int32_t *)c->img, (const int2 *)K.stage_dev, (int32_t)patch.size(),
                                  (const uint4 *)(K.stage_dev + off_tiles), (const int32_t *)(K.stage_dev + off_slot),
                                  (int32_t)slots.size(), K.pool, s),
               "k_cache_apply launch");
    }

    // 4. a fine view is available iff every tile it showed is in the cache;
    // the view mask takes the available fine views and the coarse level's fill-in
    std::vector<uint8_t> avail((size_t)std::max(nf, 1), 1);
    for (const int32_t key : K.vis_keys)
        if (K.pt[(size_t)key] < 0) avail[(size_t)(key / K.tpv)] = 0;
    int64_t missing_views = 0;
    for (int32_t v = 0; v < nf; ++v) missing_views += !avail[(size_t)v];
    if (nf < n) {
        if (nf > 0) {
            rc = lf_two_level_mask(c, nf, avail.data(), m);
            if (rc) return rc;
        } else {
            std::fill(m, m + n, (uint8_t)1);
        }
    } else {
        for (int32_t v = 0; v < n; ++v) m[v] = avail[(size_t)v];
    }
    LF_HIP(hipMemcpyAsync(c->vmask, m, (size_t)n, hipMemcpyHostToDevice, s), "copy view mask");
    LF_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
    if (fine_available)
        for (int32_t v = 0; v < nf; ++v) fine_available[v] = avail[(size_t)v];
    if (visible_out) {
        std::memset(visible_out, 0, (size_t)n * K.tpv);
        for (const int32_t key : K.vis_keys) visible_out[key] = 1;
    }
    if (stats) {
        stats[0] = visible;
        stats[1] = hits;
        stats[2] = (int64_t)slots.size();
        stats[3] = evicted;
        stats[4] = missing_views;
    }
    return LF_OK;
}

int lf_cache_resident(const lf_ctx *c, uint8_t *resident_out) {
    if (!c) return fail(LF_EINVAL, "NULL context");
    if (c->img_fmt != LF_IMG_PAGED_RGBA8) return fail(LF_ESTATE, "the context's images are not paged");
    if (!resident_out) return fail(LF_EINVAL, "resident_out must not be NULL");
    for (size_t k = 0; k < c->cache.pt.size(); ++k) resident_out[k] = c->cache.pt[k] >= 0;
    return LF_OK;
}

int lf_cache_page_misses(lf_ctx *c, uint64_t *misses) {
    if (!c) return fail(LF_EINVAL, "NULL context");
    if (!misses) return fail(LF_EINVAL, "misses must not be NULL");
    *misses = 0;
    if (!c->cache.miss_dev) return LF_OK;
    unsigned int m = 0;
    LF_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
    LF_HIP(hipMemcpy(&m, c->cache.miss_dev, sizeof m, hipMemcpyDeviceToHost), "copy page misses");
    LF_HIP(hipMemset(c->cache.miss_dev, 0, sizeof(unsigned int)), "hipMemset");
    *misses = m;
    return LF_OK;
}

int lf_prefilter(lf_ctx *c, const int32_t *views, int32_t n_views, double radius, const double *aperture_ext,
                 const double *disk_pts, const double *pix_offs, int32_t n_samples, int32_t basis, float *out_rgb,
                 float *out_wsum, void *hip_stream) {
    if (!c) return fail(LF_EINVAL, "NULL context");
    if (!views || !disk_pts || !pix_offs) return fail(LF_EINVAL, "views, disk_pts and pix_offs must not be NULL");
    if (!out_rgb || !out_wsum) return fail(LF_EINVAL, "out_rgb and out_wsum must not be NULL");
    if (n_views <= 0) return fail(LF_EINVAL, "n_views must be positive (got %d)", n_views);
    if (n_samples <= 0 || n_samples > (1 << 20)) return fail(LF_EINVAL, "n_samples must be in [1, 2^20] (got %d)", n_samples);
    if (basis != LF_BASIS_BOX && basis != LF_BASIS_LANCZOS2) return fail(LF_EINVAL, "unknown basis %d", basis);
    if (!aperture_ext && (!(radius > 0.0) || !std::isfinite(radius)))
        return fail(LF_EINVAL, "radius must be finite and > 0");
    if (aperture_ext)
        for (int64_t k = 0; k < 4 * (int64_t)n_views; ++k)
            if (!(aperture_ext[k] > 0.0) || !std::isfinite(aperture_ext[k]))
                return fail(LF_EINVAL, "aperture_ext[%d][%d] is not finite and positive", (int)(k / 4), (int)(k % 4));
    if (c->img_w != c->img_h) return fail(LF_EINVAL, "the prefilter needs square source images");
    for (int32_t k = 0; k < n_views; ++k)
        if (views[k] < 0 || views[k] >= c->n) return fail(LF_EINVAL, "views[%d] = %d out of range", k, views[k]);
    for (int32_t j = 0; j < n_samples; ++j) {
        const double du = disk_pts[2 * j], dv = disk_pts[2 * j + 1], ds = pix_offs[2 * j], dt = pix_offs[2 * j + 1];
        if (!(du * du + dv * dv <= 1.0)) return fail(LF_EINVAL, "disk_pts[%d] is not in the unit disk", j);
        if (!(std::fabs(ds) <= 64.0 && std::fabs(dt) <= 64.0))
            return fail(LF_EINVAL, "pix_offs[%d] must be finite and within 64 pixels", j);
    }
    hipStream_t s = (hipStream_t)hip_stream;
    const int64_t npx = (int64_t)c->img_w * c->img_h;
    LF_HIP(hipMemsetAsync(out_rgb, 0, sizeof(float) * 3 * npx * n_views, s), "hipMemsetAsync(out_rgb)");
    LF_HIP(hipMemsetAsync(out_wsum, 0, sizeof(float) * npx * n_views, s), "hipMemsetAsync(out_wsum)");
    const double hfov = 2.0 * std::atan(c->tan_s) * 180.0 / M_PI;
    std::vector<lf_eye> eyes(kMaxEyesPerLaunch);
    std::vector<int32_t> res(2 * kMaxEyesPerLaunch);
    double pu[kMaxEyesPerLaunch], pv[kMaxEyesPerLaunch], pw[kMaxEyesPerLaunch];
    for (int32_t j = 0; j < n_samples; ++j) {
        const double du = disk_pts[2 * j], dv = disk_pts[2 * j + 1], ds = pix_offs[2 * j], dt = pix_offs[2 * j + 1];
        const double rho = 1.0 - std::sqrt(du * du + dv * dv);
        const double wgt = rho * basis_weight(basis, ds) * basis_weight(basis, dt);
        if (!(rho > 0.0) || wgt == 0.0) continue;
        for (int32_t k0 = 0; k0 < n_views; k0 += kMaxEyesPerLaunch) {
            const int32_t nk = std::min(kMaxEyesPerLaunch, n_views - k0);
            // one eye per target view: at the sample's point of the view's disk
            // (the circle of `radius`, or the oval whose quadrant holds (du, dv)),
            // with the view's frame
            for (int32_t k = 0; k < nk; ++k) {
                const double *vc = &c->h_vt[12 * (size_t)views[k0 + k]];
                const double *R = vc + 3;
                const double *ext = aperture_ext ? aperture_ext + 4 * (size_t)(k0 + k) : nullptr;
                pu[k] = (ext ? (du >= 0.0 ? ext[0] : ext[1]) : radius) * du;
                pv[k] = (ext ? (dv >= 0.0 ? ext[2] : ext[3]) : radius) * dv;
                // uniform unit-disk points land in an oval quadrant with density
                // 1 / (e_u e_v): the area factor restores Eq. (4)'s measure
                pw[k] = ext ? (du >= 0.0 ? ext[0] : ext[1]) * (dv >= 0.0 ? ext[2] : ext[3]) : 1.0;
                for (int a = 0; a < 3; ++a) eyes[k].pos[a] = vc[a] + pu[k] * R[3 * a] + pv[k] * R[3 * a + 1];
                std::memcpy(eyes[k].rot, R, sizeof(double) * 9);
                res[2 * k] = c->img_w;
                res[2 * k + 1] = c->img_h;
            }
            EyeChunk ch;
            fill_chunk(c, ch, eyes.data(), nk, hfov, res.data(), (int64_t)k0 * npx, c->tune.tile_w, c->tune.tile_h);
            for (int32_t k = 0; k < nk; ++k) {
                EyeParam &E = ch.e[k];
                E.src_view = views[k0 + k];
                E.off_x = (float)ds;
                E.off_y = (float)dt;
                E.par_u = (float)pu[k];
                E.par_v = (float)pv[k];
                E.pf_w = (float)pw[k];
            }
            RenderArgs a = base_args(c, c->R);
            int rc = prep_and_cull(c, ch, a, c->R, s);
            if (rc) return rc;
            a.out_rgb = out_rgb;
            a.out_wsum = out_wsum;
            a.scale = (float)wgt;
            LF_HIP(launch_render(ch, a, c->img_fmt, c->geo_fmt, MODE_PREFILTER, s), "k_render launch");
        }
    }
    LF_HIP(launch_prefilter_finish(out_rgb, out_wsum, npx * n_views, s), "k_prefilter_finish launch");
    return LF_OK;
}

int lf_debug_candidates(lf_ctx *c, const lf_eye *eye, double hfov_deg, int32_t W, int32_t H, int32_t cap,
                        int32_t *out_cand, int32_t *out_contrib, int32_t *out_ncand, void *hip_stream) {
    if (!c) return fail(LF_EINVAL, "NULL context");
    if (!out_cand || !out_contrib) return fail(LF_EINVAL, "out_cand and out_contrib must not be NULL");
    if (cap < 1 || cap > 1024) return fail(LF_EINVAL, "cap must be in [1,1024] (got %d)", cap);
    const int32_t res[2] = {W, H};
    int rc = check_eyes(c, eye, 1, hfov_deg, res);
    if (rc) return rc;
    EyeChunk ch;
    fill_chunk(c, ch, eye, 1, hfov_deg, res, 0, c->tune.tile_w, c->tune.tile_h);
    RenderArgs a = base_args(c, c->R);
    rc = prep_and_cull(c, ch, a, c->R, (hipStream_t)hip_stream);
    if (rc) return rc;
    a.dbg_cand = out_cand;
    a.dbg_contrib = out_contrib;
    a.dbg_ncand = out_ncand;
    a.dbg_cap = cap;
    LF_HIP(launch_render(ch, a, c->img_fmt, c->geo_fmt, MODE_DEBUG, (hipStream_t)hip_stream), "k_render launch");
    return LF_OK;
}

static void batch_release_graph(lf_ctx *c) {
    if (c->batch.exec) (void)hipGraphExecDestroy(c->batch.exec);
    if (c->batch.graph) (void)hipGraphDestroy(c->batch.graph);
    c->batch.exec = nullptr;
    c->batch.graph = nullptr;
    c->batch.key.clear();
}

int lf_render_batch(lf_ctx *c, const lf_eye *eyes, int32_t n_eyes, double hfov_deg, const int32_t *res,
                    float *out_rgb, float *out_wsum, uint8_t *out_count, const lf_tune *tune, void *hip_stream) {
    if (!c) return fail(LF_EINVAL, "NULL context");
    if (!out_rgb) return fail(LF_EINVAL, "out_rgb must not be NULL");
    int rc = check_eyes(c, eyes, n_eyes, hfov_deg, res);
    if (rc) return rc;
    lf_tune t;
    if (!tune_ok(tune ? *tune : c->batch.tune, t))
        return fail(LF_EINVAL, "invalid tune %dx%d, cap %d", tune ? tune->tile_w : 0, tune ? tune->tile_h : 0,
                    tune ? tune->cap : 0);
    hipStream_t s = (hipStream_t)hip_stream;
    lf_ctx::Batch &B = c->batch;

    // eye table (host side), with tile and super-tile offsets for this tile shape
    std::vector<EyeParam> ep(n_eyes);
    int32_t tiles = 0, supers = 0;
    {
        EyeChunk ch;
        int64_t pix_off = 0;
        for (int32_t k0 = 0; k0 < n_eyes; k0 += kMaxEyesPerLaunch) {
            const int32_t nk = std::min(kMaxEyesPerLaunch, n_eyes - k0);
            fill_chunk(c, ch, eyes + k0, nk, hfov_deg, res + 2 * k0, pix_off, t.tile_w, t.tile_h);
            for (int32_t k = 0; k < nk; ++k) {
                ep[k0 + k] = ch.e[k];
                ep[k0 + k].tile_off += tiles;
                ep[k0 + k].super_off += supers;
                pix_off += (int64_t)ch.e[k].W * ch.e[k].H;
            }
            tiles += ch.total_tiles;
            supers += ch.total_supers;
        }
    }
    // XCD queues: queue x holds band (x + k / 2) mod kXcds (a range of tile rows)
    // of every eye k in turn
    int32_t q_len[kXcds];
    for (int x = 0; x < kXcds; ++x) {
        int32_t off = 0;
        for (int32_t k = 0; k < n_eyes; ++k) {
            EyeParam &E = ep[k];
            const int band = (x + k / 2) % kXcds;
            E.band_off[x] = off;
            off += ((band + 1) * E.tiles_y / kXcds - band * E.tiles_y / kXcds) * E.tiles_x;
        }
        q_len[x] = off;
    }
    // device buffers: eye table, eye-view records, tile lists, counts, queue, stamps
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t ev_b = al(sizeof(EyeView) * (size_t)n_eyes * c->n);
    const size_t el_b = al(sizeof(uint16_t) * (size_t)n_eyes * c->n), ec_b = al(sizeof(int32_t) * (size_t)n_eyes);
    const size_t tl_b = al(sizeof(uint32_t) * (size_t)kListCap * tiles);
    const size_t tc_b = al(sizeof(int32_t) * (size_t)tiles);
    const size_t q_b = al(sizeof(unsigned int) * kQueueStride * kXcds), ft_b = al(sizeof(unsigned long long) * 2 * (size_t)n_eyes);
    const size_t need = ev_b + tl_b + tc_b + q_b + ft_b + el_b + ec_b;
    if (need > B.buf_bytes || n_eyes > B.eyes_cap) {
        if (B.copied) LF_HIP(hipEventSynchronize(B.copied), "hipEventSynchronize");
        LF_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
        batch_release_graph(c);
        if (need > B.buf_bytes) {
            if (B.buf) LF_HIP(hipFree(B.buf), "hipFree");
            B.buf = nullptr;
            B.buf_bytes = 0;
            LF_HIP(hipMalloc(&B.buf, need), "hipMalloc(batch buffers)");
            B.buf_bytes = need;
        }
        if (n_eyes > B.eyes_cap) {
            if (B.eyes_dev) LF_HIP(hipFree(B.eyes_dev), "hipFree");
            if (B.eyes_host) LF_HIP(hipHostFree(B.eyes_host), "hipHostFree");
            B.eyes_dev = nullptr;
            B.eyes_host = nullptr;
            B.eyes_cap = 0;
            LF_HIP(hipMalloc(&B.eyes_dev, sizeof(EyeParam) * n_eyes), "hipMalloc(eye table)");
            LF_HIP(hipHostMalloc((void **)&B.eyes_host, sizeof(EyeParam) * n_eyes, hipHostMallocDefault),
                   "hipHostMalloc(eye table)");
            B.eyes_cap = n_eyes;
        }
    }
    char *p = (char *)B.buf;
    RenderArgs a = base_args(c, c->R);
    a.ev = (const EyeView *)p;
    a.tile_list = (const uint32_t *)(p + ev_b);
    a.tile_count = (const int32_t *)(p + ev_b + tl_b);
    a.out_rgb = out_rgb;
    a.out_wsum = out_wsum;
    a.out_count = out_count;
    a.list_cap = t.cap;
    BatchArgs b;
    b.eyes = B.eyes_dev;
    b.n_eyes = n_eyes;
    b.total_tiles = tiles;
    b.total_supers = supers;
    b.tile_w = t.tile_w;
    b.tile_h = t.tile_h;
    b.queue = (unsigned int *)(p + ev_b + tl_b + tc_b);
    for (int x = 0; x < kXcds; ++x) b.q_len[x] = q_len[x];
    b.frame_t = (unsigned long long *)(p + ev_b + tl_b + tc_b + q_b);
    uint16_t *elist = (uint16_t *)(p + ev_b + tl_b + tc_b + q_b + ft_b);
    int32_t *ecount = (int32_t *)(p + ev_b + tl_b + tc_b + q_b + ft_b + el_b);
    B.frame_t = b.frame_t;
    B.n_eyes = n_eyes;

    // the graph depends on the batch shape and buffers, not on the eye poses
    std::string key;
    {
        char buf[256];
        snprintf(buf, sizeof buf, "%d|%.17g|%p|%p|%p|%p|%d|%d|%d|%d|", n_eyes, hfov_deg, (void *)out_rgb,
                 (void *)out_wsum, (void *)out_count, B.buf, t.tile_w, t.tile_h, t.cap, c->profiling ? 1 : 0);
        key = buf;
        for (int32_t k = 0; k < n_eyes; ++k) key += std::to_string(res[2 * k]) + "x" + std::to_string(res[2 * k + 1]) + ",";
    }
    if (key != B.key) {
        batch_release_graph(c);
        if (!B.cap_stream) LF_HIP(hipStreamCreateWithFlags(&B.cap_stream, hipStreamNonBlocking), "hipStreamCreate");
        int per_cu = 0, n_cu = 0;
        LF_HIP(persistent_occupancy(c->img_fmt, c->geo_fmt, c->ext_inv != nullptr, t.tile_w * t.tile_h, &per_cu),
               "occupancy");
        LF_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, c->device), "CU count");
        const int grid = std::max(1, std::min(per_cu * n_cu, tiles));
        const DiskBound db{c->vrad, c->R, 1.0, c->vmask};
        if (c->profiling && !B.ph_a) {
            LF_HIP(hipEventCreate(&B.ph_a), "hipEventCreate");
            LF_HIP(hipEventCreate(&B.ph_b), "hipEventCreate");
        }
        LF_HIP(hipStreamBeginCapture(B.cap_stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
        hipError_t e = launch_batch(b, a, c->vt, c->wr, c->n, db, view_bases(c), cull_geo(c), elist, ecount, c->img_fmt,
                                    c->geo_fmt, grid, B.cap_stream, nullptr, nullptr);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(B.cap_stream, &g);
        if (e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return hip_fail(e, "batch launch capture");
        }
        if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
        B.graph = g;
        B.node_a = B.node_b = nullptr;
        if (c->profiling) {
            // the capture is a chain ending in the persistent render kernel:
            // put an event-record node right before it and one right after it
            size_t nn = 0;
            LF_HIP(hipGraphGetNodes(g, nullptr, &nn), "hipGraphGetNodes");
            std::vector<hipGraphNode_t> nodes(nn);
            LF_HIP(hipGraphGetNodes(g, nodes.data(), &nn), "hipGraphGetNodes");
            hipGraphNode_t leaf = nullptr;
            for (auto nd : nodes) {
                size_t nd_out = 0;
                LF_HIP(hipGraphNodeGetDependentNodes(nd, nullptr, &nd_out), "hipGraphNodeGetDependentNodes");
                if (nd_out == 0) leaf = nd;
            }
            if (!leaf) return fail(LF_EHIP, "batch graph has no final node");
            size_t nd_in = 0;
            LF_HIP(hipGraphNodeGetDependencies(leaf, nullptr, &nd_in), "hipGraphNodeGetDependencies");
            std::vector<hipGraphNode_t> deps(nd_in);
            if (nd_in) LF_HIP(hipGraphNodeGetDependencies(leaf, deps.data(), &nd_in), "hipGraphNodeGetDependencies");
            LF_HIP(hipGraphAddEventRecordNode(&B.node_a, g, deps.data(), nd_in, B.ph_a), "add event node");
            for (auto d : deps) LF_HIP(hipGraphRemoveDependencies(g, &d, &leaf, 1), "hipGraphRemoveDependencies");
            LF_HIP(hipGraphAddDependencies(g, &B.node_a, &leaf, 1), "hipGraphAddDependencies");
            LF_HIP(hipGraphAddEventRecordNode(&B.node_b, g, &leaf, 1, B.ph_b), "add event node");
        }
        LF_HIP(hipGraphInstantiate(&B.exec, g, nullptr, nullptr, 0), "hipGraphInstantiate");
        B.key = key;
    }
    // upload this batch's eye table through pinned staging, then replay the graph
    if (B.copied) LF_HIP(hipEventSynchronize(B.copied), "hipEventSynchronize");
    else LF_HIP(hipEventCreateWithFlags(&B.copied, hipEventDisableTiming), "hipEventCreate");
    std::memcpy(B.eyes_host, ep.data(), sizeof(EyeParam) * n_eyes);
    LF_HIP(hipMemcpyAsync(B.eyes_dev, B.eyes_host, sizeof(EyeParam) * n_eyes, hipMemcpyHostToDevice, s),
           "upload eye table");
    LF_HIP(hipEventRecord(B.copied, s), "hipEventRecord");
    if (c->profiling) {
        lf_ctx::Timed tm{2, nullptr, nullptr};
        LF_HIP(hipEventCreate(&tm.a), "hipEventCreate");
        LF_HIP(hipEventCreate(&tm.b), "hipEventCreate");
        c->timed.push_back(tm);
        LF_HIP(hipGraphExecEventRecordNodeSetEvent(B.exec, B.node_a, tm.a), "set event node");
        LF_HIP(hipGraphExecEventRecordNodeSetEvent(B.exec, B.node_b, tm.b), "set event node");
    }
    LF_HIP(hipGraphLaunch(B.exec, s), "hipGraphLaunch");
    return LF_OK;
}

int lf_autotune_batch(lf_ctx *c, const lf_eye *eyes, int32_t n_eyes, double hfov_deg, const int32_t *res,
                      float *out_rgb, int32_t reps, lf_tune *best, float *ms, void *hip_stream) {
    if (!c) return fail(LF_EINVAL, "NULL context");
    if (reps < 1 || reps > 100) return fail(LF_EINVAL, "reps must be in [1,100]");
    static const int shapes[3][2] = {{8, 8}, {16, 16}, {32, 8}};
    static const int caps[4] = {8, 16, 32, kListCap};
    hipStream_t s = (hipStream_t)hip_stream;
    hipEvent_t ea, eb;
    LF_HIP(hipEventCreate(&ea), "hipEventCreate");
    LF_HIP(hipEventCreate(&eb), "hipEventCreate");
    const bool prof = c->profiling;
    c->profiling = false;
    float best_ms = INFINITY;
    lf_tune bt = c->batch.tune;
    int rc = LF_OK;
    for (int i = 0; i < 12 && rc == LF_OK; ++i) {
        lf_tune t{shapes[i / 4][0], shapes[i / 4][1], caps[i % 4]};
        rc = lf_render_batch(c, eyes, n_eyes, hfov_deg, res, out_rgb, nullptr, nullptr, &t, hip_stream);  // capture + warm
        std::vector<float> times;
        for (int r = 0; r < reps && rc == LF_OK; ++r) {
            hipError_t e = hipEventRecord(ea, s);
            if (e == hipSuccess) rc = lf_render_batch(c, eyes, n_eyes, hfov_deg, res, out_rgb, nullptr, nullptr, &t,
                                                      hip_stream);
            if (e == hipSuccess && rc == LF_OK) e = hipEventRecord(eb, s);
            if (e == hipSuccess && rc == LF_OK) e = hipEventSynchronize(eb);
            float m = 0.0f;
            if (e == hipSuccess && rc == LF_OK) e = hipEventElapsedTime(&m, ea, eb);
            if (e != hipSuccess) rc = hip_fail(e, "autotune timing");
            times.push_back(m);
        }
        if (rc != LF_OK) break;
        std::sort(times.begin(), times.end());
        const float med = times[times.size() / 2];
        if (ms) ms[i] = med;
        if (med < best_ms) {
            best_ms = med;
            bt = t;
        }
    }
    c->profiling = prof;
    (void)hipEventDestroy(ea);
    (void)hipEventDestroy(eb);
    if (rc != LF_OK) return rc;
    c->batch.tune = bt;
    c->batch.tuned = true;
    if (best) *best = bt;
    return LF_OK;
}

int lf_batch_frame_times(lf_ctx *c, double *out_us, int32_t n_eyes) {
    if (!c) return fail(LF_EINVAL, "NULL context");
    if (!out_us) return fail(LF_EINVAL, "out_us must not be NULL");
    if (!c->batch.frame_t || n_eyes != c->batch.n_eyes)
        return fail(LF_ESTATE, "no batch of %d eyes has been rendered", n_eyes);
    std::vector<unsigned long long> h(2 * (size_t)n_eyes);
    LF_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
    LF_HIP(hipMemcpy(h.data(), c->batch.frame_t, h.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost),
           "read frame stamps");
    int khz = 0;
    LF_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, c->device), "wall clock rate");
    if (khz <= 0) return fail(LF_EHIP, "device reports no wall clock rate");
    unsigned long long t0 = ~0ull;
    for (int32_t k = 0; k < n_eyes; ++k) t0 = std::min(t0, h[2 * k]);
    for (int32_t k = 0; k < n_eyes; ++k) {
        out_us[2 * k] = (double)(h[2 * k] - t0) * 1e3 / khz;
        out_us[2 * k + 1] = (double)(h[2 * k + 1] - t0) * 1e3 / khz;
    }
    return LF_OK;
}

int lf_render_stats(lf_ctx *c, const lf_eye *eyes, int32_t n_eyes, double hfov_deg, const int32_t *res,
                    uint64_t counters[5], void *hip_stream) {
    if (!c) return fail(LF_EINVAL, "NULL context");
    if (!counters) return fail(LF_EINVAL, "counters must not be NULL");
    int rc = check_eyes(c, eyes, n_eyes, hfov_deg, res);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)hip_stream;
    unsigned long long *d = nullptr;
    LF_HIP(hipMalloc(&d, 5 * sizeof(unsigned long long)), "hipMalloc(stats)");
    hipError_t e = hipMemsetAsync(d, 0, 5 * sizeof(unsigned long long), s);
    if (e != hipSuccess) {
        (void)hipFree(d);
        return hip_fail(e, "hipMemsetAsync(stats)");
    }
    const bool prof = c->profiling;
    c->profiling = false;
    rc = render_impl(c, eyes, n_eyes, hfov_deg, res, nullptr, nullptr, nullptr, MODE_STATS, c->R, 0.5f, 0.5f, 1.0f,
                     0, s, d);
    c->profiling = prof;
    if (rc == LF_OK) {
        unsigned long long h[5];
        e = hipMemcpyAsync(h, d, sizeof h, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) rc = hip_fail(e, "read stats");
        else for (int k = 0; k < 5; ++k) counters[k] = h[k];
    }
    (void)hipFree(d);
    return rc;
}

int lf_profile(lf_ctx *c, int32_t enable) {
    if (!c) return fail(LF_EINVAL, "NULL context");
    for (auto &t : c->timed) {
        (void)hipEventSynchronize(t.b);
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    c->timed.clear();
    for (int k = 0; k < 3; ++k) c->prof_ms[k] = c->prof_n[k] = 0.0;
    c->profiling = enable != 0;
    return LF_OK;
}

int lf_profile_read(lf_ctx *c, double out[6]) {
    if (!c) return fail(LF_EINVAL, "NULL context");
    if (!out) return fail(LF_EINVAL, "out must not be NULL");
    for (auto &t : c->timed) {
        hipError_t e = hipEventSynchronize(t.b);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, t.a, t.b);
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
        if (e != hipSuccess) {
            c->timed.clear();
            return hip_fail(e, "profile events");
        }
        c->prof_ms[t.kind] += ms;
        c->prof_n[t.kind] += 1.0;
    }
    c->timed.clear();
    for (int k = 0; k < 3; ++k) {
        out[k] = c->prof_ms[k];
        out[3 + k] = c->prof_n[k];
    }
    return LF_OK;
}

void lf_free(lf_ctx *c) {
    if (!c) return;
    (void)hipDeviceSynchronize();
    if (c->img) (void)hipFree(c->img);
    if (c->img2) (void)hipFree(c->img2);
    if (c->geo) (void)hipFree(c->geo);
    if (c->vt) (void)hipFree(c->vt);
    if (c->wr) (void)hipFree(c->wr);
    if (c->blk) (void)hipFree(c->blk);
    if (c->win) (void)hipFree(c->win);
    if (c->ext_inv) (void)hipFree(c->ext_inv);
    if (c->vrad) (void)hipFree(c->vrad);
    if (c->vmask) (void)hipFree(c->vmask);
    if (c->scratch) (void)hipFree(c->scratch);
    if (c->cache.host) (void)hipHostFree(c->cache.host);
    if (c->cache.pool) (void)hipFree(c->cache.pool);
    if (c->cache.vis_dev) (void)hipFree(c->cache.vis_dev);
    if (c->cache.keys_dev) (void)hipFree(c->cache.keys_dev);
    if (c->cache.count_dev) (void)hipFree(c->cache.count_dev);
    if (c->cache.count_host) (void)hipHostFree(c->cache.count_host);
    if (c->cache.mask_host) (void)hipHostFree(c->cache.mask_host);
    if (c->cache.stage_dev) (void)hipFree(c->cache.stage_dev);
    if (c->cache.stage_host) (void)hipHostFree(c->cache.stage_host);
    if (c->cache.miss_dev) (void)hipFree(c->cache.miss_dev);
    for (auto &t : c->timed) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    batch_release_graph(c);
    if (c->batch.copied) (void)hipEventDestroy(c->batch.copied);
    if (c->batch.ph_a) (void)hipEventDestroy(c->batch.ph_a);
    if (c->batch.ph_b) (void)hipEventDestroy(c->batch.ph_b);
    if (c->batch.cap_stream) (void)hipStreamDestroy(c->batch.cap_stream);
    if (c->batch.buf) (void)hipFree(c->batch.buf);
    if (c->batch.eyes_dev) (void)hipFree(c->batch.eyes_dev);
    if (c->batch.eyes_host) (void)hipHostFree(c->batch.eyes_host);
    delete c;
}

}  // extern "C"
