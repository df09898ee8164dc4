"""Thin ctypes binding of liblf.so (include/lf.h). Argument marshalling only:
every step of the render runs in the library's HIP kernels. Device buffers are
passed as torch tensors (their data_ptr) or raw integer addresses."""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# LF_LIB may name another build of the same sources (the sanitizer test loads
# a build whose host code carries AddressSanitizer and UBSan checks)
LIB_PATH = os.environ.get("LF_LIB") or os.path.join(_HERE, "liblf.so")

LF_OK, LF_EINVAL, LF_ENOMEM, LF_EHIP, LF_ESTATE = 0, -1, -2, -3, -4
LF_IMG_RGBA8, LF_IMG_RGBA16F, LF_IMG_RGBA32F, LF_IMG_YUV420, LF_IMG_YUV420_RGTC, LF_IMG_PAGED_RGBA8 = 0, 1, 2, 3, 4, 5
LF_GEO_F32, LF_GEO_F16, LF_GEO_U16 = 0, 1, 2
LF_SRC_DEVICE = 1

IMG_FORMATS = {"rgba8": LF_IMG_RGBA8, "rgba16f": LF_IMG_RGBA16F, "rgba32f": LF_IMG_RGBA32F, "yuv420": LF_IMG_YUV420,
               "yuv420_rgtc": LF_IMG_YUV420_RGTC, "paged_rgba8": LF_IMG_PAGED_RGBA8}
GEO_FORMATS = {"f32": LF_GEO_F32, "f16": LF_GEO_F16, "u16": LF_GEO_U16}


class lf_views_desc(ctypes.Structure):
    _fields_ = [
        ("n_views", ctypes.c_int32), ("img_w", ctypes.c_int32), ("img_h", ctypes.c_int32),
        ("mesh_m", ctypes.c_int32), ("src_fov_deg", ctypes.c_double),
        ("centres", ctypes.c_void_p), ("rot", ctypes.c_void_p), ("rgba8", ctypes.c_void_p),
        ("zdepth", ctypes.c_void_p), ("disk_radius", ctypes.c_double), ("disk_ext", ctypes.c_void_p),
        ("img_fmt", ctypes.c_int32), ("geo_fmt", ctypes.c_int32), ("flags", ctypes.c_int32),
    ]


class lf_eye(ctypes.Structure):
    _fields_ = [("pos", ctypes.c_double * 3), ("rot", ctypes.c_double * 9)]


class lf_tune(ctypes.Structure):
    _fields_ = [("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32), ("cap", ctypes.c_int32)]


class LFError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"liblf error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load liblf.so; fail loudly when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is missing: build it with __graft_entry__.build()")
        # torch owns device memory and streams: load its HIP runtime first so
        # that liblf.so binds to the same runtime (same soname) instead of
        # bringing a second one into the process
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
        L.lf_load_views.argtypes = [ctypes.POINTER(lf_views_desc), ctypes.POINTER(vp)]
        L.lf_stereo_eyes.argtypes = [vp, vp, f64, ctypes.POINTER(lf_eye)]
        L.lf_disk_extents.argtypes = [i32, vp, vp, f64, vp]
        L.lf_set_tune.argtypes = [vp, ctypes.POINTER(lf_tune)]
        L.lf_render.argtypes = [vp, ctypes.POINTER(lf_eye), i32, f64, vp, vp, vp, vp, vp]
        L.lf_render_noalloc.argtypes = [vp, ctypes.POINTER(lf_eye), i32, f64, vp, vp, vp, vp, vp]
        L.lf_render_reference.argtypes = [vp, ctypes.POINTER(lf_eye), i32, f64, vp, i32, f64, vp, vp]
        L.lf_prefilter.argtypes = [vp, vp, i32, f64, vp, vp, vp, i32, i32, vp, vp, vp]
        L.lf_set_view_mask.argtypes = [vp, vp]
        L.lf_two_level_mask.argtypes = [vp, i32, vp, vp]
        L.lf_cache_config.argtypes = [vp, ctypes.c_int64, i32]
        L.lf_cache_update.argtypes = [vp, ctypes.POINTER(lf_eye), i32, f64, vp, i32, vp, vp, vp, vp]
        L.lf_cache_resident.argtypes = [vp, vp]
        L.lf_cache_page_misses.argtypes = [vp, vp]
        L.lf_stream_copy.argtypes = [vp, vp, ctypes.c_int64, vp]
        L.lf_fma_rate.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp]
        L.lf_debug_candidates.argtypes = [vp, ctypes.POINTER(lf_eye), f64, i32, i32, i32, vp, vp, vp, vp]
        L.lf_query.argtypes = [vp, vp, vp, vp, vp, vp]
        L.lf_render_stats.argtypes = [vp, ctypes.POINTER(lf_eye), i32, f64, vp, vp, vp]
        L.lf_profile.argtypes = [vp, i32]
        L.lf_profile_read.argtypes = [vp, vp]
        L.lf_render_batch.argtypes = [vp, ctypes.POINTER(lf_eye), i32, f64, vp, vp, vp, vp,
                                      ctypes.POINTER(lf_tune), vp]
        L.lf_autotune_batch.argtypes = [vp, ctypes.POINTER(lf_eye), i32, f64, vp, vp, i32, ctypes.POINTER(lf_tune),
                                        vp, vp]
        L.lf_batch_frame_times.argtypes = [vp, vp, i32]
        L.lf_corrector_create.argtypes = [vp, ctypes.POINTER(vp)]
        L.lf_corrector_set_params.argtypes = [vp, vp]
        L.lf_corrector_get_params.argtypes = [vp, vp, vp]
        L.lf_corrector_get_state.argtypes = [vp, vp, vp, vp, vp]
        L.lf_corrector_set_state.argtypes = [vp, vp, vp, vp, ctypes.c_int64]
        L.lf_corrector_apply.argtypes = [vp, vp, vp, vp, i32, i32, i32, ctypes.c_float, vp, vp, vp, vp]
        L.lf_corrector_train_step.argtypes = [vp, vp, vp, vp, vp, i32, i32, i32, ctypes.c_float, vp, vp, vp]
        L.lf_corrector_free.argtypes = [vp]
        L.lf_corrector_free.restype = None
        L.lf_last_error.restype = ctypes.c_char_p
        L.lf_free.argtypes = [vp]
        L.lf_free.restype = None
        for name in ("lf_load_views", "lf_stereo_eyes", "lf_disk_extents", "lf_set_tune", "lf_render",
                     "lf_render_noalloc",
                     "lf_render_reference",
                     "lf_debug_candidates", "lf_query", "lf_render_stats", "lf_profile", "lf_profile_read",
                     "lf_render_batch", "lf_autotune_batch", "lf_batch_frame_times", "lf_corrector_create",
                     "lf_corrector_set_params", "lf_corrector_get_params", "lf_corrector_apply",
                     "lf_corrector_train_step", "lf_corrector_get_state", "lf_corrector_set_state"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc != LF_OK:
        raise LFError(rc, lib().lf_last_error().decode())
    return rc


def _ptr(x):
    """Device (or host) address of a torch tensor / numpy array / int / None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    raise TypeError(f"cannot take the address of {type(x)}")


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def make_eyes(eyes) -> ctypes.Array:
    """Eyes from a sequence of (pos[3], rot[3,3]) pairs or an lf_eye array."""
    if isinstance(eyes, ctypes.Array):
        return eyes
    eyes = list(eyes)
    arr = (lf_eye * len(eyes))()
    for k, (p, r) in enumerate(eyes):
        arr[k].pos[:] = [float(v) for v in np.asarray(p, np.float64).reshape(3)]
        arr[k].rot[:] = [float(v) for v in np.asarray(r, np.float64).reshape(9)]
    return arr


class Context:
    """Owns an lf_ctx handle (lf_free on close / garbage collection)."""

    def __init__(self, handle, n_views, img_fmt, geo_fmt):
        self.handle = handle
        self.n_views = n_views
        self.img_fmt = img_fmt
        self.geo_fmt = geo_fmt

    def close(self):
        if self.handle:
            lib().lf_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lf_load_views(centres, rot, rgba8, zdepth, src_fov_deg, disk_radius, img_fmt="rgba8", geo_fmt="f32",
                  device_src=False, disk_ext=None) -> Context:
    """disk_ext: None for circular disks of disk_radius, else [n][4] oval extents (see lf_disk_extents)."""
    img_fmt = IMG_FORMATS.get(img_fmt, img_fmt)
    geo_fmt = GEO_FORMATS.get(geo_fmt, geo_fmt)
    centres = np.ascontiguousarray(centres, np.float64)
    rot = np.ascontiguousarray(np.asarray(rot, np.float64).reshape(-1, 9))
    if device_src:
        n, h, w, _ = tuple(rgba8.shape)
        m = int(zdepth.shape[1])
    else:
        rgba8 = np.ascontiguousarray(rgba8, np.uint8)
        zdepth = np.ascontiguousarray(zdepth, np.float32)
        n, h, w, _ = rgba8.shape
        m = zdepth.shape[1]
    ext = None if disk_ext is None else np.ascontiguousarray(disk_ext, np.float64).reshape(n, 4)
    d = lf_views_desc(n, w, h, m, float(src_fov_deg), centres.ctypes.data, rot.ctypes.data, _ptr(rgba8),
                      _ptr(zdepth), float(disk_radius), None if ext is None else ext.ctypes.data, int(img_fmt),
                      int(geo_fmt), LF_SRC_DEVICE if device_src else 0)
    h_ = ctypes.c_void_p()
    _check(lib().lf_load_views(ctypes.byref(d), ctypes.byref(h_)))
    return Context(h_.value, n, img_fmt, geo_fmt)


def lf_disk_extents(centres, rot, scale=1.0):
    """[n][4] extents (e+u, e-u, e+v, e-v) of the views' asymmetric oval disks."""
    c = np.ascontiguousarray(centres, np.float64).reshape(-1, 3)
    r = np.ascontiguousarray(np.asarray(rot, np.float64).reshape(-1, 9))
    out = np.zeros((len(c), 4), np.float64)
    _check(lib().lf_disk_extents(len(c), c.ctypes.data, r.ctypes.data, float(scale), out.ctypes.data))
    return out


def lf_stereo_eyes(head_pos, head_rot, ipd_m):
    hp = np.ascontiguousarray(head_pos, np.float64)
    hr = np.ascontiguousarray(np.asarray(head_rot, np.float64).reshape(9))
    out = (lf_eye * 2)()
    _check(lib().lf_stereo_eyes(hp.ctypes.data, hr.ctypes.data, float(ipd_m), out))
    return out


def lf_set_tune(ctx: Context, tile_w=None, tile_h=None, cap=0):
    if tile_w is None:
        return _check(lib().lf_set_tune(ctx.handle, None))
    t = lf_tune(int(tile_w), int(tile_h), int(cap))
    return _check(lib().lf_set_tune(ctx.handle, ctypes.byref(t)))


def _res(res, n):
    r = np.ascontiguousarray(np.asarray(res, np.int32).reshape(-1))
    if r.size == 2 and n > 1:
        r = np.tile(r, n)
    if r.size != 2 * n:
        raise ValueError("res must hold a (W, H) pair per eye")
    return r


def lf_render(ctx: Context, eyes, hfov_deg, res, out_rgb, out_wsum=None, out_count=None, stream=None):
    e = make_eyes(eyes)
    r = _res(res, len(e))
    _check(lib().lf_render(ctx.handle, e, len(e), float(hfov_deg), r.ctypes.data, _ptr(out_rgb), _ptr(out_wsum),
                           _ptr(out_count), _stream(stream)))


def lf_render_noalloc(ctx: Context, eyes, hfov_deg, res, out_rgb, out_wsum=None, out_count=None, stream=None):
    """lf_render with its scratch in the library's fixed device array (no
    device allocation; calls on one GPU must not overlap)."""
    e = make_eyes(eyes)
    r = _res(res, len(e))
    _check(lib().lf_render_noalloc(ctx.handle, e, len(e), float(hfov_deg), r.ctypes.data, _ptr(out_rgb),
                                   _ptr(out_wsum), _ptr(out_count), _stream(stream)))


def lf_render_reference(ctx: Context, eyes, hfov_deg, res, ss, disk_scale, out_rgb, stream=None):
    e = make_eyes(eyes)
    r = _res(res, len(e))
    _check(lib().lf_render_reference(ctx.handle, e, len(e), float(hfov_deg), r.ctypes.data, int(ss),
                                     float(disk_scale), _ptr(out_rgb), _stream(stream)))


def lf_set_view_mask(ctx: Context, enabled=None):
    """Views taking part in later renders (None: all)."""
    m = None if enabled is None else np.ascontiguousarray(enabled, np.uint8).reshape(-1)
    if m is not None and len(m) != ctx.n_views:
        raise ValueError("enabled must hold one entry per view")
    _check(lib().lf_set_view_mask(ctx.handle, None if m is None else m.ctypes.data))


def lf_two_level_mask(ctx: Context, n_fine, fine_available):
    """View mask of two-level progressive rendering (fine views first)."""
    a = np.ascontiguousarray(fine_available, np.uint8).reshape(-1)
    if len(a) != n_fine:
        raise ValueError("fine_available must hold n_fine entries")
    out = np.zeros(ctx.n_views, np.uint8)
    _check(lib().lf_two_level_mask(ctx.handle, int(n_fine), a.ctypes.data, out.ctypes.data))
    return out


def lf_cache_config(ctx: Context, pages, first_resident=None):
    """Tile cache of `pages` 64 x 64-texel pages for a paged context; views
    [first_resident, n_views) stay resident (None: none)."""
    fr = ctx.n_views if first_resident is None else int(first_resident)
    _check(lib().lf_cache_config(ctx.handle, int(pages), fr))


def lf_cache_update(ctx: Context, eyes, hfov_deg, res, budget, n_fine=None, stream=None, want_visible=True):
    """One frame of tile streaming for these eyes (visibility pass, FIFO
    uploads within the budget, view mask). Returns (fine_available [n_fine],
    visible [n_views, tiles] uint8 or None, stats dict)."""
    e = make_eyes(eyes)
    r = _res(res, len(e))
    nf = ctx.n_views if n_fine is None else int(n_fine)
    avail = np.zeros(max(nf, 1), np.uint8)
    vis = None
    if want_visible:
        q = lf_query(ctx)
        vis = np.zeros((ctx.n_views, (q[1] // 64) ** 2), np.uint8)
    st = np.zeros(5, np.int64)
    _check(lib().lf_cache_update(ctx.handle, e, len(e), float(hfov_deg), r.ctypes.data, int(budget), avail.ctypes.data,
                                 None if vis is None else vis.ctypes.data, st.ctypes.data, _stream(stream)))
    keys = ("visible", "cached", "copied", "evicted", "views_unavailable")
    return avail[:nf], vis, dict(zip(keys, (int(x) for x in st)))


def lf_cache_resident(ctx: Context):
    """uint8 [n_views, tiles]: 1 where the tile is in the cache."""
    q = lf_query(ctx)
    out = np.zeros((ctx.n_views, (q[1] // 64) ** 2), np.uint8)
    _check(lib().lf_cache_resident(ctx.handle, out.ctypes.data))
    return out


def lf_cache_page_misses(ctx: Context):
    """Samples left out for a missing tile since the last call (resets it)."""
    m = ctypes.c_uint64(0)
    _check(lib().lf_cache_page_misses(ctx.handle, ctypes.byref(m)))
    return int(m.value)


BASIS = {"box": 0, "lanczos2": 1}


def lf_prefilter(ctx: Context, views, radius, disk_pts, pix_offs, basis, out_rgb, out_wsum, stream=None,
                 aperture_ext=None):
    """Prefilter (Sec. 5, Eq. (5)) of the listed views; outputs are device
    buffers of n_views x img_h x img_w RGB floats and weight sums. The aperture
    is the circle of `radius`, or with aperture_ext (n_views, 4) each listed
    view's oval disk (e+u, e-u, e+v, e-v)."""
    v = np.ascontiguousarray(views, np.int32).reshape(-1)
    dp = np.ascontiguousarray(disk_pts, np.float64).reshape(-1, 2)
    po = np.ascontiguousarray(pix_offs, np.float64).reshape(-1, 2)
    if dp.shape != po.shape:
        raise ValueError("disk_pts and pix_offs must both be (J, 2)")
    ext = None
    if aperture_ext is not None:
        ext = np.ascontiguousarray(aperture_ext, np.float64).reshape(len(v), 4)
    _check(lib().lf_prefilter(ctx.handle, v.ctypes.data, len(v), float(radius),
                              None if ext is None else ext.ctypes.data, dp.ctypes.data, po.ctypes.data,
                              dp.shape[0], BASIS[basis] if isinstance(basis, str) else int(basis), _ptr(out_rgb),
                              _ptr(out_wsum), _stream(stream)))


def lf_debug_candidates(ctx: Context, eye, hfov_deg, W, H, cap, out_cand, out_contrib, out_ncand=None,
                        stream=None):
    e = make_eyes([eye]) if not isinstance(eye, ctypes.Array) else eye
    _check(lib().lf_debug_candidates(ctx.handle, e, float(hfov_deg), int(W), int(H), int(cap), _ptr(out_cand),
                                     _ptr(out_contrib), _ptr(out_ncand), _stream(stream)))


def lf_render_batch(ctx: Context, eyes, hfov_deg, res, out_rgb, out_wsum=None, out_count=None, tune=None,
                    stream=None):
    e = make_eyes(eyes)
    r = _res(res, len(e))
    t = ctypes.byref(lf_tune(*tune)) if tune is not None else None
    _check(lib().lf_render_batch(ctx.handle, e, len(e), float(hfov_deg), r.ctypes.data, _ptr(out_rgb),
                                 _ptr(out_wsum), _ptr(out_count), t, _stream(stream)))


TUNE_SHAPES = [(8, 8), (16, 16), (32, 8)]
TUNE_CAPS = [8, 16, 32, 64]
# the autotuner's points (tile_w, tile_h, cap), shape-major
TUNE_GRID = [(w, h, c) for (w, h) in TUNE_SHAPES for c in TUNE_CAPS]


def lf_autotune_batch(ctx: Context, eyes, hfov_deg, res, out_rgb, reps=5, stream=None):
    """Returns ((tile_w, tile_h, cap) chosen, {(tile_w, tile_h, cap): median ms})."""
    e = make_eyes(eyes)
    r = _res(res, len(e))
    best = lf_tune()
    ms = np.zeros(len(TUNE_GRID), np.float32)
    _check(lib().lf_autotune_batch(ctx.handle, e, len(e), float(hfov_deg), r.ctypes.data, _ptr(out_rgb), int(reps),
                                   ctypes.byref(best), ms.ctypes.data, _stream(stream)))
    return (best.tile_w, best.tile_h, best.cap), dict(zip(TUNE_GRID, ms.tolist()))


def lf_batch_frame_times(ctx: Context, n_eyes):
    out = np.zeros((n_eyes, 2), np.float64)
    _check(lib().lf_batch_frame_times(ctx.handle, out.ctypes.data, int(n_eyes)))
    return out


CORRECTOR_PARAMS = 20835


class Corrector:
    """Owns an lf_corrector handle."""

    def __init__(self, handle):
        self.handle = handle

    def close(self):
        if self.handle:
            lib().lf_corrector_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lf_corrector_create(params=None) -> Corrector:
    h = ctypes.c_void_p()
    p = None
    if params is not None:
        params = np.ascontiguousarray(params, np.float32)
        assert params.size == CORRECTOR_PARAMS
        p = params.ctypes.data
    _check(lib().lf_corrector_create(p, ctypes.byref(h)))
    return Corrector(h.value)


def lf_corrector_set_params(c: Corrector, params):
    params = np.ascontiguousarray(params, np.float32)
    assert params.size == CORRECTOR_PARAMS
    _check(lib().lf_corrector_set_params(c.handle, params.ctypes.data))


def lf_corrector_get_params(c: Corrector):
    out = np.zeros(CORRECTOR_PARAMS, np.float32)
    step = ctypes.c_int64()
    _check(lib().lf_corrector_get_params(c.handle, out.ctypes.data, ctypes.byref(step)))
    return out, step.value


def lf_corrector_get_state(c: Corrector) -> dict:
    """FP32 master parameters, Adam moments and step count (host copies)."""
    out = {k: np.zeros(CORRECTOR_PARAMS, np.float32) for k in ("params", "adam_m", "adam_v")}
    step = ctypes.c_int64()
    _check(lib().lf_corrector_get_state(c.handle, out["params"].ctypes.data, out["adam_m"].ctypes.data,
                                        out["adam_v"].ctypes.data, ctypes.byref(step)))
    out["step"] = int(step.value)
    return out


def lf_corrector_set_state(c: Corrector, params, adam_m, adam_v, step):
    arrs = [np.ascontiguousarray(a, np.float32).reshape(CORRECTOR_PARAMS) for a in (params, adam_m, adam_v)]
    _check(lib().lf_corrector_set_state(c.handle, arrs[0].ctypes.data, arrs[1].ctypes.data, arrs[2].ctypes.data,
                                        int(step)))


def lf_corrector_apply(c: Corrector, rgb, wsum, count, n_images, W, H, thresh, out_rgb, out_fallback=None,
                       out_resid=None, stream=None):
    _check(lib().lf_corrector_apply(c.handle, _ptr(rgb), _ptr(wsum), _ptr(count), int(n_images), int(W), int(H),
                                    float(thresh), _ptr(out_rgb), _ptr(out_fallback), _ptr(out_resid),
                                    _stream(stream)))


def lf_corrector_train_step(c: Corrector, rgb, wsum, count, ref, n_images, W, H, lr, want_loss=True,
                            want_grad=False, stream=None):
    loss = ctypes.c_float()
    grad = np.zeros(CORRECTOR_PARAMS, np.float32) if want_grad else None
    _check(lib().lf_corrector_train_step(c.handle, _ptr(rgb), _ptr(wsum), _ptr(count), _ptr(ref), int(n_images),
                                         int(W), int(H), float(lr), ctypes.byref(loss) if want_loss else None,
                                         grad.ctypes.data if want_grad else None, _stream(stream)))
    return (loss.value if want_loss else None), grad


STAT_NAMES = ("pixels", "disk_tests", "candidates", "cells", "samples")


def lf_render_stats(ctx: Context, eyes, hfov_deg, res, stream=None) -> dict:
    e = make_eyes(eyes)
    r = _res(res, len(e))
    out = np.zeros(5, np.uint64)
    _check(lib().lf_render_stats(ctx.handle, e, len(e), float(hfov_deg), r.ctypes.data, out.ctypes.data,
                                 _stream(stream)))
    return {k: int(v) for k, v in zip(STAT_NAMES, out)}


def lf_profile(ctx: Context, enable: bool):
    _check(lib().lf_profile(ctx.handle, 1 if enable else 0))


def lf_profile_read(ctx: Context) -> dict:
    out = np.zeros(6, np.float64)
    _check(lib().lf_profile_read(ctx.handle, out.ctypes.data))
    return {"prep_ms": out[0], "cull_ms": out[1], "render_ms": out[2],
            "prep_n": int(out[3]), "cull_n": int(out[4]), "render_n": int(out[5])}


def lf_query(ctx: Context):
    vals = [ctypes.c_int32() for _ in range(5)]
    _check(lib().lf_query(ctx.handle, *[ctypes.byref(v) for v in vals]))
    return tuple(v.value for v in vals)


def lf_stream_copy(src, dst, nbytes, stream=None):
    """Plain device copy of nbytes (achievable-bandwidth yardstick)."""
    _check(lib().lf_stream_copy(_ptr(src), _ptr(dst), int(nbytes), _stream(stream)))


def lf_fma_rate(out, blocks, iters, active, stream=None):
    """Independent FP32 FMA chains on `active` lanes per wavefront (vector-rate yardstick)."""
    _check(lib().lf_fma_rate(_ptr(out), int(blocks), int(iters), int(active), _stream(stream)))


def lf_last_error() -> str:
    return lib().lf_last_error().decode()


# names of every symbol include/lf.h declares (checked by the ABI test)
EXPORTS = ("lf_load_views", "lf_stereo_eyes", "lf_disk_extents", "lf_set_tune", "lf_render", "lf_render_noalloc",
           "lf_render_reference",
           "lf_prefilter", "lf_set_view_mask", "lf_two_level_mask", "lf_cache_config", "lf_cache_update",
           "lf_cache_resident", "lf_cache_page_misses", "lf_stream_copy", "lf_fma_rate",
           "lf_debug_candidates", "lf_query", "lf_render_stats", "lf_profile", "lf_profile_read",
           "lf_render_batch", "lf_autotune_batch", "lf_batch_frame_times", "lf_corrector_create",
           "lf_corrector_set_params", "lf_corrector_get_params", "lf_corrector_get_state", "lf_corrector_set_state",
           "lf_corrector_apply", "lf_corrector_train_step", "lf_corrector_free", "lf_last_error", "lf_free")
