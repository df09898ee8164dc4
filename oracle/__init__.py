"""FP64 CPU oracle for the disk-blended light field renderer (numpy wrapper).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only users. The product path never imports it.
It shares no code with the HIP library (see ``oracle.c`` for the readings of
the paper it implements).

Paper passages followed (all Sec. 4 of the paper):
  * eye rays .............. Sec. 4.1, Eq. (1)
  * disk-blended query .... Sec. 4.1, Eq. (2); linear kernel and disk placement
  * point-splat reading ... Sec. 4.1, Eq. (3) (constant-colour special case)
  * two-pass accumulate ... Sec. 4.2 (numerator / denominator, then divide)
  * intra-image occlusion . Sec. 4.2.2 (nearest hit within one view's mesh)
  * per-view mesh ......... Sec. 4.5 (depth map, two triangles per pixel)
  * offline query L-bar ... Sec. 5.1 (denser / larger support reconstruction),
    used here as the supersampled reference render.
  * prefilter ............. Sec. 5.1, Eqs. (4)-(5): Monte Carlo ratio estimate
    over disk points x pixel-basis points, rays through the real-time mesh,
    evaluated with the offline query.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# LF_ORACLE_LIB may name another build of these sources: the mutation test
# points it at copies with a planted mistake to show that the pins catch it
_SO = os.environ.get("LF_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_SRCS = [os.path.join(_HERE, "oracle.c"), os.path.join(_HERE, "conv_oracle.c")]


class _Views(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32), ("img_w", ctypes.c_int32), ("img_h", ctypes.c_int32), ("mesh_m", ctypes.c_int32),
        ("src_fov_deg", ctypes.c_double),
        ("centres", ctypes.c_void_p), ("rot", ctypes.c_void_p), ("rgba8", ctypes.c_void_p),
        ("zdepth", ctypes.c_void_p), ("zrange", ctypes.c_void_p),
        ("disk_radius", ctypes.c_double), ("disk_ext", ctypes.c_void_p),
        ("mode", ctypes.c_int32), ("threads", ctypes.c_int32),
        ("yuv_y", ctypes.c_void_p), ("yuv_uv", ctypes.c_void_p),
        ("rgtc_y", ctypes.c_void_p), ("rgtc_uv", ctypes.c_void_p),
        ("resident", ctypes.c_void_p), ("page", ctypes.c_int32),
    ]


class _Lists(ctypes.Structure):
    _fields_ = [("cap", ctypes.c_int32), ("cand", ctypes.c_void_p), ("cand_band", ctypes.c_void_p),
                ("contrib", ctypes.c_void_p), ("contrib_band", ctypes.c_void_p), ("n_cand", ctypes.c_void_p)]


REC_DTYPE = np.dtype([("a", "f8"), ("u", "f8"), ("v", "f8"), ("rho", "f8"), ("t_hit", "f8"),
                      ("Xs", "f8"), ("Ys", "f8"), ("rgb", "f8", (3,)), ("cand", "i4"), ("hit", "i4")])


def build(verbose: bool = False) -> str:
    """Compile liboracle.so with gcc (plain C, FP64, OpenMP)."""
    srcs = [s for s in _SRCS if os.path.exists(s)]
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-D_GNU_SOURCE", *srcs,
           "-o", _SO + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_SO + ".tmp", _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            raise RuntimeError(f"{_SO} is not built; run __graft_entry__.build() first")
        L = ctypes.CDLL(_SO)
        vp, i64, i32, f64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        L.orc_zrange.argtypes = [i32, i32, vp, vp]
        L.orc_eye_rays.argtypes = [vp, vp, f64, i32, i32, i64, vp, vp, vp]
        L.orc_disk.argtypes = [ctypes.POINTER(_Views), i32, vp, vp, vp, vp, vp, vp]
        L.orc_mesh_hit.argtypes = [ctypes.POINTER(_Views), i32, vp, vp]
        L.orc_mesh_hit.restype = f64
        L.orc_sample.argtypes = [ctypes.POINTER(_Views), i32, f64, f64, vp]
        L.orc_render_rays.argtypes = [ctypes.POINTER(_Views), i64, vp, vp, vp, vp, vp, ctypes.POINTER(_Lists)]
        L.orc_ray_records.argtypes = [ctypes.POINTER(_Views), vp, vp, vp]
        L.orc_prefilter.argtypes = [ctypes.POINTER(_Views), ctypes.POINTER(_Views), i32, f64, vp, i32, vp, vp, i32,
                                    i64, vp, vp, vp]
        L.orc_basis.argtypes = [i32, f64]
        L.orc_yuv420_encode.argtypes = [i32, i32, i32, vp, vp, vp]
        L.orc_rgtc_encode.argtypes = [i32, i32, i32, vp, vp, vp, vp]
        L.orc_rgtc_decode.argtypes = [i32, i32, i32, vp, vp, vp, vp]
        L.orc_visible_tiles.argtypes = [ctypes.POINTER(_Views), i64, vp, vp, i32, vp]
        L.orc_visible_tiles_band.argtypes = [ctypes.POINTER(_Views), i64, vp, vp, i32, f64, vp, vp]
        L.orc_basis.restype = f64
        L.orc_views_size.restype = i32
        L.orc_rec_size.restype = i32
        L.orc_max_threads.restype = i32
        if L.orc_views_size() != ctypes.sizeof(_Views):
            raise RuntimeError("orc_views layout mismatch")
        if L.orc_rec_size() != REC_DTYPE.itemsize:
            raise RuntimeError("orc_rec layout mismatch")
        _conv_bind(L)
        _lib = L
    return _lib


def _conv_bind(L):
    if not hasattr(L, "orc_conv3x3_fwd"):
        return
    vp, i32 = ctypes.c_void_p, ctypes.c_int32
    L.orc_conv3x3_fwd.argtypes = [vp, i32, i32, i32, i32, i32, vp, vp, vp, i32]
    L.orc_conv3x3_bwd.argtypes = [vp, vp, i32, i32, i32, i32, i32, vp, vp, vp, vp, vp, i32]


def _p(a: np.ndarray):
    return a.ctypes.data


def max_threads() -> int:
    return int(lib().orc_max_threads())


class OracleViews:
    """Light field as the oracle sees it: arrays kept alive for the C side."""

    def __init__(self, centres, rot, rgba8, zdepth, src_fov_deg, disk_radius, mode="traversal", threads=0,
                 disk_ext=None):
        self.centres = np.ascontiguousarray(centres, np.float64)
        self.rot = np.ascontiguousarray(np.asarray(rot, np.float64).reshape(-1, 9))
        self.rgba8 = np.ascontiguousarray(rgba8, np.uint8)
        self.zdepth = np.ascontiguousarray(zdepth, np.float32)
        n, h, w, _ = self.rgba8.shape
        m = self.zdepth.shape[1]
        assert self.centres.shape == (n, 3) and self.rot.shape == (n, 9) and self.zdepth.shape == (n, m, m)
        self.zrange = np.zeros((n, 2), np.float64)
        lib().orc_zrange(n, m, _p(self.zdepth), _p(self.zrange))
        self.disk_ext = None if disk_ext is None else np.ascontiguousarray(disk_ext, np.float64).reshape(n, 4)
        self.s = _Views(n, w, h, m, float(src_fov_deg), _p(self.centres), _p(self.rot), _p(self.rgba8),
                        _p(self.zdepth), _p(self.zrange), float(disk_radius),
                        None if self.disk_ext is None else _p(self.disk_ext),
                        1 if mode == "brute" else 0, int(threads), None, None, None, None, None, 0)

    @classmethod
    def from_views(cls, v, mode="traversal", threads=0, disk_radius=None, disk_ext=None):
        return cls(v.centres, v.rot, v.rgba8, v.zdepth, v.src_fov_deg,
                   v.disk_radius if disk_radius is None else disk_radius, mode, threads, disk_ext)

    @property
    def n(self):
        return self.s.n

    def with_disk_radius(self, r):
        o = OracleViews.__new__(OracleViews)
        o.__dict__.update(self.__dict__)
        o.s = _Views.from_buffer_copy(self.s)
        o.s.disk_radius = float(r)
        return o

    def with_disk_extents(self, ext):
        """Oval disks of Sec. 4.4 with per-view extents [n][4] (e+u, e-u, e+v, e-v);
        None restores circles of the disk radius."""
        o = self.with_disk_radius(self.s.disk_radius)
        o.disk_ext = None if ext is None else np.ascontiguousarray(ext, np.float64).reshape(self.n, 4)
        o.s.disk_ext = None if o.disk_ext is None else _p(o.disk_ext)
        return o

    def with_yuv420(self):
        """The same light field with its images in the YUV420 form of the
        paper's tile cache (Sec. 7.2), encoded by the oracle's own fixed-point
        BT.601 (see yuv420_encode); sampling then recombines luma and
        half-resolution chroma."""
        o = self.with_disk_radius(self.s.disk_radius)
        o.yuv_y, o.yuv_uv = yuv420_encode(self.rgba8)
        o.s.yuv_y, o.s.yuv_uv = _p(o.yuv_y), _p(o.yuv_uv)
        return o

    def with_yuv420_rgtc(self):
        """The YUV420 form transcoded to RGTC blocks (luma RGTC1, chroma RGTC2),
        the 4x smaller tile-cache form of Sec. 7.2, by the oracle's own encoder
        (see rgtc_encode); sampling reads the decoded block texels."""
        o = self.with_yuv420()
        o.rgtc_y, o.rgtc_uv = rgtc_encode(o.yuv_y, o.yuv_uv)
        o.s.rgtc_y, o.s.rgtc_uv = _p(o.rgtc_y), _p(o.rgtc_uv)
        return o

    def with_residency(self, resident, page=64):
        """Tile streaming (Sec. 4.2, Sec. 7.2): only the image tiles marked in
        resident [n][H/page][W/page] can be sampled; a view whose sample for a
        ray needs another tile is left out for that ray. None: every tile."""
        o = self.with_disk_radius(self.s.disk_radius)
        if resident is None:
            o.resident = None
            o.s.resident, o.s.page = None, 0
            return o
        H, W = self.rgba8.shape[1:3]
        if H % page or W % page:
            raise ValueError("image sizes must be multiples of the tile size")
        o.resident = np.ascontiguousarray(resident, np.uint8).reshape(self.n, H // page, W // page)
        o.s.resident, o.s.page = _p(o.resident), int(page)
        return o

    def with_mode(self, mode):
        o = self.with_disk_radius(self.s.disk_radius)
        o.s.mode = 1 if mode == "brute" else 0
        return o


# --------------------------------------------------------------------------- rays

def eye_rays(pos, rot, hfov_deg, W, H, pxy):
    """Eq. (1): rays through continuous pixel positions pxy (n,2); centre of pixel (x,y) is (x+.5, y+.5)."""
    pxy = np.ascontiguousarray(pxy, np.float64).reshape(-1, 2)
    n = pxy.shape[0]
    o = np.zeros((n, 3)); e = np.zeros((n, 3))
    pos = np.ascontiguousarray(pos, np.float64); rot = np.ascontiguousarray(np.asarray(rot, np.float64).reshape(9))
    lib().orc_eye_rays(_p(pos), _p(rot), float(hfov_deg), int(W), int(H), n, _p(pxy), _p(o), _p(e))
    return o, e


def pixel_centres(W, H, idx=None):
    if idx is None:
        idx = np.arange(W * H)
    idx = np.asarray(idx, np.int64)
    return np.stack([(idx % W) + 0.5, (idx // W) + 0.5], 1).astype(np.float64)


def stereo_eyes(head_pos, head_rot, ipd):
    """Two eyes offset by -/+ ipd/2 along the head's image +x axis, same orientation."""
    head_pos = np.asarray(head_pos, np.float64)
    R = np.asarray(head_rot, np.float64).reshape(3, 3)
    r = R[:, 0]
    return [(head_pos - 0.5 * ipd * r, R.copy()), (head_pos + 0.5 * ipd * r, R.copy())]


def render_rays(ov: OracleViews, o, e, cap: int = 0):
    o = np.ascontiguousarray(o, np.float64).reshape(-1, 3)
    e = np.ascontiguousarray(e, np.float64).reshape(-1, 3)
    n = o.shape[0]
    rgb = np.zeros((n, 3)); ws = np.zeros(n); cnt = np.zeros(n, np.int32)
    out = {"rgb": rgb, "wsum": ws, "count": cnt}
    Lp = None
    if cap > 0:
        for k in ("cand", "cand_band", "contrib", "contrib_band"):
            out[k] = np.full((n, cap), -1, np.int32)
        out["n_cand"] = np.zeros(n, np.int32)
        L = _Lists(cap, _p(out["cand"]), _p(out["cand_band"]), _p(out["contrib"]), _p(out["contrib_band"]),
                   _p(out["n_cand"]))
        Lp = ctypes.byref(L)
    lib().orc_render_rays(ctypes.byref(ov.s), n, _p(o), _p(e), _p(rgb), _p(ws), _p(cnt), Lp)
    return out


def render(ov: OracleViews, pos, rot, hfov_deg, W, H, idx=None, cap: int = 0, jitter=None):
    """Eq. (2) at the pixel centres listed in idx (all pixels if None)."""
    pxy = pixel_centres(W, H, idx)
    if jitter is not None:
        pxy = pxy + np.asarray(jitter, np.float64)
    o, e = eye_rays(pos, rot, hfov_deg, W, H, pxy)
    return render_rays(ov, o, e, cap)


def visible_tiles(ov: OracleViews, pos, rot, hfov_deg, W, H, page=64, idx=None):
    """The image tiles (n, H_src/page, W_src/page) that the eye's pixel-centre
    rays sample (every tap of every contributing view's bilinear sample)."""
    Hs, Ws = ov.rgba8.shape[1:3]
    if Hs % page or Ws % page:
        raise ValueError("image sizes must be multiples of the tile size")
    o, e = eye_rays(pos, rot, hfov_deg, W, H, pixel_centres(W, H, idx))
    vis = np.zeros((ov.n, Hs // page, Ws // page), np.uint8)
    lib().orc_visible_tiles(ctypes.byref(ov.s), o.shape[0], _p(o), _p(e), int(page), _p(vis))
    return vis


def visible_tiles_band(ov: OracleViews, pos, rot, hfov_deg, W, H, page=64, margin=1e-3, jitter=1e-3):
    """The visible tiles of an eye split by how firmly they are decided, for
    comparison with a float implementation: (must, may), each (n, H_src/page,
    W_src/page). must holds the tiles that the pixel-centre rays, and the same
    rays shifted by +-jitter pixels along x and y, all show through
    well-conditioned decisions (disk margin, mesh domain edge, taps more than
    `margin` texels from a texel boundary); may holds every tile one of those
    rays could show under a decision inside those bands (a surface flip under
    the jitter included). The exact visible set lies between the two."""
    Hs, Ws = ov.rgba8.shape[1:3]
    if Hs % page or Ws % page:
        raise ValueError("image sizes must be multiples of the tile size")
    if not 0.0 <= margin < 1.0:
        raise ValueError("margin must be in [0, 1) texels (the two tap choices around a boundary)")
    shape = (ov.n, Hs // page, Ws // page)
    must_all = np.ones(shape, np.uint8)
    may = np.zeros(shape, np.uint8)
    for d in ((0.0, 0.0), (jitter, 0.0), (-jitter, 0.0), (0.0, jitter), (0.0, -jitter)):
        o, e = eye_rays(pos, rot, hfov_deg, W, H, pixel_centres(W, H) + np.array(d))
        must = np.zeros(shape, np.uint8)
        lib().orc_visible_tiles_band(ctypes.byref(ov.s), o.shape[0], _p(o), _p(e), int(page), float(margin),
                                     _p(must), _p(may))
        must_all &= must
    return must_all, may


def render_reference(ov: OracleViews, pos, rot, hfov_deg, W, H, idx=None, ss: int = 4, disk_scale: float = 2.0,
                     jitter=None):
    """Offline reference: ss x ss regular sub-pixel rays per pixel, disks scaled by
    disk_scale, every view considered; the pixel is the box average of the sub-ray
    values (an uncovered sub-ray counts as 0). jitter (dx, dy) shifts every
    sub-ray by that many pixels (stability checks)."""
    if idx is None:
        idx = np.arange(W * H)
    idx = np.asarray(idx, np.int64)
    base = np.stack([(idx % W).astype(np.float64), (idx // W).astype(np.float64)], 1)
    if jitter is not None:
        base = base + np.asarray(jitter, np.float64)
    offs = (np.arange(ss) + 0.5) / ss
    sub = np.stack(np.meshgrid(offs, offs, indexing="xy"), -1).reshape(-1, 2)  # (ss*ss, 2) as (x, y)
    pxy = (base[:, None, :] + sub[None, :, :]).reshape(-1, 2)
    o, e = eye_rays(pos, rot, hfov_deg, W, H, pxy)
    big = ov.with_disk_radius(ov.s.disk_radius * disk_scale)
    if ov.disk_ext is not None:
        big = big.with_disk_extents(ov.disk_ext * disk_scale)
    r = render_rays(big, o, e)
    return r["rgb"].reshape(len(idx), ss * ss, 3).mean(1)


def disk_extents(centres, rot):
    """Extents (e+u, e-u, e+v, e-v) of each view's asymmetric oval disk
    (Sec. 4.4): the disk reaches the centres of its 1-ring neighbours in a
    Delaunay triangulation of the disk centres, and each extent is the furthest
    1-ring neighbour along that direction of the disk's (u, v) axes (the
    neighbour's centre offset projected on the view's r and u axes). For
    centres on a sphere about the origin the Delaunay triangulation is the
    convex hull of the centres' directions. Returns [n][4] and the 1-ring sets."""
    from scipy.spatial import ConvexHull
    c = np.asarray(centres, np.float64).reshape(-1, 3)
    R = np.asarray(rot, np.float64).reshape(-1, 3, 3)
    unit = c / np.linalg.norm(c, axis=1, keepdims=True)
    ring = [set() for _ in range(len(c))]
    for a, b, d in ConvexHull(unit).simplices:
        ring[a] |= {b, d}
        ring[b] |= {a, d}
        ring[d] |= {a, b}
    ext = np.zeros((len(c), 4))
    for i in range(len(c)):
        q = c[sorted(ring[i])] - c[i]
        du, dv = q @ R[i][:, 0], q @ R[i][:, 1]
        ext[i] = (du.max(), (-du).max(), dv.max(), (-dv).max())
    if not (ext > 0).all():
        raise ValueError("a disk has no 1-ring neighbour on one side of an axis")
    return ext, ring


def yuv420_encode(rgba8):
    """YUV420 planes (luma (n,H,W), chroma (n,H/2,W/2,2) = Cb, Cr) of RGBA8
    images by the oracle's fixed-point full-range BT.601 (oracle.c)."""
    rgba8 = np.ascontiguousarray(rgba8, np.uint8)
    n, H, W, _ = rgba8.shape
    if H % 2 or W % 2:
        raise ValueError("YUV420 needs even image sizes")
    y = np.zeros((n, H, W), np.uint8)
    uv = np.zeros((n, H // 2, W // 2, 2), np.uint8)
    lib().orc_yuv420_encode(n, W, H, _p(rgba8), _p(y), _p(uv))
    return y, uv


def rgtc_encode(y, uv):
    """RGTC blocks of YUV420 planes (oracle.c, orc_rgtc_encode): luma (n,H,W)
    as RGTC1 blocks (n,H/4,W/4,8) and chroma (n,H/2,W/2,2) as RGTC2 blocks
    (n,H/8,W/8,16), row-major over blocks. Sizes must be multiples of 8."""
    y = np.ascontiguousarray(y, np.uint8)
    uv = np.ascontiguousarray(uv, np.uint8)
    n, H, W = y.shape
    if H % 8 or W % 8:
        raise ValueError("RGTC needs image sizes that are multiples of 8")
    assert uv.shape == (n, H // 2, W // 2, 2)
    yb = np.zeros((n, H // 4, W // 4, 8), np.uint8)
    uvb = np.zeros((n, H // 8, W // 8, 16), np.uint8)
    lib().orc_rgtc_encode(n, W, H, _p(y), _p(uv), _p(yb), _p(uvb))
    return yb, uvb


def rgtc_decode(yb, uvb):
    """Decoded planes of RGTC blocks, real values in 0..255: luma (n,H,W) and
    chroma (n,H/2,W/2,2)."""
    yb = np.ascontiguousarray(yb, np.uint8)
    uvb = np.ascontiguousarray(uvb, np.uint8)
    n, H, W = yb.shape[0], 4 * yb.shape[1], 4 * yb.shape[2]
    assert uvb.shape == (n, H // 8, W // 8, 16)
    y = np.zeros((n, H, W), np.float64)
    uv = np.zeros((n, H // 2, W // 2, 2), np.float64)
    lib().orc_rgtc_decode(n, W, H, _p(yb), _p(uvb), _p(y), _p(uv))
    return y, uv


BASIS = {"box": 0, "lanczos2": 1}


def basis(kind, d):
    """Pixel reconstruction basis of the prefilter (one axis): box or Lanczos-2."""
    return float(lib().orc_basis(BASIS[kind], float(d)))


def prefilter(lbar: OracleViews, target: OracleViews, i, radius, disk_pts, pix_offs, kind="lanczos2", idx=None,
              aperture_ext=None):
    """Prefiltered colour (Sec. 5.1, Eq. (5)) of the pixels idx (all if None) of
    view i of the real-time model `target`: J samples pair the unit-disk points
    disk_pts (J,2) (scaled by the target disk radius) with pixel offsets
    pix_offs (J,2) (pixels from the pixel centre); each ray starts at the disk
    point and passes through target view i's mesh point at the offset image
    position; `lbar` (the offline model) answers the ray query. A sample
    without a mesh point or whose ray no offline disk covers is left out of
    both sums. aperture_ext (e+u, e-u, e+v, e-v) in metres makes view i's
    aperture the oval disk of Sec. 4.4 instead of the circle of `radius`: a
    unit-disk point maps by the extents of its quadrant, and its weight carries
    that quadrant's area factor e_u e_v (Eq. (4) integrates over the disk's
    area). Returns {"rgb": (n,3), "wsum": (n,)} with wsum the denominator of
    Eq. (5)."""
    W, H = target.s.img_w, target.s.img_h
    if idx is None:
        idx = np.arange(W * H)
    idx = np.ascontiguousarray(idx, np.int64)
    dp = np.ascontiguousarray(disk_pts, np.float64).reshape(-1, 2)
    po = np.ascontiguousarray(pix_offs, np.float64).reshape(-1, 2)
    assert dp.shape == po.shape
    rgb = np.zeros((len(idx), 3))
    ws = np.zeros(len(idx))
    ext = None
    if aperture_ext is not None:
        ext = np.ascontiguousarray(aperture_ext, np.float64).reshape(4)
        if not (np.isfinite(ext).all() and (ext > 0).all()):
            raise ValueError("aperture extents must be finite and positive")
    lib().orc_prefilter(ctypes.byref(lbar.s), ctypes.byref(target.s), int(i), float(radius),
                        None if ext is None else _p(ext), dp.shape[0], _p(dp), _p(po), BASIS[kind], len(idx), _p(idx),
                        _p(rgb), _p(ws))
    return {"rgb": rgb, "wsum": ws}


def disk(ov: OracleViews, i, o, e):
    o = np.ascontiguousarray(o, np.float64); e = np.ascontiguousarray(e, np.float64)
    out = np.zeros(4)
    ptrs = [out.ctypes.data + 8 * k for k in range(4)]
    lib().orc_disk(ctypes.byref(ov.s), int(i), _p(o), _p(e), *ptrs)
    return tuple(out)


def mesh_hit(ov: OracleViews, i, o, e) -> float:
    o = np.ascontiguousarray(o, np.float64); e = np.ascontiguousarray(e, np.float64)
    return float(lib().orc_mesh_hit(ctypes.byref(ov.s), int(i), _p(o), _p(e)))


def sample(ov: OracleViews, i, Xs, Ys):
    out = np.zeros(3)
    lib().orc_sample(ctypes.byref(ov.s), int(i), float(Xs), float(Ys), _p(out))
    return out


def records(ov: OracleViews, o, e):
    o = np.ascontiguousarray(o, np.float64); e = np.ascontiguousarray(e, np.float64)
    recs = np.zeros(ov.n, REC_DTYPE)
    lib().orc_ray_records(ctypes.byref(ov.s), _p(o), _p(e), _p(recs))
    return recs


# =========================================================================== corrector (conv) oracle
#
# A 4-layer 3x3 convolutional residual corrector of the rendered image
# (5 input channels: R, G, B, W/4, n/8 with W the disk-weight sum and n the
# number of contributing views; 32, 32, 32 hidden channels with ReLU; 3 output
# channels = the residual added to the render). Layer weights are
# w[ky][kx][ci][co] followed by b[co]; the flat parameter vector concatenates
# the layers in order (20,835 values).

CORRECTOR_LAYERS = ((5, 32, True), (32, 32, True), (32, 32, True), (32, 3, False))
CORRECTOR_W_SCALE, CORRECTOR_N_SCALE = 4.0, 8.0


def corrector_num_params():
    return sum(9 * ci * co + co for ci, co, _ in CORRECTOR_LAYERS)


def conv3x3_fwd(x, w, b, relu):
    """x (N,H,W,Cin), w (3,3,Cin,Cout), b (Cout,) -> act(conv(x)) (N,H,W,Cout), FP64."""
    x = np.ascontiguousarray(x, np.float64)
    w = np.ascontiguousarray(w, np.float64)
    b = np.ascontiguousarray(b, np.float64)
    N, H, W, Cin = x.shape
    Cout = w.shape[3]
    assert w.shape == (3, 3, Cin, Cout) and b.shape == (Cout,)
    y = np.zeros((N, H, W, Cout))
    lib().orc_conv3x3_fwd(_p(x), N, H, W, Cin, Cout, _p(w), _p(b), _p(y), 1 if relu else 0)
    return y


def conv3x3_bwd(x, y, w, dy, relu, want_dx=True):
    """Gradients of a layer given dL/dy: (dx, dw, db)."""
    x = np.ascontiguousarray(x, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    w = np.ascontiguousarray(w, np.float64)
    dy = np.ascontiguousarray(dy, np.float64)
    N, H, W, Cin = x.shape
    Cout = w.shape[3]
    dx = np.zeros_like(x) if want_dx else None
    dw = np.zeros_like(w)
    db = np.zeros(Cout)
    lib().orc_conv3x3_bwd(_p(x), _p(y), N, H, W, Cin, Cout, _p(w), _p(dy), _p(dx) if want_dx else None, _p(dw),
                          _p(db), 1 if relu else 0)
    return dx, dw, db


def corrector_unpack(params):
    params = np.asarray(params, np.float64)
    out, o = [], 0
    for ci, co, _ in CORRECTOR_LAYERS:
        w = params[o:o + 9 * ci * co].reshape(3, 3, ci, co)
        o += 9 * ci * co
        b = params[o:o + co]
        o += co
        out.append((w, b))
    assert o == params.size
    return out


def corrector_input(rgb, wsum, count):
    """Network input (N,H,W,5) from the render's colour, weight sum and view count."""
    rgb = np.asarray(rgb, np.float64)
    return np.concatenate([rgb, np.asarray(wsum, np.float64)[..., None] / CORRECTOR_W_SCALE,
                           np.asarray(count, np.float64)[..., None] / CORRECTOR_N_SCALE], -1)


def corrector_forward(params, x):
    """Residual (N,H,W,3) and the activations of every layer (input first)."""
    acts = [np.asarray(x, np.float64)]
    for (w, b), (_, _, relu) in zip(corrector_unpack(params), CORRECTOR_LAYERS):
        acts.append(conv3x3_fwd(acts[-1], w, b, relu))
    return acts[-1], acts


def corrector_loss_grad(params, x, render, ref):
    """Mean squared error of (render + residual) against ref over every pixel
    and channel, and its gradient w.r.t. the flat parameters."""
    resid, acts = corrector_forward(params, x)
    diff = np.asarray(render, np.float64) + resid - np.asarray(ref, np.float64)
    loss = float((diff ** 2).mean())
    g = 2.0 * diff / diff.size
    grads = []
    layers = corrector_unpack(params)
    for li in range(len(layers) - 1, -1, -1):
        w, _ = layers[li]
        relu = CORRECTOR_LAYERS[li][2]
        dx, dw, db = conv3x3_bwd(acts[li], acts[li + 1], w, g, relu, want_dx=li > 0)
        grads.append((dw, db))
        g = dx
    flat = []
    for dw, db in reversed(grads):
        flat += [dw.ravel(), db]
    return loss, np.concatenate(flat)


def corrector_apply(params, x, render, thresh):
    """render + residual, except pixels whose largest |residual| component
    exceeds thresh keep the render (fallback); returns (out, fallback mask)."""
    resid, _ = corrector_forward(params, x)
    fb = np.abs(resid).max(-1) > thresh
    out = np.where(fb[..., None], render, render + resid)
    return out, fb
