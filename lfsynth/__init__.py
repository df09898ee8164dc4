"""Seeded synthetic inputs for the light field renderer (inputs only).

The C library ``liblfsynth.so`` ray-casts an analytic scene into the source
views and depth maps; this module wraps it with numpy. Nothing here implements
the reconstruction itself: the FP64 oracle and the HIP path both consume what
this module writes, and neither shares any other code with the other.

Workload recipes follow the paper's capture geometry (Sec. 3, a 70 cm capture
sphere; Sec. 6, about a thousand views of about a megapixel; Sec. 7.1,
120-degree views; Sec. 4.5, per-view meshes from per-view depth maps):

* ``tiny``  -- 64 views, 128x128 RGBA8 images, 128x128 depth, 3 spheres in a
  6 m box; one 256x256 mono eye, 90 deg, head in a 0.2 m ball.
* ``full``  -- 1024 views, 1024x1024 RGBA8, 256x256 depth, 12 spheres;
  stereo 2 x 1440x1600 eyes, 100 deg, IPD 64 mm, 3000 heads in a 0.25 m ball.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liblfsynth.so")
_SRC = os.path.join(_HERE, "lfsynth.c")

MAX_SPHERES = 64


class SynScene(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32),
        ("texture", ctypes.c_int32),
        ("n_spheres", ctypes.c_int32),
        ("pad", ctypes.c_int32),
        ("sphere_c", (ctypes.c_double * 3) * MAX_SPHERES),
        ("sphere_r", ctypes.c_double * MAX_SPHERES),
        ("sphere_rgb", (ctypes.c_double * 3) * MAX_SPHERES),
        ("box_half", ctypes.c_double),
        ("box_rgb", (ctypes.c_double * 3) * 6),
        ("plane_n", ctypes.c_double * 3),
        ("plane_d", ctypes.c_double),
        ("const_rgb", ctypes.c_double * 3),
        ("checker", ctypes.c_double),
        ("noise_cell", ctypes.c_double),
        ("smooth_period", ctypes.c_double),
        ("noise_seed", ctypes.c_uint64),
    ]


def build(verbose: bool = False) -> str:
    """Compile liblfsynth.so with gcc (OpenMP)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-D_GNU_SOURCE",
           _SRC, "-o", _SO + ".tmp", "-lm"]
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
        dp = ctypes.POINTER(ctypes.c_double)
        L.syn_rig.argtypes = [ctypes.c_int32, ctypes.c_double, dp, dp]
        L.syn_mean_nn.argtypes = [ctypes.c_int32, dp]
        L.syn_mean_nn.restype = ctypes.c_double
        L.syn_min_nn.argtypes = [ctypes.c_int32, dp]
        L.syn_min_nn.restype = ctypes.c_double
        L.syn_scene_spheres.argtypes = [ctypes.POINTER(SynScene), ctypes.c_uint64, ctypes.c_int32, ctypes.c_double]
        L.syn_scene_plane.argtypes = [ctypes.POINTER(SynScene), dp, ctypes.c_double, ctypes.c_int32,
                                      ctypes.c_double, dp]
        L.syn_texture.argtypes = [ctypes.POINTER(SynScene), ctypes.c_int32, dp, dp]
        L.syn_cast.argtypes = [ctypes.POINTER(SynScene), dp, dp, ctypes.POINTER(ctypes.c_int32)]
        L.syn_cast.restype = ctypes.c_double
        L.syn_render_views.argtypes = [ctypes.POINTER(SynScene), ctypes.c_int32, dp, dp, ctypes.c_double,
                                       ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
                                       ctypes.c_void_p, ctypes.c_int32]
        L.syn_render_views.restype = ctypes.c_int64
        L.syn_poses.argtypes = [ctypes.c_uint64, ctypes.c_int32, ctypes.c_double, dp, dp]
        L.syn_uniform.argtypes = [ctypes.c_uint64, ctypes.c_int64, dp]
        L.syn_scene_size.restype = ctypes.c_int32
        if L.syn_scene_size() != ctypes.sizeof(SynScene):
            raise RuntimeError("syn_scene layout mismatch between C and Python")
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ----------------------------------------------------------------------------- rig / scene / poses

def rig(n: int, radius: float = 0.35):
    """Fibonacci-lattice centres (n,3) and outward frames (n,3,3), columns (r,u,f)."""
    c = np.zeros((n, 3), np.float64)
    r = np.zeros((n, 3, 3), np.float64)
    lib().syn_rig(n, radius, _dp(c), _dp(r))
    return c, r


def mean_nn(centres: np.ndarray) -> float:
    c = np.ascontiguousarray(centres, np.float64)
    return float(lib().syn_mean_nn(c.shape[0], _dp(c)))


def min_nn(centres: np.ndarray) -> float:
    c = np.ascontiguousarray(centres, np.float64)
    return float(lib().syn_min_nn(c.shape[0], _dp(c)))


def scene_spheres(seed: int, n_spheres: int, box_half: float = 6.0) -> SynScene:
    sc = SynScene()
    lib().syn_scene_spheres(ctypes.byref(sc), seed, n_spheres, box_half)
    return sc


def scene_plane(normal, d: float, texture: int = 1, period: float = 1.0, rgb=(0.5, 0.5, 0.5)) -> SynScene:
    sc = SynScene()
    n = np.asarray(normal, np.float64).copy()
    col = np.asarray(rgb, np.float64).copy()
    lib().syn_scene_plane(ctypes.byref(sc), _dp(n), d, texture, period, _dp(col))
    return sc


def texture(sc: SynScene, obj: int, p) -> np.ndarray:
    pp = np.asarray(p, np.float64).copy()
    out = np.zeros(3, np.float64)
    lib().syn_texture(ctypes.byref(sc), obj, _dp(pp), _dp(out))
    return out


def cast(sc: SynScene, o, d):
    oo = np.asarray(o, np.float64).copy()
    dd = np.asarray(d, np.float64).copy()
    obj = ctypes.c_int32(-1)
    t = lib().syn_cast(ctypes.byref(sc), _dp(oo), _dp(dd), ctypes.byref(obj))
    return t, obj.value


def render_views(sc: SynScene, centres, rot, fov_deg: float, img_res: int, mesh_m: int,
                 threads: int = 0, images: bool = True, depth: bool = True):
    """Ray-cast RGBA8 images (n,H,W,4) and z-depth maps (n,M,M) float32."""
    c = np.ascontiguousarray(centres, np.float64)
    r = np.ascontiguousarray(rot, np.float64).reshape(-1, 9)
    n = c.shape[0]
    rgba = np.empty((n, img_res, img_res, 4), np.uint8) if images else None
    z = np.empty((n, mesh_m, mesh_m), np.float32) if depth else None
    esc = lib().syn_render_views(ctypes.byref(sc), n, _dp(c), _dp(np.ascontiguousarray(r)), fov_deg,
                                 img_res, img_res,
                                 rgba.ctypes.data if rgba is not None else None, mesh_m,
                                 z.ctypes.data if z is not None else None, threads)
    return rgba, z, int(esc)


def poses(seed: int, count: int, ball_radius: float):
    """Head positions (count,3) uniform in a ball; frames (count,3,3) uniform on SO(3)."""
    p = np.zeros((count, 3), np.float64)
    r = np.zeros((count, 3, 3), np.float64)
    lib().syn_poses(seed, count, ball_radius, _dp(p), _dp(r))
    return p, r


def uniform(seed: int, count: int) -> np.ndarray:
    out = np.zeros(count, np.float64)
    lib().syn_uniform(seed, count, _dp(out))
    return out


def prefilter_samples(seed: int, count: int, half_width: float):
    """Seeded sample pattern for a Monte Carlo prefilter: count points uniform
    in the unit disk (count,2) and count offsets uniform in the square
    [-half_width, half_width]^2 (count,2). Samples come in antithetic pairs
    (p, -p) for both sets, so the pattern is point-symmetric (count even)."""
    if count % 2:
        raise ValueError("count must be even (antithetic pairs)")
    h = count // 2
    u = uniform(seed, 4 * h).reshape(h, 4)
    r = np.sqrt(u[:, 0])
    a = 2.0 * np.pi * u[:, 1]
    disk = np.stack([r * np.cos(a), r * np.sin(a)], 1)
    offs = (2.0 * u[:, 2:4] - 1.0) * half_width
    return np.concatenate([disk, -disk]), np.concatenate([offs, -offs])


# ----------------------------------------------------------------------------- workloads

@dataclass
class Views:
    """Everything the renderer needs about the captured light field."""
    centres: np.ndarray          # (n,3) float64, metres
    rot: np.ndarray              # (n,3,3) float64, columns (r,u,f)
    rgba8: np.ndarray            # (n,H,W,4) uint8
    zdepth: np.ndarray           # (n,M,M) float32, z along f, metres
    src_fov_deg: float
    disk_radius: float
    scene: SynScene = field(repr=False, default=None)

    @property
    def n(self):
        return self.centres.shape[0]

    @property
    def img_res(self):
        return self.rgba8.shape[1]

    @property
    def mesh_m(self):
        return self.zdepth.shape[1]


@dataclass
class Workload:
    name: str
    views: Views
    head_pos: np.ndarray         # (P,3)
    head_rot: np.ndarray         # (P,3,3)
    hfov_deg: float
    eye_w: int
    eye_h: int
    stereo: bool
    ipd: float
    seed: int


WORKLOADS = {
    # name: (views, img, mesh, spheres, eye_w, eye_h, hfov, stereo, poses, ball)
    "tiny": (64, 128, 128, 3, 256, 256, 90.0, False, 1, 0.2),
    "full": (1024, 1024, 256, 12, 1440, 1600, 100.0, True, 3000, 0.25),
}


def make_views(n: int, img_res: int, mesh_m: int, n_spheres: int, seed: int,
               radius: float = 0.35, fov_deg: float = 120.0, disk_factor: float = 1.5,
               threads: int = 0) -> Views:
    c, r = rig(n, radius)
    sc = scene_spheres(seed, n_spheres)
    rgba, z, esc = render_views(sc, c, r, fov_deg, img_res, mesh_m, threads)
    if esc:
        raise RuntimeError(f"{esc} rays escaped the scene")
    return Views(c, r, rgba, z, fov_deg, disk_factor * mean_nn(c), sc)


def make_workload(name: str, seed: int = 0, n_poses: int | None = None, threads: int = 0,
                  n_views: int | None = None) -> Workload:
    nv, img, mesh, ns, ew, eh, hfov, stereo, npose, ball = WORKLOADS[name]
    if n_views is not None:
        nv = n_views
    v = make_views(nv, img, mesh, ns, seed, threads=threads)
    p, r = poses(seed + 1000, n_poses or npose, ball)
    return Workload(name, v, p, r, hfov, ew, eh, stereo, 0.064 if stereo else 0.0, seed)
