"""The kernels' per-ray arithmetic (exact disk test + two-level inverse-depth
mesh walk, compiled for the host from the same header the kernels use)
against the FP64 oracle's per-view records, ray by ray, on the CPU."""
import ctypes
import os

import numpy as np
import pytest

import lfsynth
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SO = os.environ.get("LF_HOSTCHECK_LIB") or os.path.join(ROOT, "paper_1810_08860_amd", "liblf_hostcheck.so")


def _lib():
    if not os.path.exists(SO):
        pytest.skip("liblf_hostcheck.so not built")
    import torch  # noqa: F401  (same HIP runtime as the rest of the process)
    L = ctypes.CDLL(SO)
    L.lfh_trace.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                            ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p,
                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                            ctypes.c_void_p]
    return L


def _trace(V, o, e, geo_fmt=0, R=None):
    L = _lib()
    n, M = V.n, V.mesh_m
    nr = len(o)
    cand = np.zeros((nr, n), np.int32)
    hit = np.zeros((nr, n), np.int32)
    Xs = np.zeros((nr, n), np.float32)
    Ys = np.zeros((nr, n), np.float32)
    cells = np.zeros((nr, n), np.int32)
    z = np.ascontiguousarray(V.zdepth)
    c = np.ascontiguousarray(V.centres)
    r = np.ascontiguousarray(V.rot.reshape(-1, 9))
    o = np.ascontiguousarray(o, np.float64)
    e = np.ascontiguousarray(e, np.float64)
    L.lfh_trace(n, M, z.ctypes.data, c.ctypes.data, r.ctypes.data, V.src_fov_deg,
                V.disk_radius if R is None else R, geo_fmt, nr, o.ctypes.data, e.ctypes.data, cand.ctypes.data,
                hit.ctypes.data, Xs.ctypes.data, Ys.ctypes.data, cells.ctypes.data)
    return cand, hit, Xs, Ys, cells


def _compare(V, ov, o, e, geo_fmt=0, xy_tol=2e-5):
    cand, hit, Xs, Ys, cells = _trace(V, o, e, geo_fmt)
    ts = np.tan(np.radians(V.src_fov_deg / 2))
    dom = 1 - 1 / V.mesh_m
    n_hits, bad_xy = 0, 0
    for k in range(len(o)):
        rec = oracle.records(ov, o[k], e[k])
        band = np.abs(rec["rho"]) <= 1e-5
        assert ((cand[k] == rec["cand"]) | band).all(), k
        both = (cand[k] == 1) & (rec["cand"] == 1)
        edge = np.zeros(V.n, bool)
        h = rec["hit"] == 1
        edge[h] = np.minimum(dom - np.abs(rec["Xs"][h] / ts), dom - np.abs(rec["Ys"][h] / ts)) < 1e-6
        ok = (hit[k] == rec["hit"]) | ~both | edge
        assert ok.all(), (k, np.nonzero(~ok))
        m = both & (hit[k] == 1) & (rec["hit"] == 1)
        d = np.maximum(np.abs(Xs[k][m] - rec["Xs"][m]), np.abs(Ys[k][m] - rec["Ys"][m]))
        bad_xy += int((d > xy_tol).sum())
        n_hits += int(m.sum())
    return n_hits, bad_xy, cells


def test_host_ray_math_matches_oracle_tiny(tiny, tiny_oracle):
    rng = np.random.default_rng(3)
    pxy = rng.uniform(0, 256, (400, 2))
    o, e = oracle.eye_rays(tiny.head_pos[0], tiny.head_rot[0], tiny.hfov_deg, 256, 256, pxy)
    n_hits, bad, cells = _compare(tiny.views, tiny_oracle, o, e)
    # a flip between two surfaces (an occlusion fold) is the only allowed disagreement
    assert n_hits > 1500 and bad <= 0.002 * n_hits, (n_hits, bad)
    print("hits", n_hits, "xy mismatches", bad, "mean cells per candidate", cells[cells > 0].mean())


def test_host_ray_math_matches_oracle_dense_rig():
    """More views, smaller disks, different scene seed and random eyes."""
    V = lfsynth.make_views(256, 96, 96, 6, seed=9)
    ov = oracle.OracleViews.from_views(V)
    p, R = lfsynth.poses(31, 3, 0.25)
    rng = np.random.default_rng(4)
    total, bad_total = 0, 0
    for k in range(3):
        pxy = rng.uniform(0, 200, (150, 2))
        o, e = oracle.eye_rays(p[k], R[k], 100.0, 200, 180, pxy)
        n_hits, bad, _ = _compare(V, ov, o, e)
        total += n_hits
        bad_total += bad
    assert total > 1500 and bad_total <= 0.002 * total, (total, bad_total)


def test_host_ray_math_fp16_geometry_close(tiny, tiny_oracle):
    """FP16 inverse depth moves hits by a bounded amount (not a parity claim)."""
    rng = np.random.default_rng(8)
    pxy = rng.uniform(0, 256, (200, 2))
    o, e = oracle.eye_rays(tiny.head_pos[0], tiny.head_rot[0], tiny.hfov_deg, 256, 256, pxy)
    cand, hit, Xs, Ys, _ = _trace(tiny.views, o, e, geo_fmt=1)
    c32, h32, X32, Y32, _ = _trace(tiny.views, o, e, geo_fmt=0)
    assert np.array_equal(cand, c32)
    m = (hit == 1) & (h32 == 1)
    assert (hit == h32).mean() > 0.999
    d = np.maximum(np.abs(Xs[m] - X32[m]), np.abs(Ys[m] - Y32[m]))
    # 1 source pixel of the tiny views is 2 tan(60)/128 = 0.027 in X
    assert np.quantile(d, 0.99) < 0.027 * 0.05
