"""The kernels' per-ray arithmetic (exact disk test, the two-level
inverse-depth mesh walk and the single walk from a culling start bound,
compiled for the host from the same header the kernels use) against the
FP64 oracle's per-view records, ray by ray, on the CPU; and the pieces of
the start bound (cell box of a tile's rays, FP16 rounding up)."""
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
    for f in (L.lfh_trace, L.lfh_trace_top):
        f.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                      ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p,
                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                      ctypes.c_void_p]
    L.lfh_tile_box.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                               ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_int32, ctypes.c_float,
                               ctypes.c_float, ctypes.c_void_p]
    L.lfh_half_up.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]
    L.lfh_load_cell.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p]
    L.lfh_bilinear.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_float,
                               ctypes.c_float, ctypes.c_void_p]
    return L


def _trace(V, o, e, geo_fmt=0, R=None, top=False):
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
    rc = (L.lfh_trace_top if top else L.lfh_trace)(n, M, z.ctypes.data, c.ctypes.data, r.ctypes.data,
                                                    V.src_fov_deg, V.disk_radius if R is None else R, geo_fmt, nr,
                                                    o.ctypes.data, e.ctypes.data, cand.ctypes.data, hit.ctypes.data,
                                                    Xs.ctypes.data, Ys.ctypes.data, cells.ctypes.data)
    assert rc == 0, rc
    return cand, hit, Xs, Ys, cells


def _compare(V, ov, o, e, geo_fmt=0, xy_tol=2e-5, top=False):
    cand, hit, Xs, Ys, cells = _trace(V, o, e, geo_fmt, top=top)
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


@pytest.mark.parametrize("top", [False, True], ids=["two_level", "start_bound"])
def test_walk_forms_match_oracle_full_size_sample(top):
    """The full-size field (1024 views, 256^2 depth) and stereo eyes of the
    headline workload; both walks against the oracle ray by ray."""
    V = lfsynth.make_views(1024, 32, 256, 12, seed=0)
    ov = oracle.OracleViews.from_views(V)
    p, R = lfsynth.poses(1000, 2, 0.25)
    rng = np.random.default_rng(6)
    total, bad_total = 0, 0
    for k in range(2):
        eye = oracle.stereo_eyes(p[k], R[k], 0.064)[k]
        pxy = rng.uniform(0, [1440, 1600], (60, 2))
        o, e = oracle.eye_rays(eye[0], eye[1], 100.0, 1440, 1600, pxy)
        n_hits, bad, _ = _compare(V, ov, o, e, top=top)
        total += n_hits
        bad_total += bad
    assert total > 500 and bad_total <= 0.002 * total, (total, bad_total)


@pytest.mark.parametrize("geo_fmt", [0, 1])
def test_start_bound_walk_finds_the_two_level_hits(tiny, geo_fmt):
    """Same candidates and the same hits: a cell's root does not depend on
    where the walk entered the cell, so the two walks agree bit for bit
    wherever both reach the root's cell from above (all but rounding ties)."""
    rng = np.random.default_rng(12)
    pxy = rng.uniform(0, 256, (400, 2))
    o, e = oracle.eye_rays(tiny.head_pos[0], tiny.head_rot[0], tiny.hfov_deg, 256, 256, pxy)
    c0, h0, X0, Y0, n0 = _trace(tiny.views, o, e, geo_fmt=geo_fmt)
    c1, h1, X1, Y1, n1 = _trace(tiny.views, o, e, geo_fmt=geo_fmt, top=True)
    assert np.array_equal(c0, c1)
    assert (h0 == h1).mean() > 0.999, (h0 != h1).sum()
    m = (h0 == 1) & (h1 == 1)
    assert m.sum() > 1500
    d = np.maximum(np.abs(X0[m] - X1[m]), np.abs(Y0[m] - Y1[m]))
    assert (d == 0).mean() > 0.999 and d.max() < 1e-5, ((d > 0).sum(), d.max())
    assert n1[c1 == 1].mean() <= n0[c0 == 1].mean()
    print("cells per candidate: two-level", n0[c0 == 1].mean(), "start bound", n1[c1 == 1].mean())


def test_tile_cell_box_holds_every_ray_of_the_rectangle():
    """Rays through random points of a rectangle, at random inverse depths of
    the range, land (in FP64) inside the cell box computed from the corners."""
    L = _lib()
    rng = np.random.default_rng(21)
    M = 256
    sM, cM = np.float32(M / (2 * np.tan(np.radians(60)))), np.float32(0.5 * (M - 1))
    checked = 0
    for trial in range(300):
        # a rotation close to the identity (the eye looks roughly along the view's axis)
        a = rng.normal(size=3) * 0.3
        K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
        Rm = np.eye(3) + np.sin(np.linalg.norm(a)) / np.linalg.norm(a) * K + \
            (1 - np.cos(np.linalg.norm(a))) / np.linalg.norm(a) ** 2 * K @ K
        m = Rm.astype(np.float32).reshape(9)
        o = np.array([rng.uniform(-0.05, 0.05), rng.uniform(-0.05, 0.05), rng.uniform(-0.6, -0.05)], np.float32)
        wmin, wmax = np.float32(rng.uniform(0.1, 0.5)), np.float32(rng.uniform(0.6, 3.0))
        X0 = np.float32(rng.uniform(-0.8, 0.7)); X1 = np.float32(X0 + rng.uniform(0.001, 0.1))
        Y0 = np.float32(rng.uniform(-0.7, 0.8)); Y1 = np.float32(Y0 - rng.uniform(0.001, 0.1))
        box = np.zeros(4, np.int32)
        ok = L.lfh_tile_box(m.ctypes.data, o.ctypes.data, wmin, wmax, X0, X1, Y0, Y1, M, sM, cM, box.ctypes.data)
        if not ok:
            continue
        if box[0] > box[1]:
            continue  # the rectangle's rays miss the mesh domain
        X = rng.uniform(X0, X1, 200); Y = rng.uniform(Y1, Y0, 200); w = rng.uniform(wmin, wmax, 200)
        md = m.astype(np.float64).reshape(3, 3)
        ex, ey, ez = md @ np.stack([X, Y, np.ones_like(X)])
        Vx, Vy = ex / ez, ey / ez
        Dx, Dy = o[0] - o[2] * Vx, o[1] - o[2] * Vy
        gx = (Vx + w * Dx) * sM + cM
        gy = cM - (Vy + w * Dy) * sM
        inside = (gx >= 0) & (gx <= M - 1) & (gy >= 0) & (gy <= M - 1)
        j = np.minimum(np.floor(gx), M - 2); k = np.minimum(np.floor(gy), M - 2)
        assert ((j >= box[0]) & (j <= box[1]) & (k >= box[2]) & (k <= box[3]) | ~inside).all(), (trial, box)
        checked += int(inside.sum())
    assert checked > 10000, checked


def test_half_up_bits_rounds_up_to_the_next_half():
    L = _lib()
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.uniform(1e-3, 50.0, 20000), np.float16(rng.uniform(0.01, 10, 1000)).astype(np.float64),
                        [65504.0, 65520.0, 1e6]]).astype(np.float32)
    bits = np.zeros(len(x), np.uint16)
    L.lfh_half_up(len(x), x.ctypes.data, bits.ctypes.data)
    h = bits.view(np.float16).astype(np.float32)
    assert (h >= x).all()
    below = (bits - 1).view(np.float16).astype(np.float32)
    assert (below < x).all()
    # representable values are kept as they are; beyond the FP16 range: +inf
    exact = np.float16(x).astype(np.float32) == x
    assert (h[exact] == x[exact]).all()
    assert np.isinf(h[-2:]).all()


def test_sixteen_bit_cell_codes_decode_to_base_plus_code_times_scale():
    """LF_GEO_U16 layout: a view's (base, scale) as two floats, then per cell
    four little-endian 16-bit codes in the order (w00, w10, w01, w11); a
    corner decodes to base + code * scale (checked against numpy in FP64, up
    to FP32 rounding of one multiply-add)."""
    L = _lib()
    rng = np.random.default_rng(9)
    base, scale = np.float32(0.2137), np.float32(6.5 / 65535)
    codes = rng.integers(0, 65536, (37, 4)).astype(np.uint16)
    codes[0] = [0, 65535, 1, 32768]
    buf = np.concatenate([np.array([base, scale], np.float32).view(np.uint8), codes.reshape(-1).view(np.uint8)])
    out = np.zeros(4, np.float32)
    for idx in range(len(codes)):
        L.lfh_load_cell(2, buf.ctypes.data + 8, idx, out.ctypes.data)
        want = float(base) + codes[idx].astype(np.float64) * float(scale)
        assert np.allclose(out, want, rtol=2e-7, atol=0), (idx, out, want)
    # the FP16 and FP32 layouts of the same cells
    w = rng.uniform(0.1, 6.0, (5, 4)).astype(np.float32)
    for fmt, arr in ((0, w), (1, w.astype(np.float16))):
        for idx in range(5):
            L.lfh_load_cell(fmt, arr.ctypes.data, idx, out.ctypes.data)
            assert (out == arr[idx].astype(np.float32)).all()


def _bilinear_definition(img, x, y):
    """Clamp-to-edge bilinear of an (H, W, 3) FP64 image with texel (i, j)'s
    centre at (x, y) = (i, j), written out from the definition."""
    H, W = img.shape[:2]
    x = min(max(x, 0.0), W - 1.0)
    y = min(max(y, 0.0), H - 1.0)
    x0, y0 = int(np.floor(x)), int(np.floor(y))
    x1, y1 = min(x0 + 1, W - 1), min(y0 + 1, H - 1)
    fx, fy = x - x0, y - y0
    return ((1 - fx) * (1 - fy) * img[y0, x0] + fx * (1 - fy) * img[y0, x1] + (1 - fx) * fy * img[y1, x0]
            + fx * fy * img[y1, x1])


@pytest.mark.parametrize("fmt", [0, 1, 2])
@pytest.mark.parametrize("W,H", [(7, 5), (2, 2), (64, 3)])
def test_bilinear_taps_match_the_clamp_to_edge_definition(fmt, W, H):
    """The kernels' bilinear sample (the right-hand taps addressed at a fixed
    byte offset from their row's first tap) built for the host: RGBA8 (0..255),
    RGBA16F and RGBA32F images, positions inside, on and past every edge,
    against the definition in FP64; at whole texel positions the sample is the
    texel itself, exactly (a tap one texel off fails there)."""
    L = _lib()
    rng = np.random.default_rng(101 + 7 * fmt + W)
    if fmt == 0:
        buf = rng.integers(0, 256, (H, W, 4), dtype=np.uint8)
    elif fmt == 1:
        buf = rng.random((H, W, 4)).astype(np.float16)
    else:
        buf = rng.random((H, W, 4)).astype(np.float32)
    buf = np.ascontiguousarray(buf)
    ref = buf[..., :3].astype(np.float64)
    edge = lambda n: [-3.2, -1e-3, 0.0, 0.25, 0.5, n - 2.0, n - 1.5, n - 1.0 - 1e-3, n - 1.0, n - 0.9, n + 5.0]
    xs = np.float32(edge(W) + list(rng.uniform(-2.0, W + 1.0, 12)))
    ys = np.float32(edge(H) + list(rng.uniform(-2.0, H + 1.0, 12)))
    out = np.zeros(3, np.float32)
    tol = 1e-4 if fmt == 0 else 1e-6  # FP32 weights and sums of values up to 255 or 1
    for x in xs:
        for y in ys:
            assert L.lfh_bilinear(fmt, buf.ctypes.data, W, H, float(x), float(y), out.ctypes.data) == 0
            want = _bilinear_definition(ref, float(x), float(y))
            assert np.abs(out - want).max() <= tol, (fmt, W, H, x, y, out, want)
    for j in range(H):
        for i in range(W):
            assert L.lfh_bilinear(fmt, buf.ctypes.data, W, H, float(i), float(j), out.ctypes.data) == 0
            assert np.array_equal(out, ref[j, i].astype(np.float32)), (fmt, i, j)
    assert L.lfh_bilinear(3, buf.ctypes.data, W, H, 0.0, 0.0, out.ctypes.data) == 1
    assert L.lfh_bilinear(fmt, buf.ctypes.data, 1, H, 0.0, 0.0, out.ctypes.data) == 1
