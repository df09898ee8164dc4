"""Pins of the FP64 oracle's light field prefilter (Sec. 5.1, Eqs. (4)-(5)).

The prefilter sends, for every pixel of a real-time view i, rays from points
of view i's disk through the 3-D points of view i's mesh seen at points of the
pixel basis' support, asks the offline model for each ray's colour and forms
the rho-sigma-weighted ratio estimate. Pinned here against facts the paper and
the mathematics fix: the closed-form basis values, the identity for a point
aperture at the camera centre with a delta basis, exact reproduction of
constant colour, sharpness where the geometry is exact (the paper's reason
for the prefilter: it blurs only where geometries disagree), agreement of
the oracle's two mesh-intersection modes, and an independent pure-Python
evaluation on a tiny light field.
"""
import numpy as np
import pytest

import lfsynth
import oracle
from test_oracle_pins import _plane_views, _py_query


def test_basis_closed_forms():
    """Lanczos-2 is sinc(x) sinc(x/2) on |x| < 2; the box is 1 on |x| <= 1/2."""
    assert oracle.basis("lanczos2", 0.0) == 1.0
    for x in (1.0, -1.0, 2.0, -2.0, 2.5):
        assert abs(oracle.basis("lanczos2", x)) < 1e-15
    assert oracle.basis("lanczos2", 0.5) == pytest.approx(4 * np.sqrt(2) / np.pi ** 2, rel=1e-14)
    assert oracle.basis("lanczos2", 1.5) == pytest.approx(-4 * np.sqrt(2) / (9 * np.pi ** 2), rel=1e-14)
    assert oracle.basis("lanczos2", 0.3) == oracle.basis("lanczos2", -0.3)
    assert oracle.basis("box", 0.5) == 1.0 and oracle.basis("box", -0.5) == 1.0
    assert oracle.basis("box", 0.5000001) == 0.0


def test_point_aperture_delta_basis_is_identity(tiny):
    """One sample at the disk centre with a zero pixel offset: the ray leaves
    c_i through the pixel centre, meets mesh i at a point that projects back
    to that pixel centre, and with offline disks too small to reach any
    neighbour the offline query returns image i's texel exactly."""
    V = tiny.views
    W = V.img_res
    assert V.mesh_m == W
    lbar = oracle.OracleViews(V.centres, V.rot, V.rgba8, V.zdepth, V.src_fov_deg, 0.5 * lfsynth.min_nn(V.centres))
    target = oracle.OracleViews.from_views(V)
    yy, xx = np.divmod(np.arange(W * W), W)
    idx = np.nonzero((xx > 0) & (yy > 0) & (xx < W - 1) & (yy < W - 1))[0][::7]
    for i in (3, 40):
        r = oracle.prefilter(lbar, target, i, V.disk_radius, [[0.0, 0.0]], [[0.0, 0.0]], "box", idx)
        assert (r["wsum"] == 1.0).all()
        want = V.rgba8[i].reshape(-1, 4)[idx, :3] / 255.0
        assert np.abs(r["rgb"] - want).max() < 1e-12


def test_constant_colour_views_prefilter_to_the_colour(tiny):
    """Eq. (5) is a normalised weighting: constant-colour views give that
    colour wherever the denominator is non-zero, even with the negative lobes
    of Lanczos-2."""
    V = tiny.views
    col = np.array([37, 180, 222, 255], np.uint8)
    img = np.broadcast_to(col, V.rgba8.shape).copy()
    ov = oracle.OracleViews(V.centres, V.rot, img, V.zdepth, V.src_fov_deg, V.disk_radius)
    dp, po = lfsynth.prefilter_samples(7, 16, 2.0)
    idx = np.arange(0, V.img_res ** 2, 97)
    r = oracle.prefilter(ov, ov, 12, 2.0 * V.disk_radius, dp, po, "lanczos2", idx)
    ok = r["wsum"] != 0
    assert ok.mean() > 0.9
    assert np.abs(r["rgb"][ok] - col[:3] / 255.0).max() < 1e-12


def test_exact_geometry_keeps_the_prefilter_sharp():
    """Where the per-view geometry is exact (a plane), every ray of the
    aperture passes through the same scene point, so the offline query returns
    the same colour for every disk sample and the prefiltered pixel equals the
    view's own pixel up to the bilinear reconstruction error of the offline
    query (Fig. 'prefilter' (a) of the paper). Views of the plane x = 2 with a
    smooth texture of period 2 m."""
    sc, ov, c, R = _plane_views(1, period=2.0, img=64, mesh=64)
    dp, _ = lfsynth.prefilter_samples(5, 32, 2.0)
    po = np.zeros_like(dp)
    i = int(np.argmax(R[:, 0, 2]))  # the view looking most squarely at the plane
    W = 64
    yy, xx = np.divmod(np.arange(W * W), W)
    idx = np.nonzero((xx > 4) & (yy > 4) & (xx < W - 5) & (yy < W - 5))[0][::11]
    r = oracle.prefilter(ov, ov, i, 0.05, dp, po, "box", idx)
    assert (r["wsum"] > 0).all()
    want = ov.rgba8[i].reshape(-1, 4)[idx, :3] / 255.0
    # texture gradient <= 2 pi / period per metre at up to ~2.3 m over a 120-degree
    # 64-pixel view: under 0.03 per pixel, so bilinear and quantisation stay below 0.01
    assert np.abs(r["rgb"] - want).max() < 0.01


def test_wrong_geometry_blurs_the_prefilter():
    """Where the real-time mesh disagrees with the scene (here: the plane's
    mesh pulled to 0.3 of its depth), the aperture's rays spread over the
    scene and the prefilter blurs (Fig. 'prefilter' (b)). Measured against the
    same prefilter with a point aperture at the camera centre: on the checker
    texture a 0.1 m aperture moves the pixels over 3x further from it with the
    wrong mesh than with the exact one."""
    sc, ov, c, R = _plane_views(0, img=64, mesh=64)
    dp, _ = lfsynth.prefilter_samples(5, 32, 2.0)
    po = np.zeros_like(dp)
    i = int(np.argmax(R[:, 0, 2]))
    idx = np.arange(64 * 64)[::5]
    point = oracle.prefilter(ov, ov, i, 0.1, [[0.0, 0.0]], [[0.0, 0.0]], "box", idx)
    r = oracle.prefilter(ov, ov, i, 0.1, dp, po, "box", idx)
    wrong = oracle.OracleViews(ov.centres, ov.rot, ov.rgba8, ov.zdepth * np.float32(0.3), 120.0, ov.s.disk_radius)
    rw = oracle.prefilter(ov, wrong, i, 0.1, dp, po, "box", idx)
    ok = (r["wsum"] > 0) & (rw["wsum"] > 0) & (point["wsum"] > 0)
    assert ok.mean() > 0.9
    e_exact = np.abs(r["rgb"][ok] - point["rgb"][ok]).mean()
    e_wrong = np.abs(rw["rgb"][ok] - point["rgb"][ok]).mean()
    assert e_wrong > 3 * e_exact


def test_prefilter_traversal_matches_brute_force(tiny):
    V = tiny.views
    ov = oracle.OracleViews.from_views(V)
    dp, po = lfsynth.prefilter_samples(9, 4, 2.0)
    idx = np.array([130, 4000, 8257, 12000, 16000])
    a = oracle.prefilter(ov, ov, 21, V.disk_radius, dp, po, "lanczos2", idx)
    b = oracle.prefilter(ov.with_mode("brute"), ov.with_mode("brute"), 21, V.disk_radius, dp, po, "lanczos2", idx)
    assert np.abs(a["rgb"] - b["rgb"]).max() < 1e-12 and np.array_equal(a["wsum"], b["wsum"])


def _py_mesh_point(cent, rot, z, fov, i, X, Y):
    """Nearest point of view i's mesh along the ray from c_i through (X, Y, 1),
    by a linear solve against every triangle (None if missed)."""
    M = z.shape[1]
    ts = np.tan(np.radians(fov / 2))
    d = rot[i] @ np.array([X, Y, 1.0])
    vert = lambda j, k: cent[i] + z[i, k, j] * rot[i] @ np.array(
        [(2 * (j + .5) / M - 1) * ts, (1 - 2 * (k + .5) / M) * ts, 1.0])
    best = np.inf
    for k in range(M - 1):
        for j in range(M - 1):
            for tri in ((vert(j, k), vert(j + 1, k), vert(j + 1, k + 1)),
                        (vert(j, k), vert(j + 1, k + 1), vert(j, k + 1))):
                A = np.stack([-d, tri[1] - tri[0], tri[2] - tri[0]], 1)
                if abs(np.linalg.det(A)) < 1e-300:
                    continue
                t, b1, b2 = np.linalg.solve(A, cent[i] - tri[0])
                if b1 >= -1e-12 and b2 >= -1e-12 and b1 + b2 <= 1 + 1e-12 and 0 < t < best:
                    best = t
    return None if not np.isfinite(best) else cent[i] + best * d


def test_prefilter_python_brute_force_agrees_on_tiny_field():
    """Eq. (5) by plain Python loops on a 12-view field with random depth and
    colour: ray origins from the disk frame, mesh points and the offline query
    by linear solves over every triangle, Lanczos-2 from numpy's sinc."""
    rng = np.random.default_rng(5)
    c, R = lfsynth.rig(12, 0.35)
    M, Wi = 6, 9
    z = rng.uniform(0.8, 2.0, (12, M, M)).astype(np.float32)
    img = rng.integers(0, 256, (12, Wi, Wi, 4)).astype(np.uint8)
    R_d = 1.5 * lfsynth.mean_nn(c)
    ov = oracle.OracleViews(c, R, img, z, 120.0, R_d)
    dp, po = lfsynth.prefilter_samples(3, 6, 2.0)
    i, Rt = 4, 0.8 * R_d
    idx = np.array([10, 31, 40, 52, 70])
    got = oracle.prefilter(ov, ov, i, Rt, dp, po, "lanczos2", idx)
    ts = np.tan(np.radians(60))
    lz = lambda x: np.sinc(x) * np.sinc(x / 2) if abs(x) < 2 else 0.0
    for q, p in enumerate(idx):
        num, den = np.zeros(3), 0.0
        for (du, dv), (ds, dt) in zip(dp, po):
            rho = 1 - np.hypot(du, dv)
            w = rho * lz(ds) * lz(dt)
            s, t = p % Wi + 0.5 + ds, p // Wi + 0.5 + dt
            P = _py_mesh_point(c, R, z, 120.0, i, (2 * s / Wi - 1) * ts, (1 - 2 * t / Wi) * ts)
            if P is None or rho <= 0 or w == 0:
                continue
            o = c[i] + Rt * (du * R[i][:, 0] + dv * R[i][:, 1])
            col, wq = _py_query(c, R, img, z, 120.0, R_d, o, P - o)
            if wq <= 0:
                continue
            num += w * col
            den += w
        assert got["wsum"][q] == pytest.approx(den, abs=1e-9)
        assert np.allclose(got["rgb"][q], num / den if den != 0 else 0.0, atol=1e-9)


# ----------------------------------------------------------------------------- oval apertures (Sec. 4.4 disks)

_EXT = np.array([0.031, 0.017, 0.024, 0.041])  # e+u, e-u, e+v, e-v in metres, deliberately unequal


def test_oval_aperture_with_equal_extents_is_the_circle(tiny):
    """Four equal extents r make the oval the circle of radius r: the same ray
    origins and the same ratio; every weight carries the constant factor r^2."""
    V = tiny.views
    ov = oracle.OracleViews.from_views(V)
    dp, po = lfsynth.prefilter_samples(9, 8, 2.0)
    idx = np.arange(0, V.img_res ** 2, 211)
    r = 0.037
    a = oracle.prefilter(ov, ov, 17, r, dp, po, "lanczos2", idx)
    b = oracle.prefilter(ov, ov, 17, 1.0, dp, po, "lanczos2", idx, aperture_ext=[r, r, r, r])
    assert (a["wsum"] != 0).mean() > 0.9
    assert np.abs(a["rgb"] - b["rgb"]).max() < 1e-12
    assert np.allclose(b["wsum"], r * r * a["wsum"], rtol=1e-12, atol=0)


def test_oval_aperture_maps_unit_disk_points_by_quadrant(tiny):
    """A one-sample prefilter returns the offline query of its single ray. The
    oval sends a unit-disk point (du, dv) to du e_u along r and dv e_v along u,
    with e_u = e+u for du >= 0 else e-u (e_v likewise): the same ray as a
    circle aperture of any radius Rc with the point (du e_u, dv e_v) / Rc."""
    V = tiny.views
    ov = oracle.OracleViews.from_views(V)
    idx = np.arange(0, V.img_res ** 2, 173)
    eu = lambda du: _EXT[0] if du >= 0 else _EXT[1]
    ev = lambda dv: _EXT[2] if dv >= 0 else _EXT[3]
    n_checked = 0
    for du, dv in ((0.6, 0.0), (-0.6, 0.0), (0.0, 0.5), (0.0, -0.5), (0.4, -0.5), (-0.3, 0.7)):
        oval = oracle.prefilter(ov, ov, 30, 1.0, [[du, dv]], [[0.2, -0.1]], "box", idx, aperture_ext=_EXT)
        Rc = 0.1
        circ = oracle.prefilter(ov, ov, 30, Rc, [[du * eu(du) / Rc, dv * ev(dv) / Rc]], [[0.2, -0.1]], "box", idx)
        ok = oval["wsum"] != 0
        assert np.array_equal(ok, circ["wsum"] != 0)
        assert np.abs(oval["rgb"] - circ["rgb"]).max() < 1e-12
        n_checked += ok.sum()
    assert n_checked > 6 * 0.8 * len(idx)


def test_oval_aperture_weights_quadrants_by_their_area(tiny):
    """Eq. (4) integrates over the disk's area; a uniform point of the unit
    disk lands in an oval quadrant with density 1 / (e_u e_v), so the weight of
    a sample is rho sigma e_u e_v. Two samples in quadrants of different area:
    the two-sample estimate is the mean of the one-sample results weighted so,
    by hand."""
    V = tiny.views
    ov = oracle.OracleViews.from_views(V)
    idx = np.arange(0, V.img_res ** 2, 97)
    pts = np.array([[0.5, 0.3], [-0.2, -0.6]])
    offs = np.array([[0.1, 0.3], [-0.4, 0.2]])
    one = [oracle.prefilter(ov, ov, 44, 1.0, pts[j:j + 1], offs[j:j + 1], "lanczos2", idx, aperture_ext=_EXT)
           for j in range(2)]
    both = oracle.prefilter(ov, ov, 44, 1.0, pts, offs, "lanczos2", idx, aperture_ext=_EXT)
    area = np.array([_EXT[0] * _EXT[2], _EXT[1] * _EXT[3]])
    rho = 1 - np.hypot(pts[:, 0], pts[:, 1])
    sig = np.array([oracle.basis("lanczos2", a) * oracle.basis("lanczos2", b) for a, b in offs])
    w = rho * sig * area
    ok = (one[0]["wsum"] != 0) & (one[1]["wsum"] != 0)
    assert ok.mean() > 0.8
    want = (w[0] * one[0]["rgb"][ok] + w[1] * one[1]["rgb"][ok]) / w.sum()
    assert np.abs(both["rgb"][ok] - want).max() < 1e-12
    assert np.allclose(both["wsum"][ok], w.sum(), rtol=1e-12, atol=0)
    # without the area factor the estimate differs where the two rays disagree
    plain = (rho[0] * sig[0] * one[0]["rgb"][ok] + rho[1] * sig[1] * one[1]["rgb"][ok]) / (rho * sig).sum()
    assert np.abs(plain - want).max() > 1e-3


def test_oval_prefilter_python_brute_force_agrees_on_tiny_field():
    """Eq. (5) with an oval aperture by plain Python loops on a 12-view field:
    the unit-disk point mapped by its quadrant's extents, weights with the
    quadrant's area factor, mesh points and the offline query by linear
    solves over every triangle."""
    rng = np.random.default_rng(8)
    c, R = lfsynth.rig(12, 0.35)
    M, Wi = 6, 9
    z = rng.uniform(0.8, 2.0, (12, M, M)).astype(np.float32)
    img = rng.integers(0, 256, (12, Wi, Wi, 4)).astype(np.uint8)
    R_d = 1.5 * lfsynth.mean_nn(c)
    ov = oracle.OracleViews(c, R, img, z, 120.0, R_d)
    dp, po = lfsynth.prefilter_samples(4, 8, 2.0)
    i = 7
    ext = np.array([0.9, 0.5, 0.7, 1.2]) * R_d
    idx = np.array([11, 30, 40, 49, 62])
    got = oracle.prefilter(ov, ov, i, 1.0, dp, po, "lanczos2", idx, aperture_ext=ext)
    ts = np.tan(np.radians(60))
    lz = lambda x: np.sinc(x) * np.sinc(x / 2) if abs(x) < 2 else 0.0
    for q, p in enumerate(idx):
        num, den = np.zeros(3), 0.0
        for (du, dv), (ds, dt) in zip(dp, po):
            eu = ext[0] if du >= 0 else ext[1]
            ev = ext[2] if dv >= 0 else ext[3]
            rho = 1 - np.hypot(du, dv)
            w = rho * lz(ds) * lz(dt) * eu * ev
            s, t = p % Wi + 0.5 + ds, p // Wi + 0.5 + dt
            P = _py_mesh_point(c, R, z, 120.0, i, (2 * s / Wi - 1) * ts, (1 - 2 * t / Wi) * ts)
            if P is None or rho <= 0 or w == 0:
                continue
            o = c[i] + du * eu * R[i][:, 0] + dv * ev * R[i][:, 1]
            col, wq = _py_query(c, R, img, z, 120.0, R_d, o, P - o)
            if wq <= 0:
                continue
            num += w * col
            den += w
        assert got["wsum"][q] == pytest.approx(den, abs=1e-12)
        assert np.allclose(got["rgb"][q], num / den if den != 0 else 0.0, atol=1e-9)
