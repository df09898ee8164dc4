"""Pins of the FP64 oracle against what the paper and plain geometry fix.

Each test names the paper passage (Sec. 4 of the paper) it holds the oracle to.
None of these re-types the oracle's formulas: they use constructed geometry
with known answers, special cases that reduce to exact results, invariances,
and an independent brute-force evaluation on a tiny light field.
"""
import numpy as np
import pytest

import lfsynth
import oracle


def _frame_looking(f, up=(0.0, 0.0, 1.0)):
    """Columns (r, u, f) with the rig's handedness: r = f x up, u = r x f."""
    f = np.asarray(f, float) / np.linalg.norm(f)
    r = np.cross(f, up)
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    return np.stack([r, u, f], 1)


# ----------------------------------------------------------------------------- Eq. (1): eye rays

def test_eye_ray_axes_and_fov():
    R = _frame_looking([0.3, -0.5, 0.2])
    pos = np.array([0.01, 0.02, -0.03])
    W, H, hfov = 200, 100, 90.0
    o, e = oracle.eye_rays(pos, R, hfov, W, H, [[W / 2, H / 2], [W, H / 2], [W / 2, 0.0], [0.0, H]])
    assert np.allclose(o, pos)
    en = e / np.linalg.norm(e, axis=1, keepdims=True)
    # centre ray along the optical axis
    assert np.allclose(en[0], R[:, 2], atol=1e-15)
    # right edge: half the horizontal FOV, towards +r, no up component
    assert np.degrees(np.arccos(en[1] @ R[:, 2])) == pytest.approx(45.0, abs=1e-12)
    assert en[1] @ R[:, 0] > 0 and abs(en[1] @ R[:, 1]) < 1e-15
    # top edge (row 0 is the top): vertical half-angle from the aspect ratio, towards +u
    assert np.degrees(np.arccos(en[2] @ R[:, 2])) == pytest.approx(np.degrees(np.arctan(0.5)), abs=1e-12)
    assert en[2] @ R[:, 1] > 0 and abs(en[2] @ R[:, 0]) < 1e-15
    # bottom-left corner: -r, -u
    assert en[3] @ R[:, 0] < 0 and en[3] @ R[:, 1] < 0


# ----------------------------------------------------------------------------- Sec. 4.1: disk kernel

def test_disk_unit_cases(tiny, tiny_oracle):
    V, ov = tiny.views, tiny_oracle
    R_d = V.disk_radius
    o = np.array([0.01, -0.02, 0.03])
    for i in (0, 17, 40, 63):
        c, Ri = V.centres[i], V.rot[i]
        r_ax, u_ax = Ri[:, 0], Ri[:, 1]
        # through the disk centre: rho = 1, (u, v) = 0
        a, u, v, rho = oracle.disk(ov, i, o, c - o)
        assert a > 0 and abs(u) < 1e-14 and abs(v) < 1e-14 and rho == pytest.approx(1.0, abs=1e-14)
        # offset s along a known direction: (u, v) = s (cos t, sin t), rho = 1 - s / R
        for s_frac, th in ((0.3, 0.0), (0.7, 1.1), (0.95, -2.5)):
            s = s_frac * R_d
            target = c + s * (np.cos(th) * r_ax + np.sin(th) * u_ax)
            a, u, v, rho = oracle.disk(ov, i, o, 2.5 * (target - o))
            assert u == pytest.approx(s * np.cos(th), abs=1e-14)
            assert v == pytest.approx(s * np.sin(th), abs=1e-14)
            assert rho == pytest.approx(1 - s_frac, abs=1e-13)
        # just outside / inside the rim
        out_pt = c + R_d * (1 + 1e-9) * r_ax
        in_pt = c + R_d * (1 - 1e-6) * u_ax
        rec_out = oracle.records(ov, o, out_pt - o)[i]
        rec_in = oracle.records(ov, o, in_pt - o)[i]
        assert rec_out["cand"] == 0 and rec_out["rho"] < 0
        assert rec_in["cand"] == 1 and rec_in["rho"] == pytest.approx(1e-6, rel=1e-6)
        # back-facing disk: never a candidate, no disk coordinates
        rec_back = oracle.records(ov, o, -(c - o))[i]
        assert rec_back["cand"] == 0 and rec_back["a"] < 0
        assert np.isnan(oracle.disk(ov, i, o, -(c - o))[3])
        # decision band: a ray 1e-7 R inside the rim is listed as ill-conditioned,
        # one well inside is not
        rim = c + R_d * (1 - 1e-7) * r_ax
        mid = c + 0.3 * R_d * u_ax
        lists = oracle.render_rays(ov, np.stack([o, o]), np.stack([rim - o, mid - o]), cap=16)
        assert i in lists["cand_band"][0] and i in lists["cand"][0]
        assert i not in lists["cand_band"][1] and i in lists["cand"][1]


# ----------------------------------------------------------------------------- sampling

def _linear_image_views(W=32, H=24):
    y, x = np.mgrid[0:H, 0:W]
    img = np.zeros((1, H, W, 4), np.uint8)
    img[0, :, :, 0] = 10 + 2 * x + 3 * y
    img[0, :, :, 1] = 200 - 3 * x
    img[0, :, :, 2] = 7 + y
    img[0, :, :, 3] = 255
    z = np.ones((1, 4, 4), np.float32)
    R = _frame_looking([1.0, 0.0, 0.0])
    return oracle.OracleViews(np.array([[0.35, 0, 0]]), R[None], img, z, 120.0, 0.1)


def _lin(px, py):
    return np.array([10 + 2 * px + 3 * py, 200 - 3 * px, 7 + py]) / 255.0


def test_bilinear_exact_on_affine_image_and_clamps():
    ov = _linear_image_views()
    W, H, ts = 32, 24, np.tan(np.radians(60))

    def to_X(px, py):  # continuous texel coordinate -> normalised image plane
        return ((px + 0.5) * 2 / W - 1) * ts, (1 - (py + 0.5) * 2 / H) * ts

    rng = np.random.default_rng(5)
    for px, py in [(0, 0), (31, 23), (4, 7)] + [tuple(p) for p in rng.uniform([0, 0], [31, 23], (50, 2))]:
        got = oracle.sample(ov, 0, *to_X(px, py))
        assert np.allclose(got, _lin(px, py), atol=1e-12, rtol=0)
    # clamp-to-edge outside the texel-centre range
    assert np.allclose(oracle.sample(ov, 0, *to_X(-0.4, 5.0)), _lin(0, 5.0), atol=1e-12)
    assert np.allclose(oracle.sample(ov, 0, *to_X(31.3, 22.6)), _lin(31, 22.6), atol=1e-12)
    assert np.allclose(oracle.sample(ov, 0, *to_X(3.25, -3.0)), _lin(3.25, 0), atol=1e-12)


# ----------------------------------------------------------------------------- Eq. (2)/(3): normalisation

def test_constant_colour_views_reproduce_colour(tiny):
    """Eq. (3): with every image constant c the query returns c wherever any
    view contributes (the blend is a normalised convex combination)."""
    V = tiny.views
    col = np.array([37, 150, 222], np.uint8)
    img = np.empty_like(V.rgba8)
    img[..., :3] = col
    img[..., 3] = 255
    ov = oracle.OracleViews(V.centres, V.rot, img, V.zdepth, V.src_fov_deg, V.disk_radius)
    r = oracle.render(ov, tiny.head_pos[0], tiny.head_rot[0], tiny.hfov_deg, 64, 64)
    cov = r["wsum"] > 0
    assert cov.all()
    assert np.abs(r["rgb"][cov] - col / 255.0).max() < 1e-12


def test_weights_and_records_consistent(tiny, tiny_oracle, rng):
    """Sec. 4.2: numerator and denominator gather exactly the views whose
    disk covers the ray and whose mesh is hit; W > 0 iff some view contributes."""
    ov = tiny_oracle
    pxy = rng.uniform(0, 256, (40, 2))
    o, e = oracle.eye_rays(tiny.head_pos[0], tiny.head_rot[0], tiny.hfov_deg, 256, 256, pxy)
    r = oracle.render_rays(ov, o, e, cap=16)
    for k in range(len(pxy)):
        rec = oracle.records(ov, o[k], e[k])
        use = (rec["cand"] == 1) & (rec["hit"] == 1)
        assert (r["wsum"][k] > 0) == (r["count"][k] > 0) == use.any()
        assert r["count"][k] == use.sum()
        assert r["wsum"][k] == pytest.approx(rec["rho"][use].sum(), abs=1e-14)
        assert (rec["rho"][use] > 0).all() and (rec["rho"][use] <= 1).all()
        want = (rec["rho"][use, None] * rec["rgb"][use]).sum(0) / rec["rho"][use].sum()
        assert np.allclose(r["rgb"][k], want, atol=1e-14)
        assert list(r["cand"][k][r["cand"][k] >= 0]) == list(np.nonzero(rec["cand"])[0])
        assert list(r["contrib"][k][r["contrib"][k] >= 0]) == list(np.nonzero(use)[0])


# ----------------------------------------------------------------------------- camera-centre reproduction

def test_camera_centre_reproduces_source_image(tiny):
    """An eye placed at view k's centre with view k's frame, FOV and resolution,
    and disks too small to reach any neighbour, must return image k itself at
    every pixel: each pixel ray meets mesh k at a point that projects back to
    the same pixel centre (pins ray, axis, pixel-centre and projection
    conventions against the generator's independent camera)."""
    V = tiny.views
    R_small = 0.5 * lfsynth.min_nn(V.centres)
    ov = oracle.OracleViews(V.centres, V.rot, V.rgba8, V.zdepth, V.src_fov_deg, R_small)
    W = V.img_res
    assert V.mesh_m == W
    for k in (5, 33):
        r = oracle.render(ov, V.centres[k], V.rot[k], V.src_fov_deg, W, W, cap=4)
        assert (r["cand"][:, 0] == k).all() and (r["cand"][:, 1] == -1).all()
        want = V.rgba8[k, :, :, :3].reshape(-1, 3) / 255.0
        # pixel-centre rays pass exactly through mesh vertices; on the outer ring
        # those vertices lie on the mesh's domain edge, where hit/miss is decided
        # by rounding, so the ring may be empty but is never wrong
        yy, xx = np.divmod(np.arange(W * W), W)
        inner = (xx > 0) & (yy > 0) & (xx < W - 1) & (yy < W - 1)
        assert (r["count"][inner] == 1).all()
        hit = r["count"] == 1
        assert (r["count"][~inner] <= 1).all() and hit[~inner].mean() > 0.5
        assert np.abs(r["rgb"][hit] - want[hit]).max() < 1e-12
        # hits on the outer ring sit on the mesh domain edge: listed as ill-conditioned
        edge = r["contrib_band"][:, 0]
        assert (edge[inner] == -1).all()
        assert (edge[~inner & hit] == k).all()


# ----------------------------------------------------------------------------- planar scene

def _plane_views(texture, period=2.0, rgb=(0.2, 0.5, 0.8), img=128, mesh=64):
    # views whose whole 120-degree frustum meets the plane x = 2
    c, R = lfsynth.rig(1024)
    keep = R[:, 0, 2] > np.cos(np.radians(16))          # f . x_hat
    c, R = c[keep], R[keep]
    sc = lfsynth.scene_plane([1.0, 0.0, 0.0], 2.0, texture, period, rgb)
    rgba, z, esc = lfsynth.render_views(sc, c, R, 120.0, img, mesh)
    assert esc == 0
    return sc, oracle.OracleViews(c, R, rgba, z, 120.0, 1.5 * lfsynth.mean_nn(lfsynth.rig(1024)[0])), c, R


def test_planar_scene_hits_are_exact():
    """Sec. 4.5: the depth-map mesh of a plane is the plane itself, so every
    view's nearest hit is the analytic ray/plane point and its reprojection is
    that point's projection."""
    sc, ov, c, R = _plane_views(2)
    eye_R = _frame_looking([1.0, 0.02, -0.01])
    pos = np.array([0.05, -0.03, 0.02])
    rng = np.random.default_rng(0)
    pxy = rng.uniform(0, 48, (60, 2))
    o, e = oracle.eye_rays(pos, eye_R, 30.0, 48, 48, pxy)
    n_checked = 0
    for k in range(len(pxy)):
        t_plane = (2.0 - o[k, 0]) / e[k, 0]
        P = o[k] + t_plane * e[k]
        rec = oracle.records(ov, o[k], e[k])
        use = (rec["cand"] == 1) & (rec["hit"] == 1)
        assert use.any()
        for i in np.nonzero(use)[0]:
            # depth maps are stored as float32, so mesh vertices sit on the plane
            # only to 2^-24 relative; allow 16x that (slanted triangles)
            assert rec["t_hit"][i] == pytest.approx(t_plane, rel=1e-6)
            Pl = R[i].T @ (P - c[i])
            assert rec["Xs"][i] == pytest.approx(Pl[0] / Pl[2], abs=1e-6)
            assert rec["Ys"][i] == pytest.approx(Pl[1] / Pl[2], abs=1e-6)
            n_checked += 1
    assert n_checked > 100


def test_planar_scene_constant_and_smooth_texture():
    """A constant plane is reproduced exactly; a smooth texture f is reproduced
    to within quantisation plus the bilinear bound (1/8)(|g_xx| + |g_yy|) of
    the image function g, evaluated numerically around each sample."""
    eye_R = _frame_looking([1.0, -0.03, 0.02])
    pos = np.array([-0.02, 0.02, 0.01])
    sc, ov, c, R = _plane_views(2)
    r = oracle.render(ov, pos, eye_R, 20.0, 32, 32)
    want = np.round(np.array([0.2, 0.5, 0.8]) * 255) / 255
    assert (r["wsum"] > 0).all() and np.abs(r["rgb"] - want).max() < 1e-12

    sc, ov, c, R = _plane_views(1, period=2.0)
    W = H = 24
    idx = np.arange(W * H)
    r = oracle.render(ov, pos, eye_R, 20.0, W, H, idx)
    assert (r["wsum"] > 0).all()
    o, e = oracle.eye_rays(pos, eye_R, 20.0, W, H, oracle.pixel_centres(W, H, idx))
    ts, Ws = np.tan(np.radians(60)), 128

    def g(i, px, py):  # image-i function at continuous texel coordinate
        X = ((px + 0.5) * 2 / Ws - 1) * ts
        Y = (1 - (py + 0.5) * 2 / Ws) * ts
        d = R[i] @ np.array([X, Y, 1.0])
        t = (2.0 - c[i][0]) / d[0]
        return lfsynth.texture(sc, 200, c[i] + t * d)

    worst = 0.0
    for k in idx:
        rec = oracle.records(ov, o[k], e[k])
        use = np.nonzero((rec["cand"] == 1) & (rec["hit"] == 1))[0]
        P = o[k] + (2.0 - o[k, 0]) / e[k, 0] * e[k]
        f_true = lfsynth.texture(sc, 200, P)
        bound = 0.0
        for i in use:
            px = (rec["Xs"][i] / ts + 1) * 0.5 * Ws - 0.5
            py = (1 - rec["Ys"][i] / ts) * 0.5 * Ws - 0.5
            x0, y0 = np.floor(px), np.floor(py)
            gxx = gyy = 0.0
            for sx in np.linspace(0, 1, 3):
                for sy in np.linspace(0, 1, 3):
                    xx, yy, h = x0 + sx, y0 + sy, 0.25
                    gxx = max(gxx, np.abs(g(i, xx + h, yy) - 2 * g(i, xx, yy) + g(i, xx - h, yy)).max() / h**2)
                    gyy = max(gyy, np.abs(g(i, xx, yy + h) - 2 * g(i, xx, yy) + g(i, xx, yy - h)).max() / h**2)
            bound = max(bound, 1.25 * (gxx + gyy) / 8)
        err = np.abs(r["rgb"][k] - f_true).max()
        assert err <= 0.5 / 255 + bound + 1e-12
        worst = max(worst, err)
    assert worst > 0  # the smooth texture is not trivially reproduced


# ----------------------------------------------------------------------------- traversal vs brute force

def test_traversal_matches_brute_force(tiny, tiny_oracle, rng):
    """The grid walk visits every triangle that can be hit: its nearest hit
    equals the all-triangle minimum on a crop plus random rays."""
    ov_t = tiny_oracle
    ov_b = tiny_oracle.with_mode("brute")
    crop = np.array([(x + 0.5, y + 0.5) for y in range(100, 112) for x in range(60, 72)])
    pxy = np.concatenate([crop, rng.uniform(0, 256, (300, 2))])
    o, e = oracle.eye_rays(tiny.head_pos[0], tiny.head_rot[0], tiny.hfov_deg, 256, 256, pxy)
    rt = oracle.render_rays(ov_t, o, e, cap=16)
    rb = oracle.render_rays(ov_b, o, e, cap=16)
    assert (rt["contrib"] == rb["contrib"]).all()
    assert np.array_equal(rt["rgb"], rb["rgb"]) and np.array_equal(rt["wsum"], rb["wsum"])
    for k in range(0, len(pxy), 17):
        a = oracle.records(ov_t, o[k], e[k])
        b = oracle.records(ov_b, o[k], e[k])
        assert np.array_equal(a["hit"], b["hit"])
        h = a["hit"] == 1
        assert np.allclose(a["t_hit"][h], b["t_hit"][h], rtol=1e-12, atol=0)


# ----------------------------------------------------------------------------- invariances

def test_view_permutation_invariance(tiny, tiny_oracle):
    V = tiny.views
    perm = np.random.default_rng(7).permutation(V.n)
    ovp = oracle.OracleViews(V.centres[perm], V.rot[perm], V.rgba8[perm], V.zdepth[perm],
                             V.src_fov_deg, V.disk_radius)
    idx = np.arange(0, 256 * 256, 97)
    a = oracle.render(tiny_oracle, tiny.head_pos[0], tiny.head_rot[0], tiny.hfov_deg, 256, 256, idx)
    b = oracle.render(ovp, tiny.head_pos[0], tiny.head_rot[0], tiny.hfov_deg, 256, 256, idx)
    assert np.abs(a["rgb"] - b["rgb"]).max() < 1e-12
    assert np.abs(a["wsum"] - b["wsum"]).max() < 1e-12


def test_rigid_motion_invariance(tiny, tiny_oracle):
    """Moving rig, views and eye by one rigid motion leaves the image unchanged
    (depth maps and images are view-local)."""
    V = tiny.views
    q = np.random.default_rng(3).normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    Q = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                  [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                  [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
    tvec = np.array([1.7, -0.4, 3.1])
    ovm = oracle.OracleViews(V.centres @ Q.T + tvec, np.einsum("ij,njk->nik", Q, V.rot), V.rgba8, V.zdepth,
                             V.src_fov_deg, V.disk_radius)
    idx = np.arange(0, 256 * 256, 101)
    a = oracle.render(tiny_oracle, tiny.head_pos[0], tiny.head_rot[0], tiny.hfov_deg, 256, 256, idx)
    b = oracle.render(ovm, Q @ tiny.head_pos[0] + tvec, Q @ tiny.head_rot[0], tiny.hfov_deg, 256, 256, idx)
    assert np.abs(a["rgb"] - b["rgb"]).max() < 1e-9


# ----------------------------------------------------------------------------- independent brute force

def _py_query(cent, rot, img, z, fov, R_d, o, e):
    """Eq. (2) by plain loops: every triangle of every view, intersection by a
    3x3 linear solve (not Moller-Trumbore), projection and bilinear by hand."""
    n, H, W, _ = img.shape
    M = z.shape[1]
    ts = np.tan(np.radians(fov / 2))
    num, den = np.zeros(3), 0.0
    for i in range(n):
        f, ra, ua = rot[i][:, 2], rot[i][:, 0], rot[i][:, 1]
        if e @ f <= 0:
            continue
        t_disk = ((cent[i] - o) @ f) / (e @ f)
        q = o + t_disk * e - cent[i]
        rho = 1 - np.hypot(q @ ra, q @ ua) / R_d
        if rho <= 0:
            continue
        vert = lambda j, k: cent[i] + z[i, k, j] * rot[i] @ np.array(
            [(2 * (j + .5) / M - 1) * ts, (1 - 2 * (k + .5) / M) * ts, 1.0])
        best = np.inf
        for k in range(M - 1):
            for j in range(M - 1):
                for tri in ((vert(j, k), vert(j + 1, k), vert(j + 1, k + 1)),
                            (vert(j, k), vert(j + 1, k + 1), vert(j, k + 1))):
                    A = np.stack([-e, tri[1] - tri[0], tri[2] - tri[0]], 1)
                    if abs(np.linalg.det(A)) < 1e-300:
                        continue
                    t, b1, b2 = np.linalg.solve(A, o - tri[0])
                    if b1 >= -1e-12 and b2 >= -1e-12 and b1 + b2 <= 1 + 1e-12 and 0 < t < best:
                        best = t
        if not np.isfinite(best):
            continue
        Pl = rot[i].T @ (o + best * e - cent[i])
        px = (Pl[0] / Pl[2] / ts + 1) * W / 2 - .5
        py = (1 - Pl[1] / Pl[2] / ts) * H / 2 - .5
        x0, y0 = int(np.floor(px)), int(np.floor(py))
        fx, fy = px - x0, py - y0
        cl = lambda v, hi: min(max(v, 0), hi - 1)
        tex = lambda xx, yy: img[i, cl(yy, H), cl(xx, W), :3].astype(float) / 255
        col = ((1 - fx) * (1 - fy) * tex(x0, y0) + fx * (1 - fy) * tex(x0 + 1, y0)
               + (1 - fx) * fy * tex(x0, y0 + 1) + fx * fy * tex(x0 + 1, y0 + 1))
        num += rho * col
        den += rho
    return (num / den if den > 0 else np.zeros(3)), den


def test_brute_force_python_agrees_on_tiny_field():
    rng = np.random.default_rng(11)
    c, R = lfsynth.rig(12, 0.35)
    M, Wi = 7, 10
    z = rng.uniform(0.6, 2.5, (12, M, M)).astype(np.float32)
    img = rng.integers(0, 256, (12, Wi, Wi, 4)).astype(np.uint8)
    R_d = 1.5 * lfsynth.mean_nn(c)
    ov = oracle.OracleViews(c, R, img, z, 120.0, R_d)
    o = rng.normal(size=(25, 3)) * 0.05
    e = rng.normal(size=(25, 3))
    r = oracle.render_rays(ov, o, e)
    covered = 0
    for k in range(25):
        col, den = _py_query(c, R, img, z, 120.0, R_d, o[k], e[k])
        assert r["wsum"][k] == pytest.approx(den, abs=1e-9)
        assert np.allclose(r["rgb"][k], col, atol=1e-9)
        covered += den > 0
    assert covered >= 10


# ----------------------------------------------------------------------------- offline reference

def test_reference_render_reduces_to_plain_query(tiny, tiny_oracle):
    idx = np.arange(0, 256 * 256, 331)
    a = oracle.render(tiny_oracle, tiny.head_pos[0], tiny.head_rot[0], tiny.hfov_deg, 256, 256, idx)
    b = oracle.render_reference(tiny_oracle, tiny.head_pos[0], tiny.head_rot[0], tiny.hfov_deg, 256, 256, idx,
                                ss=1, disk_scale=1.0)
    assert np.array_equal(a["rgb"], b)


def _bilinear_by_hand(img, px, py):
    """Bilinear sample of an RGBA8 image at texel coordinates (px, py):
    texel centres at integers here, clamp-to-edge, RGB / 255."""
    H, W = img.shape[:2]
    x0, y0 = np.floor(px).astype(int), np.floor(py).astype(int)
    fx, fy = (px - x0)[:, None], (py - y0)[:, None]
    cx = lambda x: np.clip(x, 0, W - 1)
    cy = lambda y: np.clip(y, 0, H - 1)
    t = lambda x, y: img[cy(y), cx(x), :3].astype(np.float64) / 255.0
    return ((1 - fx) * (1 - fy) * t(x0, y0) + fx * (1 - fy) * t(x0 + 1, y0)
            + (1 - fx) * fy * t(x0, y0 + 1) + fx * fy * t(x0 + 1, y0 + 1))


def _reference_camera_centre_ok(tiny, ref_fn, k=21, ss=4):
    """Offline reference (Sec. 5.1's L-bar analogue) at a source camera: the
    eye at view k's centre with its frame, FOV and resolution, and disks that
    isolate view k even when doubled. Every sub-pixel ray then meets mesh k at
    a point that projects back to its own image position, so pixel (x, y) is
    the mean of the ss x ss bilinear samples of image k at texel coordinates
    (x + (s + 1/2)/ss - 1/2, y + (t + 1/2)/ss - 1/2), a sub-ray outside the
    mesh domain (the square of depth-pixel centres, [1/2, W - 1/2] in pixel
    units here) counting as 0. Expected values by hand in numpy. ss is even
    so that no sub-ray lies on the domain edge, where hit or miss is decided
    by rounding."""
    V = tiny.views
    W = V.img_res
    assert V.mesh_m == W
    ov = oracle.OracleViews(V.centres, V.rot, V.rgba8, V.zdepth, V.src_fov_deg, 0.2 * lfsynth.min_nn(V.centres))
    idx = np.concatenate([np.arange(0, W), np.arange(W, W * W, 37)])  # the top row (domain edge) + a spread
    got = ref_fn(ov, V.centres[k], V.rot[k], V.src_fov_deg, W, W, idx, ss=ss, disk_scale=2.0)
    x, y = (idx % W).astype(np.float64), (idx // W).astype(np.float64)
    acc = np.zeros((len(idx), 3))
    for t in range(ss):
        for s_ in range(ss):
            qx, qy = x + (s_ + 0.5) / ss, y + (t + 0.5) / ss  # continuous pixel position of the sub-ray
            inside = ((qx > 0.5) & (qx < W - 0.5) & (qy > 0.5) & (qy < W - 0.5))[:, None]
            acc += np.where(inside, _bilinear_by_hand(V.rgba8[k], qx - 0.5, qy - 0.5), 0.0)
    return np.abs(got - acc / (ss * ss)).max() < 1e-12


def _reference_by_records(tiny, ref_fn, ext_scale=None, ss=2, disk_scale=2.0):
    """The reference rebuilt from per-view ray records: sub-pixel positions
    (x + (s + 1/2)/ss, y + (t + 1/2)/ss) by hand, their rays (Eq. (1)), every
    facing view's mesh hit and sample from a field with a disk radius large
    enough to make every facing view a candidate, and the scaled falloff
    rho = 1 - r / (disk_scale R) (or the oval's normalised radius with the
    extents times disk_scale) by hand; each sub-ray is Eq. (2) over the views
    with rho > 0 and a hit (0 if none), the pixel their mean."""
    V = tiny.views
    R_d = V.disk_radius
    ext = None if ext_scale is None else oracle.disk_extents(V.centres, V.rot)[0] * ext_scale
    ov = oracle.OracleViews.from_views(V, disk_ext=ext)
    W = H = 96
    hfov, pos, rot = tiny.hfov_deg, tiny.head_pos[0], tiny.head_rot[0]
    idx = np.random.default_rng(3).integers(0, W * H, 24)
    got = ref_fn(ov, pos, rot, hfov, W, H, idx, ss=ss, disk_scale=disk_scale)
    wide = oracle.OracleViews.from_views(V, disk_radius=100.0)
    want = np.zeros((len(idx), 3))
    n_multi = 0
    for q, p in enumerate(idx):
        for t in range(ss):
            for s_ in range(ss):
                pxy = np.array([[p % W + (s_ + 0.5) / ss, p // W + (t + 0.5) / ss]])
                o, e = oracle.eye_rays(pos, rot, hfov, W, H, pxy)
                rec = oracle.records(wide, o[0], e[0])
                if ext is None:
                    rho = 1.0 - np.hypot(rec["u"], rec["v"]) / (disk_scale * R_d)
                else:
                    eu = np.where(rec["u"] >= 0, ext[:, 0], ext[:, 1]) * disk_scale
                    ev = np.where(rec["v"] >= 0, ext[:, 2], ext[:, 3]) * disk_scale
                    rho = 1.0 - np.hypot(rec["u"] / eu, rec["v"] / ev)
                use = (rec["a"] > 0) & (rho > 0) & (rec["hit"] == 1)
                n_multi += use.sum() >= 2
                if use.any():
                    want[q] += (rho[use, None] * rec["rgb"][use]).sum(0) / rho[use].sum()
    want /= ss * ss
    assert n_multi > len(idx)  # most sub-rays blend several views: the falloff's scale matters
    return np.abs(got - want).max() < 1e-10


def _ref_offsets_without_half(ov, pos, rot, hfov, W, H, idx, ss=4, disk_scale=2.0):
    """A planted mistake: sub-pixel rays at s / ss instead of (s + 1/2) / ss."""
    idx = np.asarray(idx, np.int64)
    base = np.stack([(idx % W).astype(np.float64), (idx // W).astype(np.float64)], 1)
    offs = np.arange(ss) / ss
    sub = np.stack(np.meshgrid(offs, offs, indexing="xy"), -1).reshape(-1, 2)
    o, e = oracle.eye_rays(pos, rot, hfov, W, H, (base[:, None, :] + sub[None, :, :]).reshape(-1, 2))
    big = ov.with_disk_radius(ov.s.disk_radius * disk_scale)
    if ov.disk_ext is not None:
        big = big.with_disk_extents(ov.disk_ext * disk_scale)
    return oracle.render_rays(big, o, e)["rgb"].reshape(len(idx), ss * ss, 3).mean(1)


def _ref_unscaled_disks(ov, pos, rot, hfov, W, H, idx, ss=4, disk_scale=2.0):
    """A planted mistake: the disks keep their real-time size."""
    return oracle.render_reference(ov, pos, rot, hfov, W, H, idx, ss=ss, disk_scale=1.0)


def test_reference_render_at_camera_centre_is_subpixel_box_filter(tiny):
    assert _reference_camera_centre_ok(tiny, oracle.render_reference)
    assert _reference_camera_centre_ok(tiny, oracle.render_reference, ss=2)
    assert not _reference_camera_centre_ok(tiny, _ref_offsets_without_half)


def test_reference_render_equals_scaled_disk_blend_of_subrays(tiny):
    assert _reference_by_records(tiny, oracle.render_reference)
    assert _reference_by_records(tiny, oracle.render_reference, ss=3, disk_scale=1.5)
    assert not _reference_by_records(tiny, _ref_offsets_without_half)
    assert not _reference_by_records(tiny, _ref_unscaled_disks)


def test_reference_render_scales_oval_extents(tiny):
    assert _reference_by_records(tiny, oracle.render_reference, ext_scale=1.0)
    assert not _reference_by_records(tiny, _ref_unscaled_disks, ext_scale=1.0)
