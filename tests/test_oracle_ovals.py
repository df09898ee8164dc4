"""Pins of the oracle's asymmetric oval disks (Sec. 4.4 of the paper).

The disk of a view is the union of four elliptic quarters around its centre,
one per quadrant of the disk's (u, v) axes, bounded by the extents e+u, e-u,
e+v, e-v; each extent reaches the furthest 1-ring neighbour (Delaunay
triangulation of the disk centres) in that direction. The extents are pinned
on rigs whose triangulation and projections are known in closed form, the
falloff on constructed rays in every quadrant, and equal extents against the
circular disk.
"""
import numpy as np
import pytest

import lfsynth
import oracle

RIG_R = 0.35


def _rig_frame(c):
    """The rig's frame convention: f = c/|c|, r = f x z (f x y at the poles), u = r x f."""
    f = np.asarray(c, float) / np.linalg.norm(c)
    r = np.cross(f, [0.0, 0.0, 1.0])
    if np.linalg.norm(r) < 1e-9:
        r = np.cross(f, [0.0, 1.0, 0.0])
    r /= np.linalg.norm(r)
    return np.stack([r, np.cross(r, f), f], 1)


def _rig(dirs):
    c = RIG_R * np.asarray(dirs, float)
    return c, np.stack([_rig_frame(x) for x in c])


def test_bipyramid_extents_closed_form():
    """Poles and three equatorial views 120 deg apart: the hull is six
    triangles, each pole's 1-ring is the equator, each equatorial view's ring is
    both poles and the two other equatorial views. Projections on the frames
    give the extents below (an asymmetric disk at the north pole)."""
    th = np.radians([0.0, 120.0, 240.0])
    dirs = [[0, 0, 1], [0, 0, -1]] + [[np.cos(t), np.sin(t), 0.0] for t in th]
    c, R = _rig(dirs)
    ext, ring = oracle.disk_extents(c, R)
    assert ring[0] == {2, 3, 4} and ring[1] == {2, 3, 4}
    assert ring[2] == {0, 1, 3, 4}
    s3 = RIG_R * np.sqrt(3) / 2
    # north pole: r = -x, u = y; equator points project to (-0.35 cos t, 0.35 sin t)
    np.testing.assert_allclose(ext[0], [RIG_R / 2, RIG_R, s3, s3], atol=1e-12)
    # south pole: r = +x, u = y
    np.testing.assert_allclose(ext[1], [RIG_R, RIG_R / 2, s3, s3], atol=1e-12)
    # equatorial view at t = 0: r = -y, u = z; poles at v = +-0.35, others at u = -+0.35 sin 120
    np.testing.assert_allclose(ext[2], [s3, s3, RIG_R, RIG_R], atol=1e-12)


def test_octahedron_extents_are_the_edge_projection():
    dirs = [[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]]
    c, R = _rig(dirs)
    ext, ring = oracle.disk_extents(c, R)
    for i in range(6):
        assert len(ring[i]) == 4 and (i ^ 1) not in ring[i]  # never the antipode
    np.testing.assert_allclose(ext, RIG_R, atol=1e-12)


def test_fibonacci_rig_extents_reach_every_ring_neighbour(tiny):
    """Every 1-ring neighbour's projected centre lies in the extents' box, and
    the box touches the furthest neighbour on each side."""
    V = tiny.views
    ext, ring = oracle.disk_extents(V.centres, V.rot)
    for i in range(V.n):
        q = V.centres[sorted(ring[i])] - V.centres[i]
        du, dv = q @ V.rot[i][:, 0], q @ V.rot[i][:, 1]
        assert (du <= ext[i, 0] + 1e-15).all() and (-du <= ext[i, 1] + 1e-15).all()
        assert (dv <= ext[i, 2] + 1e-15).all() and (-dv <= ext[i, 3] + 1e-15).all()
        assert np.isclose(du.max(), ext[i, 0]) and np.isclose(dv.min(), -ext[i, 3])
        assert 4 <= len(ring[i]) <= 8


def test_oval_falloff_in_every_quadrant(tiny, tiny_oracle):
    V = tiny.views
    ext = np.tile([0.10, 0.20, 0.15, 0.05], (V.n, 1))
    ov = tiny_oracle.with_disk_extents(ext)
    o = np.array([0.01, -0.02, 0.03])
    for i in (0, 21, 50):
        c, Ri = V.centres[i], V.rot[i]
        r_ax, u_ax = Ri[:, 0], Ri[:, 1]
        for a, b in ((0.3, 0.4), (-0.6, 0.2), (-0.1, -0.7), (0.5, -0.5), (0.9, 0.0), (0.0, -0.9), (-0.95, 0.0)):
            eu = ext[i, 0] if a >= 0 else ext[i, 1]
            ev = ext[i, 2] if b >= 0 else ext[i, 3]
            target = c + a * eu * r_ax + b * ev * u_ax
            _, u, v, rho = oracle.disk(ov, i, o, 1.7 * (target - o))
            assert u == pytest.approx(a * eu, abs=1e-14) and v == pytest.approx(b * ev, abs=1e-14)
            assert rho == pytest.approx(1.0 - np.hypot(a, b), abs=1e-13), (a, b)
        # outside the oval but inside its bounding box: not a candidate
        target = c + 0.8 * ext[i, 0] * r_ax + 0.8 * ext[i, 2] * u_ax
        rec = oracle.records(ov, o, target - o)[i]
        assert rec["cand"] == 0 and rec["rho"] == pytest.approx(1.0 - 0.8 * np.sqrt(2), abs=1e-13)


def test_equal_extents_reduce_to_the_circle(tiny, tiny_oracle, rng):
    V = tiny.views
    ov_o = tiny_oracle.with_disk_extents(np.full((V.n, 4), V.disk_radius))
    pxy = rng.uniform(0, 256, (300, 2))
    o, e = oracle.eye_rays(tiny.head_pos[0], tiny.head_rot[0], tiny.hfov_deg, 256, 256, pxy)
    for k in range(0, 300, 37):
        rc, ro = oracle.records(tiny_oracle, o[k], e[k]), oracle.records(ov_o, o[k], e[k])
        ok = np.isfinite(rc["rho"])
        np.testing.assert_allclose(ro["rho"][ok], rc["rho"][ok], atol=1e-12)
    a = oracle.render_rays(tiny_oracle, o, e)
    b = oracle.render_rays(ov_o, o, e)
    np.testing.assert_allclose(b["rgb"], a["rgb"], atol=1e-10)
    np.testing.assert_array_equal(b["count"], a["count"])


def test_reference_render_scales_oval_extents(tiny, tiny_oracle):
    """The offline reference scales oval extents like it scales the radius."""
    V = tiny.views
    ext, _ = oracle.disk_extents(V.centres, V.rot)
    ov = tiny_oracle.with_disk_extents(ext)
    idx = np.array([1000, 30000, 45000])
    ref = oracle.render_reference(ov, tiny.head_pos[0], tiny.head_rot[0], tiny.hfov_deg, 256, 256, idx, ss=1,
                                  disk_scale=2.0)
    plain = oracle.render(ov.with_disk_extents(2.0 * ext), tiny.head_pos[0], tiny.head_rot[0], tiny.hfov_deg,
                          256, 256, idx)
    np.testing.assert_allclose(ref, plain["rgb"], atol=1e-12)
