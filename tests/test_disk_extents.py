"""Oval disk extents (Sec. 4.4) of the library (host C++, through the C ABI)
against the oracle's (scipy's convex hull of the centre directions), on the
rig the workloads use. Where the four centres of two adjacent triangles are
(nearly) co-circular both diagonals are Delaunay and the two hulls may choose
differently; views of such quads are excluded from the exact comparison and
only checked to be valid (each extent reached by some ring neighbour)."""
import numpy as np
import pytest

import lfsynth
import oracle
from paper_1810_08860_amd import lf


def _near_cocircular_views(centres, tol):
    from scipy.spatial import ConvexHull
    u = centres / np.linalg.norm(centres, axis=1, keepdims=True)
    opp = {}
    for f in ConvexHull(u).simplices:
        for k in range(3):
            a, b, c = int(f[k]), int(f[(k + 1) % 3]), int(f[(k + 2) % 3])
            opp.setdefault((min(a, b), max(a, b)), []).append(c)
    views, smallest = set(), np.inf
    for (a, b), (c, d) in opp.items():
        vol = abs(np.linalg.det(np.stack([u[b] - u[a], u[c] - u[a], u[d] - u[a]])))
        smallest = min(smallest, vol)
        if vol < tol:
            views |= {a, b, c, d}
    return views, smallest


@pytest.mark.parametrize("n", [64, 1024])
def test_library_extents_match_oracle(n):
    c, r = lfsynth.rig(n)
    got = lf.lf_disk_extents(c, r)
    want, ring = oracle.disk_extents(c, r)
    amb, smallest = _near_cocircular_views(c, 1e-9)
    print(f"n={n}: smallest quad volume {smallest:.3g}, near-co-circular views {len(amb)}")
    keep = np.array([i not in amb for i in range(n)])
    np.testing.assert_allclose(got[keep], want[keep], rtol=0, atol=1e-12)
    assert (got > 0).all()
    np.testing.assert_allclose(lf.lf_disk_extents(c, r, scale=1.5), 1.5 * got, rtol=1e-15)


def test_library_extents_closed_form_bipyramid():
    th = np.radians([0.0, 120.0, 240.0])
    dirs = np.array([[0, 0, 1], [0, 0, -1]] + [[np.cos(t), np.sin(t), 0.0] for t in th])
    c = 0.35 * dirs
    R = []
    for x in dirs:
        f = x / np.linalg.norm(x)
        rr = np.cross(f, [0, 0, 1.0])
        if np.linalg.norm(rr) < 1e-9:
            rr = np.cross(f, [0, 1.0, 0])
        rr /= np.linalg.norm(rr)
        R.append(np.stack([rr, np.cross(rr, f), f], 1))
    got = lf.lf_disk_extents(c, np.stack(R))
    s3 = 0.35 * np.sqrt(3) / 2
    np.testing.assert_allclose(got[0], [0.175, 0.35, s3, s3], atol=1e-12)
    np.testing.assert_allclose(got[2], [s3, s3, 0.35, 0.35], atol=1e-12)


def test_library_extents_reject_degenerate_rigs():
    c, r = lfsynth.rig(16)
    with pytest.raises(lf.LFError):
        lf.lf_disk_extents(c[:3], r[:3])                      # fewer than four views
    flat = c.copy()
    flat[:, 2] = 0.0                                           # every direction on one great circle
    flat[np.linalg.norm(flat, axis=1) < 1e-9] = [0.35, 0.0, 0.0]
    with pytest.raises(lf.LFError):
        lf.lf_disk_extents(flat, r)
    dup = c.copy()
    dup[5] = 2.0 * dup[4]                                      # same direction twice
    with pytest.raises(lf.LFError):
        lf.lf_disk_extents(dup, r)
    with pytest.raises(lf.LFError):
        lf.lf_disk_extents(c, r, scale=0.0)
