"""Pins of the oracle's tile streaming model (Sec. 4.2, tile streaming and
caching; Sec. 7.2): images cut into square tiles, only the tiles in the cache
can be sampled, and a view whose sample needs a missing tile is left out for
that ray.

Pinned by the camera-centre case (an eye at a source camera sees that view
alone, one texel centre per pixel, so every tile is needed and a missing tile
blanks exactly the pixels whose taps reach it), by sufficiency and
minimality of the visible-tile set (a render restricted to it equals the full
render, and dropping any one of its tiles changes some pixel's weight sum),
and by the empty cache."""
import ctypes

import numpy as np
import pytest

import lfsynth
import oracle


@pytest.mark.parametrize("page", [32, 64])
def test_visible_tiles_are_sufficient_and_minimal(tiny, tiny_oracle, page):
    pos, rot, hfov = tiny.head_pos[0], tiny.head_rot[0], tiny.hfov_deg
    vis = oracle.visible_tiles(tiny_oracle, pos, rot, hfov, 256, 256, page=page)
    full = oracle.render(tiny_oracle, pos, rot, hfov, 256, 256)
    part = oracle.render(tiny_oracle.with_residency(vis, page), pos, rot, hfov, 256, 256)
    assert 0 < vis.sum() < vis.size
    assert np.array_equal(full["rgb"], part["rgb"]) and np.array_equal(full["wsum"], part["wsum"])
    # tiles outside the set do not matter
    rng = np.random.default_rng(page)
    extra = vis | (rng.random(vis.shape) < 0.3)
    more = oracle.render(tiny_oracle.with_residency(extra, page), pos, rot, hfov, 256, 256)
    assert np.array_equal(full["rgb"], more["rgb"])
    # every tile of the set is needed: without it some ray loses a view
    on = np.argwhere(vis)
    for k in rng.choice(len(on), 4, replace=False):
        drop = vis.copy()
        drop[tuple(on[k])] = 0
        r = oracle.render(tiny_oracle.with_residency(drop, page), pos, rot, hfov, 256, 256)
        assert (r["wsum"] < full["wsum"]).any() and (r["count"] <= full["count"]).all()


def test_empty_cache_renders_nothing(tiny, tiny_oracle):
    none = np.zeros((tiny_oracle.n, 2, 2), np.uint8)
    r = oracle.render(tiny_oracle.with_residency(none, 64), tiny.head_pos[0], tiny.head_rot[0], tiny.hfov_deg,
                      64, 64)
    assert (r["wsum"] == 0).all() and (r["count"] == 0).all() and (r["rgb"] == 0).all()


def test_camera_centre_needs_every_tile_of_its_view_only(tiny):
    """Eye at view k's centre with its frame and FOV at twice its resolution,
    disks too small to reach a neighbour: every ray passes through the
    centre of view k's disk and no other disk, and eye pixel x' samples view
    k at texel coordinate x'/2 - 1/4 (never a texel centre), with taps
    x0 = floor(x'/2 - 1/4) and x0 + 1, likewise in y (away from the rim
    outside the mesh domain). All of view k's tiles are needed and no other
    view's; without tile (ty, tx) exactly the pixels with a tap column in
    [P tx, P tx + P - 1] and a tap row in [P ty, P ty + P - 1] render
    nothing, and every other pixel is unchanged."""
    V = tiny.views
    n, H, W = V.rgba8.shape[:3]
    P = 32
    R_small = 0.5 * lfsynth.min_nn(V.centres)
    ov = oracle.OracleViews(V.centres, V.rot, V.rgba8, V.zdepth, V.src_fov_deg, R_small)
    k = 21
    We, He = 2 * W, 2 * H
    vis = oracle.visible_tiles(ov, V.centres[k], V.rot[k], V.src_fov_deg, We, He, page=P)
    assert vis[k].all() and vis.sum() == vis[k].size
    full = oracle.render(ov, V.centres[k], V.rot[k], V.src_fov_deg, We, He)
    seen = (full["count"] == 1).reshape(He, We)  # all but the rim outside the mesh domain
    assert seen.mean() > 0.95 and (full["count"] <= 1).all()
    ty, tx = 1, 2
    res = np.ones_like(vis)
    res[k, ty, tx] = 0
    r = oracle.render(ov.with_residency(res, P), V.centres[k], V.rot[k], V.src_fov_deg, We, He)
    blank = (r["count"] == 0).reshape(He, We)
    y, x = np.mgrid[0:He, 0:We]
    x0, y0 = np.floor(x / 2 - 0.25), np.floor(y / 2 - 0.25)
    want = (x0 >= P * tx - 1) & (x0 <= P * tx + P - 1) & (y0 >= P * ty - 1) & (y0 <= P * ty + P - 1)
    assert np.array_equal(blank[seen], want[seen])
    same = ~blank.reshape(-1)
    assert np.array_equal(r["rgb"][same], full["rgb"][same]) and np.array_equal(r["count"][same], full["count"][same])


def test_band_classified_visible_tiles_bracket_the_visible_set(tiny, tiny_oracle):
    """must (tiles shown only through well-conditioned decisions, for the
    centre rays and their +-1e-3 px shifts) lies within the plain visible set
    of every one of those ray sets, and each of them within may; with no
    margin and no shift the bracket is tight up to the ill-conditioned
    decisions, which are rare (a few pairs)."""
    pos, rot, hfov = tiny.head_pos[0], tiny.head_rot[0], tiny.hfov_deg
    must, may = oracle.visible_tiles_band(tiny_oracle, pos, rot, hfov, 256, 256, page=32)
    assert must.sum() > 0 and (must <= may).all()
    for d in ((0.0, 0.0), (1e-3, 0.0), (0.0, -1e-3)):
        idx = None
        o, e = oracle.eye_rays(pos, rot, hfov, 256, 256, oracle.pixel_centres(256, 256, idx) + np.array(d))
        vis = np.zeros_like(must)
        oracle.lib().orc_visible_tiles(ctypes.byref(tiny_oracle.s), o.shape[0], o.ctypes.data, e.ctypes.data, 32,
                                       vis.ctypes.data)
        assert (must <= vis).all() and (vis <= may).all()
    tight_must, tight_may = oracle.visible_tiles_band(tiny_oracle, pos, rot, hfov, 256, 256, page=32, margin=0.0,
                                                      jitter=0.0)
    plain = oracle.visible_tiles(tiny_oracle, pos, rot, hfov, 256, 256, page=32)
    assert (tight_must <= plain).all() and (plain <= tight_may).all()
    assert int(tight_may.sum() - tight_must.sum()) <= max(2, plain.sum() // 200)
    # the margin makes the taps near a texel boundary undecided: with 0.49
    # texels almost every tap is, and may reaches tiles next to the visible ones
    wide_must, wide_may = oracle.visible_tiles_band(tiny_oracle, pos, rot, hfov, 256, 256, page=32, margin=0.49,
                                                    jitter=0.0)
    assert (wide_must <= plain).all() and (plain <= wide_may).all()
    assert wide_must.sum() < plain.sum() < wide_may.sum()
