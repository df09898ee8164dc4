"""Pins of the oracle's YUV420 image form (the paper's tile cache stores its
tiles as a full-resolution luma plane and a half-resolution two-channel chroma
plane, sampled separately and recombined to RGB, Sec. 7.2).

Pinned against the real-valued full-range BT.601 transform (the fixed-point
encoder stays within one 8-bit step of it), against lossless special cases
(grey images carry no chroma) and against exact reproduction of 2x2-block
constant images at block centres up to the 8-bit rounding of the transform.
"""
import numpy as np

import lfsynth
import oracle


def _bt601(rgb):
    R, G, B = [rgb[..., k].astype(np.float64) for k in range(3)]
    Y = 0.299 * R + 0.587 * G + 0.114 * B
    Cb = 128 - 0.168736 * R - 0.331264 * G + 0.5 * B
    Cr = 128 + 0.5 * R - 0.418688 * G - 0.081312 * B
    return np.stack([Y, Cb, Cr], -1)


def test_encoder_within_one_step_of_bt601():
    rng = np.random.default_rng(4)
    cols = rng.integers(0, 256, (500, 3))
    cols = np.concatenate([cols, [[255, 0, 0], [0, 255, 0], [0, 0, 255], [255, 255, 255], [0, 0, 0]]])
    # every colour fills a 2x2 block, so its chroma sample is its own chroma
    img = np.zeros((1, 2, 2 * len(cols), 4), np.uint8)
    img[0, :, :, :3] = np.repeat(cols, 2, axis=0)[None]
    img[..., 3] = 255
    y, uv = oracle.yuv420_encode(img)
    want = np.clip(_bt601(cols), 0, 255)
    got = np.stack([y[0, 0, 0::2], uv[0, 0, :, 0], uv[0, 0, :, 1]], -1).astype(np.float64)
    assert np.abs(got - want).max() <= 1.0
    assert (y[0, 1, 0::2] == y[0, 0, 0::2]).all() and (y[0, :, 1::2] == y[0, :, 0::2]).all()


def test_chroma_is_the_rounded_block_mean():
    rng = np.random.default_rng(5)
    img = rng.integers(0, 256, (2, 6, 8, 4)).astype(np.uint8)
    y, uv = oracle.yuv420_encode(img)
    # chroma of each pixel alone: the pixel repeated over a 2x2 block
    one = np.repeat(np.repeat(img, 2, axis=1), 2, axis=2)
    _, uv1 = oracle.yuv420_encode(one)
    per_px = uv1.astype(np.int64)  # (2, 6, 8, 2): the chroma of pixel (r, c)
    blocks = per_px.reshape(2, 3, 2, 4, 2, 2).sum(axis=(2, 4))
    assert np.array_equal(uv, ((blocks + 2) >> 2).astype(np.uint8))


def test_grey_views_are_lossless(tiny):
    """Grey texels have Cb = Cr = 128 and Y equal to the grey level, so the
    YUV420 render equals the RGB render."""
    V = tiny.views
    g = V.rgba8[..., :3].mean(-1).astype(np.uint8)
    grey = np.stack([g, g, g, np.full_like(g, 255)], -1)
    ov = oracle.OracleViews(V.centres, V.rot, grey, V.zdepth, V.src_fov_deg, V.disk_radius)
    oy = ov.with_yuv420()
    assert (oy.yuv_uv == 128).all()
    idx = np.arange(0, 256 * 256, 53)
    a = oracle.render(ov, tiny.head_pos[0], tiny.head_rot[0], tiny.hfov_deg, 256, 256, idx)
    b = oracle.render(oy, tiny.head_pos[0], tiny.head_rot[0], tiny.hfov_deg, 256, 256, idx)
    assert np.abs(a["rgb"] - b["rgb"]).max() < 1e-12 and np.array_equal(a["wsum"], b["wsum"])


def test_block_constant_views_reproduce_block_colours(tiny):
    """Views whose 2x2 blocks are constant, seen from view k's own centre with
    disks too small to reach a neighbour, by an eye of half the view's
    resolution: every eye ray passes through a block centre, where luma and
    chroma are sampled exactly, so the render is the block colour up to the
    8-bit rounding of the transform: |dR| <= (1 + 1.402) / 255,
    |dG| <= (1 + 0.344 + 0.714) / 255, |dB| <= (1 + 1.772) / 255 (one step of
    luma and chroma each). A chroma plane read with the wrong offset or
    stride, or a wrong sign in the inverse, moves colours by far more."""
    V = tiny.views
    rng = np.random.default_rng(6)
    n, H, W = V.rgba8.shape[:3]
    blocks = rng.integers(0, 256, (n, H // 2, W // 2, 3)).astype(np.uint8)
    img = np.zeros_like(V.rgba8)
    img[..., :3] = np.repeat(np.repeat(blocks, 2, axis=1), 2, axis=2)
    img[..., 3] = 255
    R_small = 0.5 * lfsynth.min_nn(V.centres)
    oy = oracle.OracleViews(V.centres, V.rot, img, V.zdepth, V.src_fov_deg, R_small).with_yuv420()
    bound = np.array([2.402, 2.058, 2.772]) / 255 + 1e-9
    for k in (9, 50):
        r = oracle.render(oy, V.centres[k], V.rot[k], V.src_fov_deg, W // 2, H // 2)
        ok = r["count"] == 1
        assert ok.mean() > 0.95
        want = blocks[k].reshape(-1, 3)[ok] / 255.0
        assert (np.abs(r["rgb"][ok] - want) <= bound).all()
