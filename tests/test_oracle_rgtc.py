"""Pins of the oracle's RGTC form of the YUV420 planes (the paper's renderer
can transcode its cached YUV420 tiles to RGTC, a 4x smaller tile cache,
Sec. 7.2).

The block format is the published RGTC1/RGTC2 (BC4/BC5) one, so the decoder is
pinned by blocks assembled bit by bit from that layout (endpoint bytes, then
3-bit codes of texel 4 y + x at bit 3 (4 y + x) of a little-endian 48-bit
field) whose palettes fall on integers; the encoder by lossless special cases,
by the nearest-palette property checked by brute force over all eight points,
and by the error bound it implies; the plumbing by renders of block-constant
views, which RGTC codes exactly and must therefore equal the YUV420 render.
"""
import numpy as np

import oracle


def _block(e0, e1, codes):
    bits = 0
    for t, c in enumerate(codes):
        bits |= int(c) << (3 * t)
    return np.array([e0, e1] + [(bits >> (8 * b)) & 255 for b in range(6)], np.uint8)


def _decode_luma(block):
    """Decode one RGTC1 block as the 4 x 4 luma plane of a 1 x 8 x 8 light
    field (its other three blocks zero)."""
    yb = np.zeros((1, 2, 2, 8), np.uint8)
    yb[0, 0, 0] = block
    y, _ = oracle.rgtc_decode(yb, np.zeros((1, 1, 1, 16), np.uint8))
    return y[0, :4, :4]


def test_decode_eight_point_palette_and_bit_layout():
    # e0 = 210 > e1 = 70: points 210, 70, then sevenths from e0 towards e1,
    # 190, 170, 150, 130, 110, 90 (all integers since 140 = 7 * 20)
    codes = [t % 8 for t in range(16)]
    got = _decode_luma(_block(210, 70, codes))
    value = {0: 210, 1: 70, 2: 190, 3: 170, 4: 150, 5: 130, 6: 110, 7: 90}
    want = np.array([value[c] for c in codes], np.float64).reshape(4, 4)
    assert np.array_equal(got, want)
    # one code in an otherwise zero field lands on exactly texel (x, y)
    for t in (0, 5, 10, 15):
        c = [0] * 16
        c[t] = 1
        g = _decode_luma(_block(210, 70, c))
        assert g[t // 4, t % 4] == 70 and (g == 70).sum() == 1


def test_decode_six_point_palette():
    # e0 = 40 <= e1 = 240: points 40, 240, fifths 80, 120, 160, 200, then 0 and 255
    codes = [t % 8 for t in range(16)]
    got = _decode_luma(_block(40, 240, codes))
    value = {0: 40, 1: 240, 2: 80, 3: 120, 4: 160, 5: 200, 6: 0, 7: 255}
    want = np.array([value[c] for c in codes], np.float64).reshape(4, 4)
    assert np.array_equal(got, want)


def _palette(e0, e1):
    if e0 > e1:
        return np.array([e0, e1] + [((8 - c) * e0 + (c - 1) * e1) / 7 for c in range(2, 8)])
    return np.array([e0, e1] + [((6 - c) * e0 + (c - 1) * e1) / 5 for c in range(2, 6)] + [0.0, 255.0])


def test_encoder_picks_the_nearest_palette_point():
    rng = np.random.default_rng(7)
    n, H, W = 3, 16, 24
    y = rng.integers(0, 256, (n, H, W)).astype(np.uint8)
    y[0, :4, :4] = 99  # a constant block
    y[1, 4:8, 8:12] = rng.choice([3, 250], (4, 4))  # two values
    y[2, :4, 4:8] = rng.integers(100, 106, (4, 4))  # a narrow range
    uv = rng.integers(0, 256, (n, H // 2, W // 2, 2)).astype(np.uint8)
    yb, uvb = oracle.rgtc_encode(y, uv)
    dy, duv = oracle.rgtc_decode(yb, uvb)
    for plane, dec, blocks, ch in ((y[..., None], dy[..., None], yb[..., None, :8], 1),
                                   (uv, duv, uvb.reshape(*uvb.shape[:3], 2, 8), 2)):
        for i in range(n):
            for by in range(blocks.shape[1]):
                for bx in range(blocks.shape[2]):
                    for c in range(ch):
                        src = plane[i, 4 * by:4 * by + 4, 4 * bx:4 * bx + 4, c].astype(np.float64)
                        got = dec[i, 4 * by:4 * by + 4, 4 * bx:4 * bx + 4, c]
                        e0, e1 = blocks[i, by, bx, c, :2]
                        assert e0 == src.max() and e1 == src.min()
                        pal = _palette(float(e0), float(e1))
                        assert np.isin(got, pal).all()
                        best = np.abs(src[..., None] - pal).min(-1)
                        assert np.allclose(np.abs(got - src), best, atol=1e-12)
                        assert np.abs(got - src).max() <= (e0 - e1) / 14 + 1e-12
    assert (dy[0, :4, :4] == 99).all()
    assert np.array_equal(dy[1, 4:8, 8:12], y[1, 4:8, 8:12])


def test_blocks_on_their_own_palette_are_lossless():
    rng = np.random.default_rng(8)
    y = np.zeros((1, 8, 8), np.uint8)
    for by in range(2):
        for bx in range(2):
            lo = int(rng.integers(0, 100))
            step = int(rng.integers(1, 22))
            vals = lo + step * rng.integers(0, 8, 16)
            vals[:2] = [lo, lo + 7 * step]
            y[0, 4 * by:4 * by + 4, 4 * bx:4 * bx + 4] = rng.permutation(vals).reshape(4, 4)
    yb, uvb = oracle.rgtc_encode(y, np.full((1, 4, 4, 2), 128, np.uint8))
    dy, duv = oracle.rgtc_decode(yb, uvb)
    assert np.array_equal(dy, y) and (duv == 128).all()


def test_chroma_channels_are_separate_blocks():
    """Cb constant a and Cr constant b: the RGTC2 block is a's RGTC1 block then
    b's, and both decode exactly."""
    uv = np.zeros((1, 8, 12, 2), np.uint8)
    uv[..., 0], uv[..., 1] = 37, 201
    _, uvb = oracle.rgtc_encode(np.zeros((1, 16, 24), np.uint8), uv)
    assert (uvb[..., 0] == 37).all() and (uvb[..., 1] == 37).all()
    assert (uvb[..., 8] == 201).all() and (uvb[..., 9] == 201).all()
    _, duv = oracle.rgtc_decode(np.zeros((1, 4, 6, 8), np.uint8), uvb)
    assert (duv[..., 0] == 37).all() and (duv[..., 1] == 201).all()


def test_block_constant_views_render_as_yuv420(tiny):
    """Views constant over 8 x 8 blocks have luma constant over every RGTC1
    block and chroma constant over every RGTC2 block, which RGTC codes
    exactly: the RGTC render equals the YUV420 render. A block read at the
    wrong address or a chroma channel swapped breaks the equality."""
    V = tiny.views
    n, H, W = V.rgba8.shape[:3]
    rng = np.random.default_rng(9)
    cols = rng.integers(0, 256, (n, H // 8, W // 8, 3)).astype(np.uint8)
    img = np.zeros_like(V.rgba8)
    img[..., :3] = np.repeat(np.repeat(cols, 8, axis=1), 8, axis=2)
    img[..., 3] = 255
    ov = oracle.OracleViews(V.centres, V.rot, img, V.zdepth, V.src_fov_deg, V.disk_radius)
    a = ov.with_yuv420()
    b = ov.with_yuv420_rgtc()
    dy, duv = oracle.rgtc_decode(b.rgtc_y, b.rgtc_uv)
    assert np.array_equal(dy, a.yuv_y) and np.array_equal(duv, a.yuv_uv)
    idx = np.arange(0, 256 * 256, 37)
    ra = oracle.render(a, tiny.head_pos[0], tiny.head_rot[0], tiny.hfov_deg, 256, 256, idx)
    rb = oracle.render(b, tiny.head_pos[0], tiny.head_rot[0], tiny.hfov_deg, 256, 256, idx)
    assert np.abs(ra["rgb"] - rb["rgb"]).max() < 1e-12 and np.array_equal(ra["wsum"], rb["wsum"])


def test_rgtc_render_stays_near_yuv420(tiny):
    """On the textured views the RGTC render differs from the YUV420 one by
    the block quantisation only: at most (max - min) / 14 per texel of a
    block, so the render moves by a few 8-bit steps at most (a sanity bound;
    a mis-addressed block moves colours by far more)."""
    V = tiny.views
    ov = oracle.OracleViews.from_views(V)
    a = ov.with_yuv420()
    b = ov.with_yuv420_rgtc()
    idx = np.arange(0, 256 * 256, 41)
    ra = oracle.render(a, tiny.head_pos[0], tiny.head_rot[0], tiny.hfov_deg, 256, 256, idx)
    rb = oracle.render(b, tiny.head_pos[0], tiny.head_rot[0], tiny.hfov_deg, 256, 256, idx)
    d = np.abs(ra["rgb"] - rb["rgb"]).max(1)
    print(f"rgtc vs yuv420: mean {d.mean():.3g}, max {d.max():.3g}")
    assert d.mean() < 4 / 255
