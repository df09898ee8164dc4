"""Edge cases of the render path on the GPU: degenerate and extreme inputs.

A 1 x 1 eye and a one-pixel-wide eye against the oracle; more eyes in one call
than one launch carries (the chunked path) against per-eye renders; every
view disabled (Eq. 2's empty denominator: colour, weight sum and count all 0);
the input checks (no eyes, zero or oversized resolutions); the bandwidth
yardstick; and the work counters against the oracle's totals."""
import numpy as np
import pytest

import lfsynth
import oracle
from lfcheck import check_eye, gpu_render

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(tiny):
    from lfcheck import gpu_context
    c = gpu_context(tiny.views, "rgba32f", "f32")
    yield c
    c.close()


def test_single_pixel_and_single_column_eyes(tiny, tiny_oracle, ctx):
    p, R = tiny.head_pos[0], tiny.head_rot[0]
    for W, H in [(1, 1), (1, 37), (29, 1)]:
        s = check_eye(tiny_oracle, ctx, p, R, 60.0, W, H)
        print((W, H), s)


def test_more_eyes_than_one_launch(tiny, ctx):
    """17 eyes in one call (one launch carries 16): the same pixels as 17
    separate calls, bit for bit."""
    import torch
    from paper_1810_08860_amd import lf
    p, R = lfsynth.poses(91, 17, 0.2)
    eyes = [(p[k], R[k]) for k in range(17)]
    res = [(24 + 3 * k, 20 + k) for k in range(17)]
    got = gpu_render(ctx, eyes, 80.0, res)
    for e, r, g in zip(eyes, res, got):
        one = gpu_render(ctx, [e], 80.0, [r])[0]
        for x, y in zip(g, one):
            assert np.array_equal(x, y)
    torch.cuda.synchronize()


def test_every_view_disabled_renders_zero(tiny, ctx):
    from paper_1810_08860_amd import lf
    lf.lf_set_view_mask(ctx, np.zeros(tiny.views.n, np.uint8))
    try:
        rgb, ws, cnt = gpu_render(ctx, [(tiny.head_pos[0], tiny.head_rot[0])], tiny.hfov_deg, [(64, 48)])[0]
    finally:
        lf.lf_set_view_mask(ctx, None)
    assert (rgb == 0).all() and (ws == 0).all() and (cnt == 0).all()


def test_input_checks(tiny, ctx):
    import torch
    from paper_1810_08860_amd import lf
    out = torch.zeros(16 * 16 * 3, dtype=torch.float32, device="cuda")
    e = lf.make_eyes([(tiny.head_pos[0], tiny.head_rot[0])])
    L = lf.lib()
    for res in ([0, 16], [16, 0], [32769, 16], [16, -1]):
        r = np.array(res, np.int32)
        assert L.lf_render(ctx.handle, e, 1, 90.0, r.ctypes.data, out.data_ptr(), None, None, None) == lf.LF_EINVAL
        assert "resolution" in lf.lf_last_error()
    r = np.array([16, 16], np.int32)
    assert L.lf_render(ctx.handle, e, 0, 90.0, r.ctypes.data, out.data_ptr(), None, None, None) == lf.LF_EINVAL
    assert L.lf_render(ctx.handle, e, 1, 180.0, r.ctypes.data, out.data_ptr(), None, None, None) == lf.LF_EINVAL
    assert L.lf_render(ctx.handle, e, 1, 90.0, r.ctypes.data, None, None, None, None) == lf.LF_EINVAL


def test_stream_copy():
    """The bandwidth yardstick copies exactly and rejects misaligned or
    partial-vector sizes."""
    import torch
    from paper_1810_08860_amd import lf
    src = torch.randint(0, 2**31 - 1, (3 << 18,), dtype=torch.int32, device="cuda")
    dst = torch.zeros_like(src)
    lf.lf_stream_copy(src, dst, src.numel() * 4)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
    L = lf.lib()
    assert L.lf_stream_copy(src.data_ptr(), dst.data_ptr(), 20, None) == lf.LF_EINVAL
    assert L.lf_stream_copy(src.data_ptr() + 4, dst.data_ptr(), 64, None) == lf.LF_EINVAL
    assert L.lf_stream_copy(None, dst.data_ptr(), 64, None) == lf.LF_EINVAL


@pytest.mark.parametrize("active", [64, 17, 16, 1])
def test_fma_rate_yardstick(active):
    """The vector-rate yardstick runs its FMA chains on exactly the first
    `active` lanes of each wavefront (chain k of lane l starts at l + k and
    steps x -> 0.999 x + 0.001 in FP32 FMAs); the other lanes keep their start
    values. Bad arguments are rejected."""
    import torch
    from paper_1810_08860_amd import lf
    blocks, iters = 3, 100
    out = torch.full((blocks * 256,), -1.0, dtype=torch.float32, device="cuda")
    lf.lf_fma_rate(out, blocks, iters, active)
    torch.cuda.synchronize()
    got = out.cpu().numpy().reshape(blocks, 4, 64)
    lane = np.arange(64)
    x = (lane[:, None] + np.arange(8)[None, :]).astype(np.float32)
    y = x.copy()
    a, b = np.float32(0.999), np.float32(0.001)
    for _ in range(iters):  # one rounding per step: the FP64 product of two FP32 values is exact
        y = (y.astype(np.float64) * np.float64(a) + np.float64(b)).astype(np.float32)
    x = np.where((lane < active)[:, None], y, x)
    want = ((x[:, 0] + x[:, 1]) + (x[:, 2] + x[:, 3])) + ((x[:, 4] + x[:, 5]) + (x[:, 6] + x[:, 7]))
    for blk in got.reshape(-1, 64):
        np.testing.assert_allclose(blk[:active], want[:active], rtol=1e-6)
        assert np.array_equal(blk[active:], want[active:])  # untouched start values, exact
    L = lf.lib()
    assert L.lf_fma_rate(None, 1, 1, 64, None) == lf.LF_EINVAL
    for bad in ((0, 1, 64), (1, 0, 64), (1, 1, 0), (1, 1, 65)):
        assert L.lf_fma_rate(out.data_ptr(), *bad, None) == lf.LF_EINVAL


def test_work_counters_match_oracle(tiny, tiny_oracle, ctx):
    """The work counters behind the bench's algorithmic flop count: pixels,
    candidates and samples are the oracle's own totals over a full frame (up
    to the (ray, view) pairs whose disk or hit decision is ill-conditioned);
    every pixel tests its tile's list, so disk tests >= candidates, and every
    sample needs a visited mesh cell, so cells >= samples."""
    from paper_1810_08860_amd import lf
    p, R = tiny.head_pos[0], tiny.head_rot[0]
    lf.lf_set_view_mask(ctx, None)
    st = lf.lf_render_stats(ctx, [(p, R)], tiny.hfov_deg, [(256, 256)])
    ref = oracle.render(tiny_oracle, p, R, tiny.hfov_deg, 256, 256, cap=32)
    band_c = int((ref["cand_band"] >= 0).sum())
    band_h = int((ref["contrib_band"] >= 0).sum())
    print(st, "oracle candidates", int(ref["n_cand"].sum()), "samples", int(ref["count"].sum()),
          "band pairs", band_c, band_h)
    assert st["pixels"] == 256 * 256
    assert abs(st["candidates"] - int(ref["n_cand"].sum())) <= band_c
    assert abs(st["samples"] - int(ref["count"].sum())) <= band_c + band_h
    assert st["disk_tests"] >= st["candidates"] and st["cells"] >= st["samples"]
