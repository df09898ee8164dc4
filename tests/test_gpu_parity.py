"""GPU parity of the HIP path against the FP64 oracle on the tiny light field
(64 views, 128^2 images and depth), through the C ABI."""
import numpy as np
import pytest

import lfsynth
import oracle
from lfcheck import check_reference, check_eye, gpu_candidates, gpu_context, gpu_render, unstable_mask

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx32(tiny):
    c = gpu_context(tiny.views, "rgba32f", "f32")
    yield c
    c.close()


def test_full_frame_fp32_matches_oracle(tiny, tiny_oracle, ctx32):
    s = check_eye(tiny_oracle, ctx32, tiny.head_pos[0], tiny.head_rot[0], tiny.hfov_deg, 256, 256)
    print("tiny 256^2 fp32:", s)


@pytest.mark.parametrize("img,geo,tol", [("rgba8", "f32", 1e-4), ("rgba16f", "f32", 2.0 / 255),
                                         ("rgba8", "f16", 2.0 / 255), ("rgba16f", "f16", 2.0 / 255),
                                         ("rgba8", "u16", 1e-3)])
def test_storage_formats(tiny, tiny_oracle, img, geo, tol):
    """Compact storage keeps FP32 arithmetic; error against the FP64 oracle on
    stable pixels stays within tol (RGBA8 is the source data itself). The
    16-bit inverse-depth codes err by at most range / 131070 (range below
    1 / 0.15 m): with disk offsets |D| below 0.05 m and about 300 source pixels
    per unit of the image plane, a sample moves by under 1e-3 pixel, so an
    image whose values change by at most 1 per pixel moves by under 1e-3."""
    ctx = gpu_context(tiny.views, img, geo)
    W = H = 256
    idx = np.arange(0, W * H, 3)
    pos, rot = tiny.head_pos[0], tiny.head_rot[0]
    rgb, ws, cnt = gpu_render(ctx, [(pos, rot)], tiny.hfov_deg, [(W, H)])[0]
    ref = oracle.render(tiny_oracle, pos, rot, tiny.hfov_deg, W, H, idx)["rgb"]
    unstable = unstable_mask(tiny_oracle, pos, rot, tiny.hfov_deg, W, H, idx, ref)
    err = np.abs(rgb[idx] - ref).max(1)
    print(f"{img}/{geo}: max err stable {err[~unstable].max():.3g}, all {err.max():.3g}, "
          f"unstable {unstable.mean() * 100:.3f}%")
    assert err[~unstable].max() <= tol
    ctx.close()


def test_u16_codes_of_a_flat_view_decode_exactly(tiny):
    """A view whose vertices all share one depth has a zero code step: every
    code is 0 and decodes to the view's base, its FP32 inverse depth exactly,
    so with such meshes the 16-bit form renders the FP32 form's image bit for
    bit (one depth per view, different across views)."""
    import dataclasses
    V = tiny.views
    z = np.repeat(np.linspace(1.8, 4.5, V.n, dtype=np.float32)[:, None, None], V.mesh_m, 1)
    z = np.ascontiguousarray(np.repeat(z, V.mesh_m, 2))
    flat = dataclasses.replace(V, zdepth=z)
    c32, c16 = gpu_context(flat, "rgba8", "f32"), gpu_context(flat, "rgba8", "u16")
    p, R = tiny.head_pos[0], tiny.head_rot[0]
    a = gpu_render(c32, [(p, R)], 90.0, [(128, 96)])[0]
    b = gpu_render(c16, [(p, R)], 90.0, [(128, 96)])[0]
    assert (a[2] > 0).mean() > 0.5  # most pixels see the flat meshes
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    c32.close()
    c16.close()


def test_eye_next_to_a_source_camera_centre(tiny, tiny_oracle, ctx32):
    """An eye 1 mm inside the capture sphere behind view k's centre, with view
    k's frame and field of view: its rays cross disk k within millimetres of
    the centre, so view k's lines through its mesh are nearly single points
    (steep lines, huge cell-exit steps). The image matches the oracle, lists
    included. The centre itself lies on disk k's plane, which the boundary
    rejects."""
    import torch
    from paper_1810_08860_amd import lf
    V = tiny.views
    for k in (5, 33):
        c = V.centres[k]
        pos = c * (1.0 - 1e-3 / np.linalg.norm(c))
        s = check_eye(tiny_oracle, ctx32, pos, V.rot[k], V.src_fov_deg, 96, 96)
        print(f"eye 1 mm behind view {k}'s centre:", s)
    out = torch.zeros(16 * 16 * 3, dtype=torch.float32, device="cuda")
    with pytest.raises(lf.LFError) as ei:
        lf.lf_render(ctx32, [(V.centres[5], V.rot[5])], V.src_fov_deg, (16, 16), out)
    assert ei.value.code == lf.LF_EINVAL and "disk plane" in str(ei.value)


def test_ragged_sizes_and_several_eyes(tiny, tiny_oracle, ctx32):
    """Eyes of ragged sizes (partial tiles on both axes) in one call."""
    p, R = tiny.head_pos[0], tiny.head_rot[0]
    p2, R2 = lfsynth.poses(77, 1, 0.2)
    eyes = [(p, R), (p2[0], R2[0]), (p + np.array([0.01, 0.0, -0.02]), R)]
    res = [(250, 130), (131, 77), (8, 9)]
    outs = gpu_render(ctx32, eyes, 75.0, res)
    for (pos, rot), (W, H), got in zip(eyes, res, outs):
        s = check_eye(tiny_oracle, ctx32, pos, rot, 75.0, W, H, gpu=got, lists=(W * H < 20000))
        print((W, H), s)


def test_launch_shapes_give_identical_images(tiny, ctx32):
    """The tile shape and candidate cap change the schedule, never the
    result: every pixel blends the same exact candidate set in the same order."""
    from paper_1810_08860_amd import lf
    p, R = tiny.head_pos[0], tiny.head_rot[0]
    res = [(200, 120)]
    base = gpu_render(ctx32, [(p, R)], 90.0, res)[0]
    for tw, th, cap in ((8, 8, 0), (32, 8, 0), (16, 8, 0), (8, 32, 0), (8, 16, 0), (16, 16, 8), (16, 16, 1),
                        (32, 8, 16), (8, 8, 32)):
        # a candidate cap below a tile's candidate count sends that tile to the
        # exact scan over every view: the same views in the same order
        lf.lf_set_tune(ctx32, tw, th, cap)
        got = gpu_render(ctx32, [(p, R)], 90.0, res)[0]
        for a, b in zip(base, got):
            assert np.array_equal(a, b), (tw, th, cap)
    lf.lf_set_tune(ctx32)


def test_candidate_list_overflow_falls_back_exactly():
    """Disks large enough that tile candidate lists exceed their 64-entry
    capacity (256 views, 6x radius): overflowing tiles scan every view and
    stay exact."""
    v = lfsynth.make_views(256, 64, 64, 3, 5)
    R_big = 6.0 * v.disk_radius
    ctx = gpu_context(v, "rgba32f", "f32", disk_radius=R_big)
    ov = oracle.OracleViews.from_views(v, disk_radius=R_big)
    p, R = lfsynth.poses(1005, 1, 0.2)
    W = H = 96
    _, _, ncand = gpu_candidates(ctx, (p[0], R[0]), 90.0, W, H, cap=192)
    assert ncand.max() > 64
    s = check_eye(ov, ctx, p[0], R[0], 90.0, W, H, idx=np.arange(0, W * H, 5), cap=192)
    print("overflow:", s, "max candidates per pixel", ncand.max())
    ctx.close()


def test_render_is_deterministic(tiny, ctx32):
    p, R = tiny.head_pos[0], tiny.head_rot[0]
    a = gpu_render(ctx32, [(p, R)], 90.0, [(256, 256)])[0]
    b = gpu_render(ctx32, [(p, R)], 90.0, [(256, 256)])[0]
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_reference_render_matches_oracle(tiny, tiny_oracle, ctx32):
    import torch
    from paper_1810_08860_amd import lf
    p, R = tiny.head_pos[0], tiny.head_rot[0]
    W = H = 64
    out = torch.zeros(W * H * 3, dtype=torch.float32, device="cuda")
    lf.lf_render_reference(ctx32, [(p, R)], 90.0, (W, H), 3, 2.0, out)
    torch.cuda.synchronize()
    got = out.view(-1, 3).cpu().numpy().astype(np.float64)
    check_reference(tiny_oracle, got, p, R, 90.0, W, H, np.arange(0, W * H, 7), 3, 2.0, "reference ss=3")
    # 4 x 4 sub-rays (the corrector's target), a ragged eye
    W, H = 72, 40
    out = torch.zeros(W * H * 3, dtype=torch.float32, device="cuda")
    lf.lf_render_reference(ctx32, [(p, R)], 90.0, (W, H), 4, 2.0, out)
    torch.cuda.synchronize()
    got = out.view(-1, 3).cpu().numpy().astype(np.float64)
    check_reference(tiny_oracle, got, p, R, 90.0, W, H, np.arange(0, W * H, 5), 4, 2.0, "reference ss=4")


def test_eye_outside_capture_surface_is_rejected(tiny, ctx32):
    import torch
    from paper_1810_08860_amd import lf
    out = torch.zeros(16 * 16 * 3, dtype=torch.float32, device="cuda")
    with pytest.raises(lf.LFError) as ei:
        lf.lf_render(ctx32, [(np.array([0.5, 0.0, 0.0]), np.eye(3))], 90.0, (16, 16), out)
    assert ei.value.code == lf.LF_EINVAL and "disk plane" in str(ei.value)
    with pytest.raises(lf.LFError):
        lf.lf_render(ctx32, [(np.zeros(3), np.eye(3) * 1.01)], 90.0, (16, 16), out)
    with pytest.raises(lf.LFError):
        lf.lf_set_tune(ctx32, 12, 8)
