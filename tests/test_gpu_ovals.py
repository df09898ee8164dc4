"""Asymmetric oval disks (Sec. 4.4) on the GPU against the FP64 oracle.

Both sides take the same per-view extents (e+u, e-u, e+v, e-v) as input, so
the render parity does not depend on how a triangulation breaks ties; the
library's own extents are checked against the oracle's on the CPU. Parity
criteria as for circular disks: candidate and contributing sets equal outside
the ill-conditioned bands, colours within 1e-4 on stable pixels."""
import numpy as np
import pytest

import oracle
from lfcheck import check_reference, check_eye, gpu_context, gpu_render

pytestmark = pytest.mark.gpu

W, H, HFOV, IPD = 1440, 1600, 100.0, 0.064


@pytest.fixture(scope="module")
def full():
    import lfsynth
    return lfsynth.make_workload("full", seed=0, n_poses=8)


@pytest.fixture(scope="module")
def full_ext(full):
    from paper_1810_08860_amd import lf
    return lf.lf_disk_extents(full.views.centres, full.views.rot)


def test_tiny_full_frame_oval_parity(tiny, tiny_oracle):
    from paper_1810_08860_amd import lf
    V = tiny.views
    ext = lf.lf_disk_extents(V.centres, V.rot)
    ov = tiny_oracle.with_disk_extents(ext)
    ctx = gpu_context(V, disk_ext=ext)
    import lfsynth
    p2, R2 = lfsynth.poses(77, 1, 0.2)
    for k, (pos, rot) in enumerate([(tiny.head_pos[0], tiny.head_rot[0]), (p2[0], R2[0])]):
        s = check_eye(ov, ctx, pos, rot, tiny.hfov_deg, 256, 256)
        print(f"pose {k}:", s)
    ctx.close()


def test_full_size_oval_sampled_parity(full, full_ext):
    from paper_1810_08860_amd import lf
    ov = oracle.OracleViews.from_views(full.views, disk_ext=full_ext)
    ctx = gpu_context(full.views, disk_ext=full_ext)
    for k in range(2):
        eyes = lf.lf_stereo_eyes(full.head_pos[k], full.head_rot[k], IPD)
        pairs = [(np.array(e.pos), np.array(e.rot).reshape(3, 3)) for e in eyes]
        outs = gpu_render(ctx, pairs, HFOV, [(W, H), (W, H)])
        for e, ((pos, rot), got) in enumerate(zip(pairs, outs)):
            idx = np.sort(np.random.default_rng(50 + 10 * k + e).choice(W * H, 1500, replace=False))
            s = check_eye(ov, ctx, pos, rot, HFOV, W, H, idx=idx, gpu=got, lists=(k == 0))
            print(f"pose {k} eye {e}:", s)
    ctx.close()


def test_oval_batch_matches_per_eye_render(tiny):
    import torch
    from paper_1810_08860_amd import lf
    V = tiny.views
    ext = lf.lf_disk_extents(V.centres, V.rot)
    ctx = gpu_context(V, "rgba16f", "f16", disk_ext=ext)
    import lfsynth
    p, R = lfsynth.poses(78, 4, 0.2)
    eyes = [(p[k], R[k]) for k in range(4)]
    res = [(120, 136), (200, 176), (64, 64), (96, 80)]
    outs = []
    for (pp, rr), (w, h) in zip(eyes, res):
        o = torch.zeros(w * h * 3, dtype=torch.float32, device="cuda")
        lf.lf_render(ctx, [(pp, rr)], 90.0, (w, h), o)
        outs.append(o)
    ref = torch.cat(outs)
    got = torch.full_like(ref, -5.0)
    lf.lf_render_batch(ctx, eyes, 90.0, np.array(res, np.int32), got)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
    ctx.close()


def test_ovals_tighten_candidate_lists(full, full_ext):
    """Work counters of one stereo frame with circles (R = 1.5 x mean
    nearest-neighbour spacing) and with the Delaunay ovals; and the share of
    pixels no disk covers."""
    import torch
    from paper_1810_08860_amd import lf
    eyes = lf.lf_stereo_eyes(full.head_pos[0], full.head_rot[0], IPD)
    res = np.array([[W, H]] * 2, np.int32)
    out = {}
    for name, ext in (("circle", None), ("oval", full_ext)):
        ctx = gpu_context(full.views, "rgba16f", "f16", disk_ext=ext)
        st = lf.lf_render_stats(ctx, eyes, HFOV, res)
        ws = torch.empty(2 * W * H, dtype=torch.float32, device="cuda")
        rgb = torch.empty(2 * W * H * 3, dtype=torch.float32, device="cuda")
        lf.lf_render(ctx, eyes, HFOV, res, rgb, ws)
        torch.cuda.synchronize()
        out[name] = {k: v / st["pixels"] for k, v in st.items() if k != "pixels"}
        out[name]["uncovered"] = float((ws == 0).float().mean())
        ctx.close()
    print(out)
    assert out["oval"]["candidates"] < out["circle"]["candidates"]
    assert out["oval"]["uncovered"] < 1e-2


def test_oval_reference_render_scales_extents(tiny, tiny_oracle):
    """The offline reference with oval disks grows every extent by the disk
    scale: 3 x 3 sub-pixel rays with extents doubled against the oracle."""
    import torch
    from paper_1810_08860_amd import lf
    V = tiny.views
    ext, _ = oracle.disk_extents(V.centres, V.rot)
    ov = tiny_oracle.with_disk_extents(ext)
    ctx = gpu_context(V, "rgba32f", "f32", disk_ext=ext)
    p, R = tiny.head_pos[0], tiny.head_rot[0]
    Wr = Hr = 64
    out = torch.zeros(Wr * Hr * 3, dtype=torch.float32, device="cuda")
    lf.lf_render_reference(ctx, [(p, R)], 90.0, (Wr, Hr), 3, 2.0, out)
    torch.cuda.synchronize()
    ctx.close()
    got = out.view(-1, 3).cpu().numpy().astype(np.float64)
    check_reference(ov, got, p, R, 90.0, Wr, Hr, np.arange(0, Wr * Hr, 7), 3, 2.0, "oval reference ss=3")
