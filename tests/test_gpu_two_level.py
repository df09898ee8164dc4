"""Two-level progressive rendering (Sec. 7.2) on the GPU: a fine level (all
views, small disks) and a coarse level (every 4th capture again, with disks
sized for its own spacing) in one context; a per-frame view mask says which
views take part. Each case is checked against the FP64 oracle evaluating
Eq. (2) over exactly the enabled views."""
import numpy as np
import pytest

import lfsynth
import oracle
from lfcheck import check_eye, gpu_context, gpu_render

pytestmark = pytest.mark.gpu


class _Views:
    def __init__(self, **kw):
        self.__dict__.update(kw)


@pytest.fixture(scope="module")
def two_level(tiny):
    V = tiny.views
    coarse = np.arange(0, V.n, 4)
    R_f, R_c = V.disk_radius, 1.5 * lfsynth.mean_nn(V.centres[coarse])
    idx = np.concatenate([np.arange(V.n), coarse])
    ext = np.concatenate([np.full((V.n, 4), R_f), np.full((len(coarse), 4), R_c)])
    tl = _Views(centres=V.centres[idx], rot=V.rot[idx], rgba8=V.rgba8[idx], zdepth=V.zdepth[idx],
                src_fov_deg=V.src_fov_deg, disk_radius=R_f)
    ctx = gpu_context(tl, "rgba32f", "f32", disk_ext=ext)
    yield tl, ext, V.n, ctx
    ctx.close()


def _oracle_subset(tl, ext, keep):
    k = np.nonzero(keep)[0]
    return oracle.OracleViews(tl.centres[k], tl.rot[k], tl.rgba8[k], tl.zdepth[k], tl.src_fov_deg,
                              tl.disk_radius, disk_ext=ext[k])


def _mask_rule(tl, ext, n_fine, avail):
    """Reference of the two-level rule: available fine views, plus coarse views
    whose disk reaches the centre of an unavailable fine view."""
    m = np.zeros(len(tl.centres), np.uint8)
    m[:n_fine] = avail
    miss = tl.centres[:n_fine][avail == 0]
    for j in range(n_fine, len(tl.centres)):
        if len(miss) and (np.linalg.norm(miss - tl.centres[j], axis=1) < ext[j, 0]).any():
            m[j] = 1
    return m


@pytest.mark.parametrize("case", ["all_fine", "no_fine", "half", "both_levels"])
def test_two_level_masks_match_oracle(tiny, two_level, case):
    from paper_1810_08860_amd import lf
    tl, ext, n_fine, ctx = two_level
    rng = np.random.default_rng(3)
    if case == "both_levels":
        mask = np.ones(len(tl.centres), np.uint8)
        lf.lf_set_view_mask(ctx, None)
    else:
        avail = {"all_fine": np.ones(n_fine, np.uint8), "no_fine": np.zeros(n_fine, np.uint8),
                 "half": (rng.uniform(size=n_fine) < 0.5).astype(np.uint8)}[case]
        mask = lf.lf_two_level_mask(ctx, n_fine, avail)
        assert np.array_equal(mask, _mask_rule(tl, ext, n_fine, avail))
        lf.lf_set_view_mask(ctx, mask)
    ov = _oracle_subset(tl, ext, mask)
    s = check_eye(ov, ctx, tiny.head_pos[0], tiny.head_rot[0], tiny.hfov_deg, 256, 256,
                  lists=(case == "all_fine"))
    print(case, int(mask[:n_fine].sum()), "fine +", int(mask[n_fine:].sum()), "coarse:", s)
    lf.lf_set_view_mask(ctx, None)


def test_masked_batch_matches_per_eye(tiny, two_level):
    import torch
    from paper_1810_08860_amd import lf
    tl, ext, n_fine, ctx = two_level
    avail = (np.random.default_rng(8).uniform(size=n_fine) < 0.3).astype(np.uint8)
    lf.lf_set_view_mask(ctx, lf.lf_two_level_mask(ctx, n_fine, avail))
    p, R = lfsynth.poses(41, 2, 0.2)
    eyes = []
    for k in range(2):
        eyes += [(np.array(e.pos), np.array(e.rot).reshape(3, 3)) for e in lf.lf_stereo_eyes(p[k], R[k], 0.064)]
    res = [(120, 96)] * len(eyes)
    ref = torch.cat([torch.from_numpy(o[0].astype(np.float32).ravel()) for o in gpu_render(ctx, eyes, 90.0, res)])
    got = torch.full((sum(w * h for w, h in res) * 3,), -5.0, dtype=torch.float32, device="cuda")
    lf.lf_render_batch(ctx, eyes, 90.0, np.array(res, np.int32), got)
    torch.cuda.synchronize()
    lf.lf_set_view_mask(ctx, None)
    assert torch.equal(got.cpu(), ref)
