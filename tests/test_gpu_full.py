"""GPU parity at the full workload size (1024 views of 1024^2, 256^2 depth,
stereo 2 x 1440x1600 eyes at 100 deg), in the launch configuration the
benchmark times, on sampled pixels the oracle computes one by one."""
import numpy as np
import pytest

import oracle
from lfcheck import MAX_UNSTABLE, check_eye, gpu_context, gpu_render, unstable_mask

pytestmark = pytest.mark.gpu

W, H, HFOV, IPD = 1440, 1600, 100.0, 0.064


@pytest.fixture(scope="module")
def full():
    import lfsynth
    return lfsynth.make_workload("full", seed=0, n_poses=8)


@pytest.fixture(scope="module")
def full_oracle(full):
    return oracle.OracleViews.from_views(full.views)


def _sample(n, seed):
    return np.sort(np.random.default_rng(seed).choice(W * H, n, replace=False))


def test_full_size_fp32_sampled_parity(full, full_oracle):
    from paper_1810_08860_amd import lf
    ctx = gpu_context(full.views, "rgba32f", "f32")
    for k in range(3):
        eyes = lf.lf_stereo_eyes(full.head_pos[k], full.head_rot[k], IPD)
        pairs = [(np.array(e.pos), np.array(e.rot).reshape(3, 3)) for e in eyes]
        outs = gpu_render(ctx, pairs, HFOV, [(W, H), (W, H)])
        for e, ((pos, rot), got) in enumerate(zip(pairs, outs)):
            s = check_eye(full_oracle, ctx, pos, rot, HFOV, W, H, idx=_sample(1500, 10 * k + e), gpu=got,
                          lists=(k == 0))
            print(f"pose {k} eye {e}:", s)
    ctx.close()


@pytest.mark.parametrize("img,geo,tol", [("rgba16f", "f16", 2.0 / 255), ("rgba8", "f16", 2.0 / 255),
                                         ("rgba8", "f32", 2.0 / 255), ("rgba16f", "u16", 2.0 / 255),
                                         ("rgba8", "u16", 1e-3)])
def test_full_size_compact_storage_error(full, full_oracle, img, geo, tol):
    """Compact storage against the FP64 oracle: max abs error <= 2/255 on
    stable pixels (reported with the all-pixel maximum and PSNR); RGBA8
    images with 16-bit inverse-depth codes within 1e-3 (the bound of
    test_storage_formats)."""
    from paper_1810_08860_amd import lf
    ctx = gpu_context(full.views, img, geo)
    errs, sq = [], []
    for k in range(4):
        eyes = lf.lf_stereo_eyes(full.head_pos[k], full.head_rot[k], IPD)
        pairs = [(np.array(e.pos), np.array(e.rot).reshape(3, 3)) for e in eyes]
        outs = gpu_render(ctx, pairs, HFOV, [(W, H), (W, H)], want_aux=False)
        for e, ((pos, rot), got) in enumerate(zip(pairs, outs)):
            idx = _sample(1000, 100 + 10 * k + e)
            ref = oracle.render(full_oracle, pos, rot, HFOV, W, H, idx)["rgb"]
            unst = unstable_mask(full_oracle, pos, rot, HFOV, W, H, idx, ref)
            err = np.abs(got[0][idx] - ref).max(1)
            errs.append((err[~unst].max(), err.max(), unst.mean()))
            sq.append(((got[0][idx] - ref) ** 2).mean())
            assert unst.sum() <= max(2, MAX_UNSTABLE * len(idx))
    stable_max = max(x[0] for x in errs)
    psnr = 10 * np.log10(1.0 / max(np.mean(sq), 1e-30))
    print(f"{img}/{geo}: max err stable {stable_max:.4g} (2/255 = {2 / 255:.4g}), "
          f"all {max(x[1] for x in errs):.4g}, PSNR {psnr:.1f} dB, unstable {[round(x[2] * 100, 3) for x in errs]} %")
    assert stable_max <= tol
    ctx.close()
