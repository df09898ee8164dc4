"""The corrector trained on pairs the method itself generates (real-time FP16
render vs offline reference: 4x4 sub-pixel rays, disks of twice the radius)
on the full-size light field, then evaluated on held-out poses: it must beat
the plain render against the reference."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

W, H, HFOV, IPD = 1440, 1600, 100.0, 0.064


def test_corrector_gains_psnr_on_held_out_poses():
    import lfsynth
    from lfcheck import gpu_context
    from paper_1810_08860_amd import corrector, lf

    V = lfsynth.make_views(1024, 1024, 256, 12, seed=0)
    ctx_rt = gpu_context(V, "rgba16f", "f16")
    ctx_ref = gpu_context(V, "rgba32f", "f32")

    def eyes(seed, n):
        p, R = lfsynth.poses(seed, n, 0.25)
        out = []
        for k in range(n):
            out += [(np.array(e.pos), np.array(e.rot).reshape(3, 3)) for e in lf.lf_stereo_eyes(p[k], R[k], IPD)]
        return out

    train_frames = corrector.make_frames(ctx_rt, ctx_ref, eyes(500, 8), HFOV, W, H)
    test_frames = corrector.make_frames(ctx_rt, ctx_ref, eyes(900, 2), HFOV, W, H)
    corr = lf.lf_corrector_create(corrector.init_params(0))
    before = corrector.evaluate(corr, test_frames)
    log = corrector.train(corr, train_frames, steps=500, batch=16, crop=96, seed=1)
    after = corrector.evaluate(corr, test_frames)
    print("loss log:", [(s, round(v, 7)) for s, v in log])
    print("before:", before)
    print("after:", after)
    assert log[-1][1] < log[0][1]
    assert after["psnr_gain_db"] > 0.2
    # threshold 0 is the plain render
    assert corrector.evaluate(corr, test_frames[:1], thresh=0.0)["psnr_gain_db"] == 0.0
    corr.close()
    ctx_rt.close()
    ctx_ref.close()
