"""The corrector trained on pairs the method itself generates (real-time FP16
render vs offline reference: 4x4 sub-pixel rays, disks of twice the radius)
from three seeded scenes, then evaluated on held-out poses of a training
scene and on a fourth scene it never saw: it must beat the plain render
against the reference on both. Reduced size (1024 views of 512^2, eyes of
720 x 800) so the test runs in seconds; the bench runs the full size."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

W, H, HFOV, IPD = 720, 800, 100.0, 0.064


def test_corrector_gains_psnr_on_held_out_scene_and_poses():
    import lfsynth
    from lfcheck import gpu_context
    from paper_1810_08860_amd import corrector, lf

    def eyes(seed, n):
        p, R = lfsynth.poses(seed, n, 0.25)
        out = []
        for k in range(n):
            out += [(np.array(e.pos), np.array(e.rot).reshape(3, 3)) for e in lf.lf_stereo_eyes(p[k], R[k], IPD)]
        return out

    def frames(scene, pose_seed, n_poses):
        V = lfsynth.make_views(1024, 512, 256, 12, seed=scene)
        rt = gpu_context(V, "rgba16f", "f32")
        ref = gpu_context(V, "rgba32f", "f32")
        fr = corrector.make_frames(rt, ref, eyes(pose_seed, n_poses), HFOV, W, H)
        rt.close()
        ref.close()
        return fr

    train = []
    for scene in (0, 1, 2):
        train += frames(scene, 500 + scene, 4)
    held_poses = frames(0, 900, 2)
    held_scene = frames(3, 950, 2)
    corr = lf.lf_corrector_create(corrector.init_params(0))
    before = corrector.evaluate(corr, held_scene)
    log = corrector.train(corr, train, steps=500, batch=16, crop=96, seed=1, log_every=100)
    poses = corrector.evaluate(corr, held_poses)
    scene = corrector.evaluate(corr, held_scene)
    print("loss log:", [(s, round(v, 7)) for s, v in log])
    print("held-out scene before training:", before)
    print("held-out poses of scene 0:", poses)
    print("held-out scene 3:", scene)
    assert log[-1][1] < log[0][1]
    assert poses["psnr_gain_db"] > 0.25
    assert scene["psnr_gain_db"] > 0.25
    # threshold 0 is the plain render
    assert corrector.evaluate(corr, held_scene[:1], thresh=0.0)["psnr_gain_db"] == 0.0
    corr.close()
