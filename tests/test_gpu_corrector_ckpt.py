"""Checkpoint and resume of corrector training: a run saved after some steps
(FP32 master parameters, Adam moments and step count from the library, the
crop sampler's generator and the schedule position from the driver) and
resumed in a fresh corrector ends with the same parameters and optimiser
state, bit for bit, as the same run without the interruption."""
import json

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HFOV = 90.0


@pytest.fixture(scope="module")
def frames(tiny):
    from lfcheck import gpu_context
    from paper_1810_08860_amd import corrector
    V = tiny.views
    ctx_rt = gpu_context(V, "rgba16f", "f16")
    ctx_ref = gpu_context(V, "rgba32f", "f32")
    eyes = [(tiny.head_pos[0], tiny.head_rot[0])]
    import lfsynth
    p, R = lfsynth.poses(77, 3, 0.2)
    eyes += [(p[k], R[k]) for k in range(3)]
    fr = corrector.make_frames(ctx_rt, ctx_ref, eyes, HFOV, 160, 144)
    ctx_rt.close()
    ctx_ref.close()
    return fr


def _state_equal(a, b):
    return (a["step"] == b["step"] and all(np.array_equal(a[k], b[k]) for k in ("params", "adam_m", "adam_v")))


def test_resumed_training_matches_uninterrupted_run(frames, tmp_path):
    from paper_1810_08860_amd import corrector, lf
    total, cut = 14, 6
    # uninterrupted
    a = lf.lf_corrector_create(corrector.init_params(3))
    corrector.train(a, frames, steps=total, batch=4, crop=48, seed=11)
    sa = lf.lf_corrector_get_state(a)
    # interrupted after `cut` steps, checkpointed, resumed in a fresh corrector
    b = lf.lf_corrector_create(corrector.init_params(3))
    st = corrector.TrainState(11, total)
    corrector.train(b, frames, steps=cut, batch=4, crop=48, state=st)
    assert st.it == cut and lf.lf_corrector_get_state(b)["step"] == cut
    path = str(tmp_path / "ckpt.npz")
    corrector.save_checkpoint(b, st, path)
    b.close()
    c = lf.lf_corrector_create(None)
    st2 = corrector.load_checkpoint(c, path)
    assert st2.it == cut and st2.total == total
    corrector.train(c, frames, steps=total, batch=4, crop=48, state=st2)
    sc = lf.lf_corrector_get_state(c)
    assert sc["step"] == total and st2.it == total
    assert _state_equal(sa, sc)
    # and the run moved: the state differs from the one at the cut
    assert not np.array_equal(sa["params"], np.load(path)["params"])
    # resuming with the parameters only (set_params resets Adam's moments and
    # step) does not reproduce the run: the optimiser state matters
    d = lf.lf_corrector_create(None)
    with np.load(path) as z:
        lf.lf_corrector_set_params(d, z["params"])
        st3 = corrector.TrainState(total=total)
        st3.it = cut
        st3.rng.bit_generator.state = json.loads(str(z["rng"]))
    corrector.train(d, frames, steps=total, batch=4, crop=48, state=st3)
    assert not np.array_equal(lf.lf_corrector_get_state(d)["params"], sa["params"])
    for x in (a, c, d):
        x.close()


def test_set_state_rejects_bad_values():
    from paper_1810_08860_amd import lf
    c = lf.lf_corrector_create(None)
    s = lf.lf_corrector_get_state(c)
    bad = s["adam_v"].copy()
    bad[5] = -1.0
    with pytest.raises(lf.LFError):
        lf.lf_corrector_set_state(c, s["params"], s["adam_m"], bad, 0)
    with pytest.raises(lf.LFError):
        lf.lf_corrector_set_state(c, s["params"], s["adam_m"], s["adam_v"], -1)
    nan = s["params"].copy()
    nan[0] = np.nan
    with pytest.raises(lf.LFError):
        lf.lf_corrector_set_state(c, nan, s["adam_m"], s["adam_v"], 0)
    c.close()
