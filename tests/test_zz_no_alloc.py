"""The allocation-free render entry point (lf_render_noalloc), called through
the C ABI: its per-launch scratch lives in the library's fixed device array,
and its images equal lf_render's bit for bit (colour, weight sum, view count)
on consecutive calls, the second with a smaller input (the array keeps the
first call's contents). Launches beyond the array's 16 MiB are rejected
before anything runs."""
import ctypes

import numpy as np
import pytest

import lfsynth
from lfcheck import gpu_context

pytestmark = pytest.mark.gpu


def _eyes(seed, sizes):
    from paper_1810_08860_amd import lf
    p, R = lfsynth.poses(seed, len(sizes), 0.2)
    eyes, res = [], []
    for k, (w, h) in enumerate(sizes):
        for e in lf.lf_stereo_eyes(p[k], R[k], 0.064):
            eyes.append((np.array(e.pos), np.array(e.rot).reshape(3, 3)))
            res.append((w, h))
    return eyes, np.array(res, np.int32)


def _outputs(res, fill):
    import torch
    npx = int((res[:, 0].astype(np.int64) * res[:, 1]).sum())
    return (torch.full((npx * 3,), fill, dtype=torch.float32, device="cuda"),
            torch.full((npx,), fill, dtype=torch.float32, device="cuda"),
            torch.full((npx,), 201, dtype=torch.uint8, device="cuda"))


def _noalloc_raw(ctx, eyes, hfov, res, outs):
    """Direct ctypes call of the C entry point (no binding logic in between)."""
    import torch
    from paper_1810_08860_amd import lf
    e = lf.make_eyes(eyes)
    r = np.ascontiguousarray(res, np.int32)
    rc = lf.lib().lf_render_noalloc(ctx.handle, e, len(e), ctypes.c_double(hfov), r.ctypes.data,
                                    outs[0].data_ptr(), outs[1].data_ptr(), outs[2].data_ptr(),
                                    torch.cuda.current_stream().cuda_stream)
    return rc


@pytest.fixture(scope="module")
def ctx(tiny):
    c = gpu_context(tiny.views, "rgba16f", "f16")
    yield c
    c.close()


def _check_pair(ctx, eyes, hfov, res):
    import torch
    from paper_1810_08860_amd import lf
    ref = _outputs(res, -3.0)
    lf.lf_render(ctx, eyes, hfov, res, *ref)
    got = _outputs(res, 9.0)
    assert _noalloc_raw(ctx, eyes, hfov, res, got) == lf.LF_OK, lf.lf_last_error()
    torch.cuda.synchronize()
    for a, b in zip(got, ref):
        assert torch.equal(a, b)
    return ref


def test_noalloc_equals_render_on_two_calls_second_smaller(tiny, ctx):
    # first call: 3 stereo poses (6 eyes) of uneven sizes, ragged against the tiles
    eyes, res = _eyes(31, [(200, 176), (120, 136), (1440, 1600)])
    ref = _check_pair(ctx, eyes, tiny.hfov_deg, res)
    assert (ref[1] > 0).float().mean() > 0.9
    # second call, smaller: one stereo pair of 64 x 48
    eyes2, res2 = _eyes(32, [(64, 48)])
    _check_pair(ctx, eyes2, tiny.hfov_deg, res2)
    # and a larger one again after the smaller one (17 eyes: two launches sharing the array in order)
    eyes3, res3 = _eyes(33, [(96, 80)] * 9)
    _check_pair(ctx, eyes3[:17], tiny.hfov_deg, res3[:17])


def test_noalloc_full_size_stereo_pair(tiny, ctx):
    """The largest per-eye size of the mixed batch (2160 x 2160), both eyes in
    one launch (about 9 MiB of scratch over the tiny field's 64 views)."""
    eyes, res = _eyes(34, [(2160, 2160)])
    _check_pair(ctx, eyes, tiny.hfov_deg, res)


def test_noalloc_rejects_launches_beyond_its_scratch(tiny, ctx):
    import torch
    from paper_1810_08860_amd import lf
    # 4 eyes of 4096 x 4096: 262,144 tiles of 260 bytes = 65 MiB in one launch
    eyes, res = _eyes(35, [(4096, 4096)] * 2)
    outs = _outputs(res, 5.0)
    rc = _noalloc_raw(ctx, eyes, tiny.hfov_deg, res, outs)
    assert rc == lf.LF_EINVAL
    assert "scratch" in lf.lf_last_error()
    torch.cuda.synchronize()
    assert bool((outs[0] == 5.0).all())  # nothing was launched
