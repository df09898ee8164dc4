"""Training and evaluation driver of the learned residual corrector.

The corrector (include/lf.h, lf_corrector_*) refines the real-time render
towards an offline reference of the same pose: the same disk-blended query
with 4x4 sub-pixel rays and disks of twice the radius over all views (the
analogue of the high-quality offline query of Sec. 5.1 of the paper). Pairs
are produced on the GPU by the library itself; this module only orchestrates
them (pose selection, crop gathering, learning-rate schedule) and measures
PSNR. Every forward, backward and optimiser step runs in the library's kernels.
"""
from __future__ import annotations

import json
import math
from dataclasses import dataclass

import numpy as np

from . import lf

LAYERS = ((5, 32), (32, 32), (32, 32), (32, 3))


def init_params(seed: int, last_scale: float = 0.1) -> np.ndarray:
    """He-normal convolution weights (the last layer scaled down so the first
    residual is small), zero biases; the flat layout of lf_corrector_create."""
    rng = np.random.default_rng(seed)
    out = []
    for li, (ci, co) in enumerate(LAYERS):
        w = rng.normal(size=9 * ci * co) * math.sqrt(2.0 / (9 * ci))
        if li == len(LAYERS) - 1:
            w *= last_scale
        out += [w, np.zeros(co)]
    p = np.concatenate(out).astype(np.float32)
    assert p.size == lf.CORRECTOR_PARAMS
    return p


@dataclass
class Frame:
    rgb: object      # (H, W, 3) FP32 device tensor: real-time render
    wsum: object     # (H, W) FP32: disk-weight sum
    count: object    # (H, W) u8: contributing views
    ref: object      # (H, W, 3) FP32: offline reference


def make_frames(ctx_rt, ctx_ref, eyes, hfov, W, H, ss=4, disk_scale=2.0):
    """Render each eye with the real-time path (colour, W, n) and the offline
    reference; returns a list of Frame on the device."""
    import torch
    frames = []
    for eye in eyes:
        rgb = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
        ws = torch.empty((H, W), dtype=torch.float32, device="cuda")
        cnt = torch.empty((H, W), dtype=torch.uint8, device="cuda")
        ref = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
        lf.lf_render(ctx_rt, [eye], hfov, (W, H), rgb, ws, cnt)
        lf.lf_render_reference(ctx_ref, [eye], hfov, (W, H), ss, disk_scale, ref)
        frames.append(Frame(rgb, ws, cnt, ref))
    torch.cuda.synchronize()
    return frames


class TrainState:
    """Where a training run stands: the crop sampler's generator and the next
    step of the schedule (the optimiser state lives in the corrector)."""

    def __init__(self, seed: int = 0, total: int = 0):
        self.rng = np.random.default_rng(seed)
        self.it = 0
        self.total = total


def save_checkpoint(corr, state: TrainState, path: str):
    """Everything a resumed run needs to continue bit for bit: the FP32 master
    parameters, Adam's moments and step count (from the library), the crop
    sampler's generator state and the schedule position. A plain .npz (no
    pickled objects)."""
    st = lf.lf_corrector_get_state(corr)
    np.savez(path, params=st["params"], adam_m=st["adam_m"], adam_v=st["adam_v"],
             step=np.int64(st["step"]), it=np.int64(state.it), total=np.int64(state.total),
             rng=np.array(json.dumps(state.rng.bit_generator.state)))


def load_checkpoint(corr, path: str) -> TrainState:
    """Restore a checkpoint written by save_checkpoint into corr; returns the
    training state to pass to train()."""
    with np.load(path, allow_pickle=False) as z:
        lf.lf_corrector_set_state(corr, z["params"], z["adam_m"], z["adam_v"], int(z["step"]))
        state = TrainState(total=int(z["total"]))
        state.it = int(z["it"])
        state.rng.bit_generator.state = json.loads(str(z["rng"]))
    return state


def train(corr, frames, steps, batch=16, crop=96, lr=2e-3, lr_end=2e-4, seed=0, log_every=100, state=None):
    """Adam on random crops of the frames with a cosine learning-rate decay
    over `steps` steps. With a TrainState (fresh, or from load_checkpoint) the
    run takes up to `steps` further steps of that schedule from where the
    state stands (its total fixes the schedule) and leaves the state at the
    step reached. Returns [(step, loss)] at every log_every steps and at the
    end."""
    import torch
    if state is None:
        state = TrainState(seed, steps)
    if state.total == 0:
        state.total = steps
    rng = state.rng
    H, W = frames[0].rgb.shape[:2]
    c_rgb = torch.empty((batch, crop, crop, 3), dtype=torch.float32, device="cuda")
    c_ws = torch.empty((batch, crop, crop), dtype=torch.float32, device="cuda")
    c_cnt = torch.empty((batch, crop, crop), dtype=torch.uint8, device="cuda")
    c_ref = torch.empty((batch, crop, crop, 3), dtype=torch.float32, device="cuda")
    log = []
    last = min(state.total, state.it + steps)
    for it in range(state.it, last):
        for b in range(batch):
            f = frames[rng.integers(len(frames))]
            y = int(rng.integers(0, H - crop + 1))
            x = int(rng.integers(0, W - crop + 1))
            c_rgb[b].copy_(f.rgb[y:y + crop, x:x + crop])
            c_ws[b].copy_(f.wsum[y:y + crop, x:x + crop])
            c_cnt[b].copy_(f.count[y:y + crop, x:x + crop])
            c_ref[b].copy_(f.ref[y:y + crop, x:x + crop])
        t = it / max(state.total - 1, 1)
        lr_t = lr_end + 0.5 * (lr - lr_end) * (1.0 + math.cos(math.pi * t))
        want = (it % log_every == 0) or it == last - 1
        loss, _ = lf.lf_corrector_train_step(corr, c_rgb, c_ws, c_cnt, c_ref, batch, crop, crop, lr_t,
                                             want_loss=want)
        if want:
            log.append((it, loss))
        state.it = it + 1
    return log


def psnr(a, b) -> float:
    mse = float(((a.double() - b.double()) ** 2).mean())
    return 10.0 * math.log10(1.0 / max(mse, 1e-20))


def evaluate(corr, frames, thresh=8.0 / 255.0):
    """PSNR of the plain render and of the corrected render against the
    reference, the largest errors and the fraction of pixels that fell back."""
    import torch
    res = {"psnr_plain": [], "psnr_corrected": [], "max_err_plain": [], "max_err_corrected": [],
           "fallback_frac": []}
    for f in frames:
        H, W = f.rgb.shape[:2]
        out = torch.empty_like(f.rgb)
        fb = torch.empty((H, W), dtype=torch.uint8, device="cuda")
        lf.lf_corrector_apply(corr, f.rgb, f.wsum, f.count, 1, W, H, thresh, out, fb)
        torch.cuda.synchronize()
        res["psnr_plain"].append(psnr(f.rgb, f.ref))
        res["psnr_corrected"].append(psnr(out, f.ref))
        res["max_err_plain"].append(float((f.rgb - f.ref).abs().max()))
        res["max_err_corrected"].append(float((out - f.ref).abs().max()))
        res["fallback_frac"].append(float(fb.float().mean()))
    summary = {k: float(np.mean(v)) for k, v in res.items()}
    summary["psnr_gain_db"] = summary["psnr_corrected"] - summary["psnr_plain"]
    return summary
