"""Learned residual corrector: MFMA forward and backward kernels against the
FP64 conv oracle, fallback rule, and training through the C ABI.

The GPU keeps weights and activations in BF16 (FP32 accumulation); the oracle
is evaluated in FP64 on the BF16-rounded parameters and inputs, so the only
remaining differences are the BF16 roundings of the hidden activations and
layer gradients (relative 2^-9 each)."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

N, H, W = 2, 28, 40  # ragged against the 16 x 8 conv tiles


def bf16_round(a):
    a = np.ascontiguousarray(a, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32)


def _params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    out = []
    for ci, co, _ in oracle.CORRECTOR_LAYERS:
        out.append(rng.normal(size=9 * ci * co) * scale * np.sqrt(2.0 / (9 * ci)))
        out.append(rng.normal(size=co) * 0.05)
    return np.concatenate(out).astype(np.float32)


def _images(seed):
    rng = np.random.default_rng(seed)
    rgb = rng.uniform(0, 1, (N, H, W, 3)).astype(np.float32)
    ws = rng.uniform(0, 3, (N, H, W)).astype(np.float32)
    cnt = rng.integers(0, 10, (N, H, W)).astype(np.uint8)
    ref = np.clip(rgb + rng.normal(size=rgb.shape) * 0.05, 0, 1).astype(np.float32)
    return rgb, ws, cnt, ref


def _dev(*arrs):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrs]


def _oracle_inputs(rgb, ws, cnt):
    """Input as the kernels see it: every channel rounded to BF16."""
    x = oracle.corrector_input(rgb, ws, cnt)
    return bf16_round(x).astype(np.float64)


def test_forward_matches_oracle():
    import torch
    from paper_1810_08860_amd import lf
    prm = _params(1)
    rgb, ws, cnt, _ = _images(2)
    c = lf.lf_corrector_create(prm)
    d_rgb, d_ws, d_cnt = _dev(rgb, ws, cnt)
    out = torch.zeros_like(d_rgb)
    resid = torch.zeros_like(d_rgb)
    lf.lf_corrector_apply(c, d_rgb, d_ws, d_cnt, N, W, H, float("inf"), out, None, resid)
    torch.cuda.synchronize()
    got = resid.cpu().numpy().astype(np.float64)
    want, _ = oracle.corrector_forward(bf16_round(prm).astype(np.float64), _oracle_inputs(rgb, ws, cnt))
    rel = np.linalg.norm(got - want) / np.linalg.norm(want)
    print(f"forward: relative L2 {rel:.3g}, max abs {np.abs(got - want).max():.3g}, scale {np.abs(want).max():.3g}")
    assert rel < 1e-2
    assert np.allclose(out.cpu().numpy(), rgb + got, atol=1e-6)
    c.close()


@pytest.mark.parametrize("shape", [(2, 28, 40), (1, 97, 161), (2, 392, 584)])
def test_fused_inference_matches_training_forward(shape):
    """Inference runs all four layers in one fused kernel over 16 x 16 tiles
    with LDS halos; training runs them layer by layer. The training step's
    loss (from its own forward) must equal the MSE of the fused residual
    against the same reference, up to the summation order of the loss, so a
    tile left out or computed twice shows. The last shape (1,850 ragged
    tiles) has more tiles than resident workgroups, a grid that is a multiple
    of 8, so each XCD takes its own range of tiles, and ranges of unequal
    length."""
    import torch
    from paper_1810_08860_amd import lf
    n, h, w = shape
    prm = _params(11)
    rng = np.random.default_rng(12)
    rgb = rng.uniform(0, 1, (n, h, w, 3)).astype(np.float32)
    ws = rng.uniform(0, 3, (n, h, w)).astype(np.float32)
    cnt = rng.integers(0, 10, (n, h, w)).astype(np.uint8)
    ref = np.clip(rgb + rng.normal(size=rgb.shape) * 0.05, 0, 1).astype(np.float32)
    c = lf.lf_corrector_create(prm)
    d_rgb, d_ws, d_cnt, d_ref = _dev(rgb, ws, cnt, ref)
    out = torch.zeros_like(d_rgb)
    resid = torch.zeros_like(d_rgb)
    lf.lf_corrector_apply(c, d_rgb, d_ws, d_cnt, n, w, h, float("inf"), out, None, resid)
    torch.cuda.synchronize()
    r = resid.cpu().numpy().astype(np.float64)
    mse_fused = float(np.mean((rgb.astype(np.float64) + r - ref) ** 2))
    loss, _ = lf.lf_corrector_train_step(c, d_rgb, d_ws, d_cnt, d_ref, n, w, h, 0.0)
    print(f"{shape}: train-step loss {loss:.9g}, fused MSE {mse_fused:.9g}")
    assert abs(loss - mse_fused) <= 1e-5 * mse_fused
    c.close()


def test_fused_inference_many_tiles_per_workgroup():
    """An image with several times more 16 x 16 tiles than the fused kernel
    has resident workgroups, so every workgroup runs several tiles and reads
    each next tile's input while the current one computes. Windows at the
    corners and inside are checked against the FP64 oracle on crops grown by
    the network's 4-pixel reach (cut at the image edge, where the oracle's
    zero padding is the image's)."""
    import torch
    from paper_1810_08860_amd import lf
    n, h, w = 2, 392, 584  # 25 x 37 tiles per image, ragged in both directions
    prm = _params(21)
    rng = np.random.default_rng(22)
    rgb = rng.uniform(0, 1, (n, h, w, 3)).astype(np.float32)
    ws = rng.uniform(0, 3, (n, h, w)).astype(np.float32)
    cnt = rng.integers(0, 10, (n, h, w)).astype(np.uint8)
    c = lf.lf_corrector_create(prm)
    d_rgb, d_ws, d_cnt = _dev(rgb, ws, cnt)
    resid = torch.zeros_like(d_rgb)
    out = torch.zeros_like(d_rgb)
    lf.lf_corrector_apply(c, d_rgb, d_ws, d_cnt, n, w, h, float("inf"), out, None, resid)
    torch.cuda.synchronize()
    got = resid.cpu().numpy().astype(np.float64)
    c.close()
    p64 = bf16_round(prm).astype(np.float64)
    wins = [(0, 0, 0), (1, h - 20, w - 20), (0, 0, w - 20), (1, h - 20, 0)]
    wins += [(int(rng.integers(n)), int(rng.integers(h - 20)), int(rng.integers(w - 20))) for _ in range(6)]
    for k, y0, x0 in wins:
        ya, yb, xa, xb = max(0, y0 - 4), min(h, y0 + 24), max(0, x0 - 4), min(w, x0 + 24)
        x = _oracle_inputs(rgb[k:k + 1, ya:yb, xa:xb], ws[k:k + 1, ya:yb, xa:xb], cnt[k:k + 1, ya:yb, xa:xb])
        want = oracle.corrector_forward(p64, x)[0][0, y0 - ya:y0 - ya + 20, x0 - xa:x0 - xa + 20]
        g = got[k, y0:y0 + 20, x0:x0 + 20]
        rel = np.linalg.norm(g - want) / np.linalg.norm(want)
        print(f"window image {k} at ({y0}, {x0}): relative L2 {rel:.3g}")
        assert rel < 1e-2


def test_fallback_threshold_rule():
    import torch
    from paper_1810_08860_amd import lf
    prm = _params(3)
    rgb, ws, cnt, _ = _images(4)
    c = lf.lf_corrector_create(prm)
    d_rgb, d_ws, d_cnt = _dev(rgb, ws, cnt)
    out = torch.zeros_like(d_rgb)
    fb = torch.zeros((N, H, W), dtype=torch.uint8, device="cuda")
    resid = torch.zeros_like(d_rgb)
    lf.lf_corrector_apply(c, d_rgb, d_ws, d_cnt, N, W, H, 0.0, out, fb, resid)
    torch.cuda.synchronize()
    assert torch.equal(out, d_rgb) and bool((fb == 1).all())  # threshold 0: the plain render, bit for bit
    r = resid.cpu().numpy()
    t = float(np.median(np.abs(r).max(-1)))
    lf.lf_corrector_apply(c, d_rgb, d_ws, d_cnt, N, W, H, t, out, fb, resid)
    torch.cuda.synchronize()
    f = fb.cpu().numpy().astype(bool)
    o = out.cpu().numpy()
    assert np.array_equal(f, np.abs(r).max(-1) > t) and 0 < f.sum() < f.size
    assert np.array_equal(o[f], rgb[f]) and np.allclose(o[~f], (rgb + r)[~f], atol=1e-6)
    c.close()


def test_gradients_match_oracle():
    from paper_1810_08860_amd import lf
    prm = _params(5)
    rgb, ws, cnt, ref = _images(6)
    c = lf.lf_corrector_create(prm)
    d_rgb, d_ws, d_cnt, d_ref = _dev(rgb, ws, cnt, ref)
    loss, g = lf.lf_corrector_train_step(c, d_rgb, d_ws, d_cnt, d_ref, N, W, H, 0.0, want_grad=True)
    p64 = bf16_round(prm).astype(np.float64)
    x = _oracle_inputs(rgb, ws, cnt)
    loss_o, g_o = oracle.corrector_loss_grad(p64, x, rgb.astype(np.float64), ref.astype(np.float64))
    print(f"loss gpu {loss:.6g} oracle {loss_o:.6g}")
    assert abs(loss - loss_o) <= 5e-3 * loss_o
    off = 0
    for li, (ci, co, _) in enumerate(oracle.CORRECTOR_LAYERS):
        for part, n in (("w", 9 * ci * co), ("b", co)):
            a, b = g[off:off + n].astype(np.float64), g_o[off:off + n]
            cos = a @ b / (np.linalg.norm(a) * np.linalg.norm(b))
            rel = np.linalg.norm(a - b) / np.linalg.norm(b)
            # element by element: each gradient sums products of BF16 activations
            # and BF16 upstream gradients (relative rounding 2^-9 each), so an
            # element stays within a few 2^-8 of the layer's largest gradient;
            # 2 % of it catches a single wrong element the cosine would hide
            elem = np.abs(a - b).max() / np.abs(b).max()
            print(f"layer {li} {part}: cosine {cos:.6f}, relative L2 {rel:.3g}, "
                  f"max element error / max |grad| {elem:.3g}")
            assert cos > 0.9999 and rel < 1e-2, (li, part, cos, rel)
            assert elem < 2e-2, (li, part, elem)
            off += n
    # lr = 0 leaves the parameters alone
    p_after, step = lf.lf_corrector_get_params(c)
    assert step == 0 and np.array_equal(p_after, prm)
    c.close()


def test_training_reduces_loss():
    """A learnable target: ref = render + a fixed smooth function of (R, G, B).
    Adam steps through the C ABI must drive the loss well down."""
    import torch
    from paper_1810_08860_amd import lf
    rng = np.random.default_rng(7)
    n, h, w = 8, 32, 48
    rgb = rng.uniform(0, 1, (n, h, w, 3)).astype(np.float32)
    ws = np.full((n, h, w), 2.0, np.float32)
    cnt = np.full((n, h, w), 6, np.uint8)
    ref = (rgb + 0.05 * np.stack([rgb[..., 1] - rgb[..., 2], rgb[..., 2] - rgb[..., 0],
                                  rgb[..., 0] - rgb[..., 1]], -1)).astype(np.float32)
    c = lf.lf_corrector_create(_params(8, 0.5))
    d = _dev(rgb, ws, cnt, ref)
    losses = []
    for it in range(300):
        loss, _ = lf.lf_corrector_train_step(c, *d, n, w, h, 2e-3, want_loss=(it % 50 == 0 or it == 299))
        if loss is not None:
            losses.append(loss)
    print("losses:", [round(v, 6) for v in losses])
    _, step = lf.lf_corrector_get_params(c)
    assert step == 300
    assert losses[-1] < 0.2 * losses[0]
    torch.cuda.synchronize()
    c.close()
