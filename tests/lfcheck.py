"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI
and compare it with the FP64 oracle under the parity criteria.

Parity criteria (GPU FP32 against oracle FP64):
  * candidate sets (views with rho > 0) identical except for views the oracle
    lists as ill-conditioned (|rho| <= 1e-5 or a grazing disk plane);
  * contributing sets (candidates whose mesh is hit) identical except for those
    and for hits within 1e-6 (normalised image units) of the mesh domain edge;
  * colours within 1e-4 on STABLE pixels. A pixel is unstable when its colour
    is so sensitive to the ray's position that an FP32-sized perturbation of
    the ray (POS_ERR = 1e-5 px) could move it by more than the tolerance:
    measured with a +-1e-3 px jitter of the oracle's ray, unstable means a
    change above 1e-4 * (1e-3 / 1e-5) = 1e-2 (a surface flip, or a hit/miss
    change at a mesh domain edge); unstable pixels must stay below 0.1 % of
    a frame (at most 2 on eyes too small for a fraction to mean anything).
"""
from __future__ import annotations

import numpy as np

import oracle

COLOUR_TOL = 1e-4
JITTER = 1e-3
POS_ERR = 1e-5
MAX_UNSTABLE = 1e-3


def torch_mod():
    import torch
    return torch


def gpu_context(views, img_fmt="rgba32f", geo_fmt="f32", disk_radius=None, disk_ext=None):
    from paper_1810_08860_amd import lf
    return lf.lf_load_views(views.centres, views.rot, views.rgba8, views.zdepth, views.src_fov_deg,
                            views.disk_radius if disk_radius is None else disk_radius, img_fmt=img_fmt,
                            geo_fmt=geo_fmt, disk_ext=disk_ext)


def gpu_render(ctx, eyes, hfov, res, want_aux=True):
    """Render eyes = [(pos, rot), ...] with res = [(W, H), ...]; returns per-eye
    arrays (rgb (H*W,3), wsum (H*W,), count (H*W,))."""
    torch = torch_mod()
    from paper_1810_08860_amd import lf
    res = [tuple(r) for r in res]
    npx = sum(w * h for w, h in res)
    rgb = torch.full((npx * 3,), -7.0, dtype=torch.float32, device="cuda")
    ws = torch.full((npx,), -7.0, dtype=torch.float32, device="cuda") if want_aux else None
    cnt = torch.full((npx,), 77, dtype=torch.uint8, device="cuda") if want_aux else None
    lf.lf_render(ctx, eyes, hfov, np.array(res, np.int32), rgb, ws, cnt)
    torch.cuda.synchronize()
    out, off = [], 0
    rgb_h = rgb.view(-1, 3).cpu().numpy().astype(np.float64)
    ws_h = ws.cpu().numpy().astype(np.float64) if want_aux else None
    cnt_h = cnt.cpu().numpy().astype(np.int32) if want_aux else None
    for w, h in res:
        sl = slice(off, off + w * h)
        out.append((rgb_h[sl], ws_h[sl] if want_aux else None, cnt_h[sl] if want_aux else None))
        off += w * h
    return out


def gpu_candidates(ctx, eye, hfov, W, H, cap=32):
    torch = torch_mod()
    from paper_1810_08860_amd import lf
    cand = torch.full((W * H * cap,), -9, dtype=torch.int32, device="cuda")
    contrib = torch.full((W * H * cap,), -9, dtype=torch.int32, device="cuda")
    ncand = torch.full((W * H,), -9, dtype=torch.int32, device="cuda")
    lf.lf_debug_candidates(ctx, eye, hfov, W, H, cap, cand, contrib, ncand)
    torch.cuda.synchronize()
    return (cand.view(W * H, cap).cpu().numpy(), contrib.view(W * H, cap).cpu().numpy(),
            ncand.cpu().numpy())


def lists_to_mask(lists, n_views):
    lists = np.asarray(lists)
    m = np.zeros((lists.shape[0], n_views), bool)
    r, c = np.nonzero(lists >= 0)
    m[r, lists[r, c]] = True
    return m


def set_mismatch(gpu_lists, orc_lists, band_lists, n_views):
    """(pairs differing outside the band, pairs differing inside the band)."""
    g = lists_to_mask(gpu_lists, n_views)
    o = lists_to_mask(orc_lists, n_views)
    b = lists_to_mask(band_lists, n_views)
    diff = g ^ o
    return int((diff & ~b).sum()), int((diff & b).sum())


def unstable_mask(ov, pos, rot, hfov, W, H, idx, ref_rgb, tol=COLOUR_TOL, jitter=JITTER, pos_err=POS_ERR):
    bad = np.zeros(len(idx), bool)
    limit = tol * jitter / pos_err
    for dx, dy in ((jitter, 0.0), (-jitter, 0.0), (0.0, jitter), (0.0, -jitter)):
        r = oracle.render(ov, pos, rot, hfov, W, H, idx, jitter=(dx, dy))["rgb"]
        bad |= np.abs(r - ref_rgb).max(1) > limit
    return bad


def reference_unstable_mask(ov, pos, rot, hfov, W, H, idx, ref_rgb, ss, disk_scale, tol=COLOUR_TOL, jitter=JITTER,
                            pos_err=POS_ERR):
    """unstable_mask for the offline reference render: the whole pixel (all
    its sub-rays) shifted by +-jitter px along x and y."""
    bad = np.zeros(len(idx), bool)
    limit = tol * jitter / pos_err
    for d in ((jitter, 0.0), (-jitter, 0.0), (0.0, jitter), (0.0, -jitter)):
        r = oracle.render_reference(ov, pos, rot, hfov, W, H, idx, ss=ss, disk_scale=disk_scale, jitter=d)
        bad |= np.abs(r - ref_rgb).max(1) > limit
    return bad


def check_reference(ov, got, pos, rot, hfov, W, H, idx, ss, disk_scale, label):
    """Offline reference render against the oracle's: within COLOUR_TOL on
    stable pixels, unstable pixels at most MAX_UNSTABLE of the sample (2 on
    samples too small for the fraction to mean anything)."""
    ref = oracle.render_reference(ov, pos, rot, hfov, W, H, idx, ss=ss, disk_scale=disk_scale)
    unst = reference_unstable_mask(ov, pos, rot, hfov, W, H, idx, ref, ss, disk_scale)
    err = np.abs(got[idx] - ref).max(1)
    stable_max = float(err[~unst].max())
    print(f"{label}: max err stable {stable_max:.3g}, all {err.max():.3g}, unstable {int(unst.sum())} of {len(idx)}")
    assert unst.sum() <= max(2, MAX_UNSTABLE * len(idx))
    assert stable_max <= COLOUR_TOL
    return stable_max


def check_eye(ov, ctx, pos, rot, hfov, W, H, idx=None, gpu=None, colour_tol=COLOUR_TOL, lists=True, cap=32,
              max_unstable=MAX_UNSTABLE):
    """Full parity check of one eye on pixel indices idx (all if None).
    Returns a dict of statistics; asserts the parity criteria."""
    n_views = ov.n
    if idx is None:
        idx = np.arange(W * H)
    ref = oracle.render(ov, pos, rot, hfov, W, H, idx, cap=cap)
    if gpu is None:
        gpu = gpu_render(ctx, [(pos, rot)], hfov, [(W, H)])[0]
    rgb, ws, cnt = gpu
    unstable = unstable_mask(ov, pos, rot, hfov, W, H, idx, ref["rgb"])
    err = np.abs(rgb[idx] - ref["rgb"]).max(1)
    stable = ~unstable
    stats = {
        "pixels": len(idx),
        "unstable_frac": float(unstable.mean()),
        "max_err_stable": float(err[stable].max()) if stable.any() else 0.0,
        "max_err_all": float(err.max()),
    }
    # the fraction bound is meant for whole frames; tiny eyes may hold a pixel or two
    assert unstable.sum() <= max(2, max_unstable * len(idx)), stats
    assert stats["max_err_stable"] <= colour_tol, stats
    if ws is not None:
        # W > 0 iff some view contributes, and W matches the oracle's rho sum
        assert ((ws[idx] > 0) == (cnt[idx] > 0)).all()
        werr = np.abs(ws[idx] - ref["wsum"])
        stats["max_wsum_err_stable"] = float(werr[stable].max()) if stable.any() else 0.0
        assert stats["max_wsum_err_stable"] <= 1e-4, stats
    if lists:
        gc, gh, gn = gpu_candidates(ctx, (pos, rot), hfov, W, H, cap)
        out_c, in_c = set_mismatch(gc[idx], ref["cand"], ref["cand_band"], n_views)
        band_h = np.concatenate([ref["cand_band"], ref["contrib_band"]], 1)
        out_h, in_h = set_mismatch(gh[idx], ref["contrib"], band_h, n_views)
        stats.update(cand_mismatch=out_c, cand_band_diff=in_c, contrib_mismatch=out_h, contrib_band_diff=in_h)
        assert out_c == 0, stats
        assert out_h == 0, stats
        assert (gn[idx] == ref["n_cand"]).mean() > 0.999, stats
    return stats
