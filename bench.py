#!/usr/bin/env python3
"""Benchmark of the light field renderer on one MI355X.

Workload (synthetic, seeded): 1024 source views of 1024x1024 RGBA8 on a
0.35 m Fibonacci capture sphere with 256x256 z-depth meshes, a scene of 12
textured spheres in a 6 m box; stereo eye pairs of 2 x 1440x1600 at 100 deg
horizontal FOV, IPD 64 mm, for 3000 seeded head poses in a 0.25 m ball. One
step is one stereo frame through the whole path (per-eye set-up, tile
culling, fused reproject + gather + blend), with the light field already
resident in HBM.

Prints ONE JSON line. `value` is eye-view Mpix/s of the FP16/batched path
(FP16 images, FP32 geometry, FP32 arithmetic, 16 stereo frames per persistent
graph-captured launch); the plain FP32 path (FP32 images and geometry, one
launch sequence per stereo frame) is timed beside it, and so are the batched
path with FP16 geometry too and with RGBA8 images (the oracle leg gives each
batched form's error table on 32 poses), a mixed-size
batch (64 stereo poses at 1080x1200 / 1440x1600 / 2160x2160 per eye, autotuned
tile shape) and the FP64 oracle on the host cores. The per-frame path is also
timed with the images in the YUV420 form of the paper's tile cache (1.5 bytes
per texel). The batched FP16 path is
also timed with the asymmetric oval disks of Sec. 4.4 (extents from the
Delaunay 1-ring of each view) in place of the workload's circular disks: a
different blending field, reported beside the headline, never as it. A last
leg times the light field prefilter of Sec. 5 (Eq. (5)): 16 views of a
real-time model (every 4th view) prefiltered at full resolution with 16
Lanczos-2 samples per pixel against the whole view set as the offline model.
The two-level leg renders with half the fine views available and the coarse
level (every 4th capture, larger disks) filling in (Sec. 7.2). The YUV420
form is also timed transcoded to RGTC blocks (0.75 bytes per texel). The
streaming leg pages the fine views' 64x64 image tiles from host memory into a
2 GB device cache (FIFO, at most 128 tiles per frame) along a turning head
path, with the coarse level resident (Sec. 4.2 and Sec. 7.2).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "eye-view Mpix/s + ms/stereo frame, FP16/batched vs plain FP32 at ≤2/255 err"
EYE_W, EYE_H, HFOV, IPD = 1440, 1600, 100.0, 0.064
FP32_VECTOR_PEAK_TFLOPS = 157.3
HBM_PEAK_GBS = 8000.0
# algorithmic FP32 operations per counted unit of k_render: a disk test (2 dot
# products, a reciprocal, 2 products, the offset, a square root), a candidate's
# march set-up (grid transform, domain clip), a mesh cell (exit inverse depths,
# local coordinates, triangle select, field evaluation, sign test), a bilinear
# sample with its accumulation (texel coordinates, 9 lerps as FMAs, 4 sums)
FLOPS_PER = {"disk_tests": 25, "candidates": 30, "cells": 28, "samples": 50}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


RENDER_SOURCES = ("lf_kernels.hip", "lf_ray.h", "lf_internal.h")
RENDER_KERNEL = "k_render_persistent<1, 0, 0>"


def kernel_source_hash() -> str:
    """Hash of the sources the render kernels are compiled from."""
    h = hashlib.sha256()
    for name in RENDER_SOURCES:
        with open(os.path.join(ROOT, "paper_1810_08860_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _counter_means(path):
    """{kernel name: {counter: mean value per dispatch}} from a rocprofv3 --pmc CSV."""
    import csv
    acc = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            acc.setdefault(r["Kernel_Name"], {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    return {k: {c: sum(v) / len(v) for c, v in d.items()} for k, d in acc.items()}


def write_traffic(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, copy_bytes, out_path, commands):
    """HBM bytes per launch of the batched render kernel from FETCH_SIZE and
    WRITE_SIZE (KiB per dispatch), each scaled by what the same counter reads
    for a device copy of copy_bytes (the kernel with the largest reading in the
    calibration runs)."""
    def pick(path, counter, name=None):
        m = _counter_means(path)
        if name is None:
            return max(v[counter] for v in m.values())
        hits = [v[counter] for k, v in m.items() if name in k]
        if not hits:
            raise SystemExit(f"no kernel matching {name!r} in {path}")
        return hits[0]
    cf, cw = pick(copy_fetch_csv, "FETCH_SIZE"), pick(copy_write_csv, "WRITE_SIZE")
    rf, rw = pick(fetch_csv, "FETCH_SIZE", RENDER_KERNEL), pick(write_csv, "WRITE_SIZE", RENDER_KERNEL)
    fs, wsc = copy_bytes / (cf * 1024.0), copy_bytes / (cw * 1024.0)
    t = {
        "kernel": f"{RENDER_KERNEL} (FP16 images, FP32 geometry, 16 stereo frames of 2 x {EYE_W} x {EYE_H} per launch)",
        "kernel_hash": kernel_source_hash(),
        "calibration": {"copy_bytes": copy_bytes, "fetch_kib_read": cf, "write_kib_read": cw,
                        "fetch_scale": fs, "write_scale": wsc},
        "variants": {"fp16_batched": {"fetch_kib_raw": rf, "write_kib_raw": rw,
                                      "fetch_bytes": rf * 1024.0 * fs, "write_bytes": rw * 1024.0 * wsc}},
        "commands": commands,
    }
    with open(out_path, "w") as f:
        json.dump(t, f, indent=1)
        f.write("\n")
    return t


def load_traffic(path, variant):
    """HBM bytes per k_render launch measured by rocprofv3 --pmc (FETCH_SIZE,
    WRITE_SIZE), scaled by a copy-kernel calibration; None when absent or
    taken on a different kernel source."""
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_source_hash():
        return None
    v = t.get("variants", {}).get(variant)
    if not v:
        return None
    return v.get("fetch_bytes", 0) + v.get("write_bytes", 0)


def time_variant(lf, torch, ctx, eyes_all, steps, warmup, profile=False):
    npx = 2 * EYE_W * EYE_H
    out = torch.empty(npx * 3, dtype=torch.float32, device="cuda")
    res = np.array([[EYE_W, EYE_H], [EYE_W, EYE_H]], np.int32)
    P = len(eyes_all)
    for k in range(warmup):  # warm-up poses from the end of the list, timed poses from the start
        lf.lf_render(ctx, eyes_all[P - 1 - k % P], HFOV, res, out)
    torch.cuda.synchronize()
    if profile:
        lf.lf_profile(ctx, True)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        ev[k][0].record()
        lf.lf_render(ctx, eyes_all[k % P], HFOV, res, out)
        ev[k][1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = None
    if profile:
        prof = lf.lf_profile_read(ctx)
        lf.lf_profile(ctx, False)
    frame_ms = np.array([a.elapsed_time(b) for a, b in ev])
    total_s = t1 - t0
    return {
        "frames": steps,
        "mpix_s": npx * steps / total_s / 1e6,
        "ms_per_stereo_frame": 1e3 * total_s / steps,
        "p50_ms": float(np.percentile(frame_ms, 50)),
        "p99_ms": float(np.percentile(frame_ms, 99)),
        "prof": prof,
        "out": out,
    }


def achievable_hbm(lf, torch, nbytes=2 << 30, reps=10):
    """Achievable HBM bandwidth: the library's plain streaming copy of 2 GiB
    (each byte read once and written once), median of 10 timed copies."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(2):
        lf.lf_stream_copy(src, dst, nbytes)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record()
        lf.lf_stream_copy(src, dst, nbytes)
        b.record()
    torch.cuda.synchronize()
    assert torch.equal(src[:1024], dst[:1024])
    ms = float(np.median([a.elapsed_time(b) for a, b in ev]))
    del src, dst
    return 2 * nbytes / (ms * 1e-3) / 1e9


def achievable_fma(lf, torch, waves_per_simd=7, iters=4096, reps=5):
    """Achievable rate of wave-level FP32 FMA instructions: the library's FMA
    yardstick (eight independent chains per lane) on seven workgroups of four
    wavefronts per CU, the render kernel's occupancy, with all 64 lanes of a
    wavefront live and with 16; median of `reps` timed launches. Rates are
    per SIMD (four per CU) and per second; x 2 flops x live lanes gives FLOP/s."""
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    blocks = cus * waves_per_simd
    out = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
    res = {"waves_per_simd": waves_per_simd, "fma_per_lane": 8 * iters}
    for active in (64, 16):
        for _ in range(2):
            lf.lf_fma_rate(out, blocks, iters, active)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in ev:
            a.record()
            lf.lf_fma_rate(out, blocks, iters, active)
            b.record()
        torch.cuda.synchronize()
        ms = float(np.median([a.elapsed_time(b) for a, b in ev]))
        per_simd = blocks * 4 * 8 * iters / (ms * 1e-3) / (4 * cus)
        res[f"lanes{active}"] = {"ms": ms, "wave_fma_per_simd_per_s": per_simd,
                                 "tflops": per_simd * 4 * cus * 2 * active / 1e12}
    del out
    return res


def cpu_baseline(lf, torch, views, head_pos, head_rot, ctx_plain, seconds):
    """FP64 oracle on a bounded sample of the same workload (pixels of the
    first stereo frame, strided), on all host cores; also the largest
    difference of the plain FP32 GPU render from it on that sample."""
    import oracle
    ov = oracle.OracleViews.from_views(views)
    eyes = oracle.stereo_eyes(head_pos[0], head_rot[0], IPD)
    npx = EYE_W * EYE_H
    gpu = torch.empty(2 * npx * 3, dtype=torch.float32, device="cuda")
    lf.lf_render(ctx_plain, lf.lf_stereo_eyes(head_pos[0], head_rot[0], IPD), HFOV,
                 np.array([[EYE_W, EYE_H]] * 2, np.int32), gpu)
    torch.cuda.synchronize()
    gpu_h = gpu.view(2, npx, 3).cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(0)
    done, t_used, errs = 0, 0.0, []
    worst = None
    chunk = 4096
    while t_used < seconds:
        e = done % 2
        idx = rng.integers(0, npx, chunk)
        t0 = time.perf_counter()
        r = oracle.render(ov, eyes[e][0], eyes[e][1], HFOV, EYE_W, EYE_H, idx)
        t_used += time.perf_counter() - t0
        d = np.abs(gpu_h[e][idx] - r["rgb"]).max(1)
        errs.append(d)
        i = int(d.argmax())
        if worst is None or d[i] > worst["abs"]:
            worst = {"abs": float(d[i]), "eye": e, "x": int(idx[i] % EYE_W), "y": int(idx[i] // EYE_W),
                     "gpu": gpu_h[e][idx[i]].tolist(), "oracle": r["rgb"][i].tolist()}
        done += chunk
    err = np.concatenate(errs)
    if worst is not None:
        # how far the oracle itself moves under a +-1e-3 px shift of that pixel's ray:
        # above 1e-2 the pixel sits on an edge and either side is a correct answer
        pix = np.array([worst["y"] * EYE_W + worst["x"]])
        e = worst["eye"]
        c0 = np.array(worst["oracle"])
        span = 0.0
        for jt in ((1e-3, 0.0), (-1e-3, 0.0), (0.0, 1e-3), (0.0, -1e-3)):
            rj = oracle.render(ov, eyes[e][0], eyes[e][1], HFOV, EYE_W, EYE_H, pix, jitter=jt)
            span = max(span, float(np.abs(rj["rgb"][0] - c0).max()))
        worst["oracle_span_under_1e-3px_jitter"] = span
        worst["unstable"] = span > 1e-2
    return {
        "value": done / t_used / 1e6,
        "unit": "Mpix/s",
        "cores": oracle.max_threads(),
        "kind": "oracle",
        "sample": f"{done} random pixels of the first stereo frame (2x{EYE_W}x{EYE_H}), FP64, all views, "
                  f"{t_used:.1f} s",
        "s_per_stereo_frame": 2 * npx / (done / t_used),
        "gpu_fp32_vs_oracle": {"max_abs": float(err.max()), "p999_abs": float(np.quantile(err, 0.999)),
                               "frac_gt_1e-4": float((err > 1e-4).mean()), "worst_pixel": worst},
    }


MIN_LAUNCHES = 10


def batch_poses(w, first, per_batch):
    """Eye table of one batched launch: per_batch consecutive stereo poses from
    pose `first` on (wrapping around the pose list)."""
    from paper_1810_08860_amd import lf
    P = len(w.head_pos)
    eyes = []
    for k in range(per_batch):
        q = (first + k) % P
        eyes.extend(lf.lf_stereo_eyes(w.head_pos[q], w.head_rot[q], IPD))
    return lf.make_eyes([(np.array(e.pos), np.array(e.rot)) for e in eyes])


def batched_error_table(lf, torch, ov, ctx, w, per_batch, path, n_poses=32, px_per_eye=4096, seed=7):
    """Error of the batched FP16 path itself against the FP64 oracle: poses
    0..n_poses-1 rendered by lf_render_batch in launches of per_batch poses
    (exactly as timed), px_per_eye random pixels per eye. Per stereo frame:
    max abs error on stable pixels (the oracle moves by at most 1e-2 under a
    +-1e-3 px shift of the ray) and over all sampled pixels, PSNR over the
    sampled pixels, unstable count. Part of the oracle leg (FP64 CPU work)."""
    import oracle
    npx = EYE_W * EYE_H
    res = np.array([[EYE_W, EYE_H]] * (2 * per_batch), np.int32)
    out = torch.empty(2 * per_batch * npx * 3, dtype=torch.float32, device="cuda")
    rng = np.random.default_rng(seed)
    rows, t_oracle = [], 0.0
    for b in range(-(-n_poses // per_batch)):
        lf.lf_render_batch(ctx, batch_poses(w, b * per_batch, per_batch), HFOV, res, out)
        torch.cuda.synchronize()
        host = out.view(2 * per_batch, npx, 3)
        for k in range(per_batch):
            q = b * per_batch + k
            if q >= n_poses:
                break
            eyes = oracle.stereo_eyes(w.head_pos[q], w.head_rot[q], IPD)
            st, al, sq, un, n = 0.0, 0.0, 0.0, 0, 0
            for e in range(2):
                idx = np.sort(rng.choice(npx, px_per_eye, replace=False))
                got = host[2 * k + e][torch.from_numpy(idx).cuda()].cpu().numpy().astype(np.float64)
                t0 = time.perf_counter()
                ref = oracle.render(ov, eyes[e][0], eyes[e][1], HFOV, EYE_W, EYE_H, idx)["rgb"]
                span = np.zeros(len(idx))
                for d in ((1e-3, 0.0), (-1e-3, 0.0), (0.0, 1e-3), (0.0, -1e-3)):
                    rj = oracle.render(ov, eyes[e][0], eyes[e][1], HFOV, EYE_W, EYE_H, idx, jitter=d)["rgb"]
                    span = np.maximum(span, np.abs(rj - ref).max(1))
                t_oracle += time.perf_counter() - t0
                err = np.abs(got - ref).max(1)
                unst = span > 1e-2
                st = max(st, float(err[~unst].max()))
                al = max(al, float(err.max()))
                sq += float(((got - ref) ** 2).sum())
                un += int(unst.sum())
                n += len(idx)
            rows.append({"pose": q, "max_abs_stable": st, "max_abs_all": al,
                         "psnr_db": 10 * np.log10(1.0 / max(sq / (3 * n), 1e-30)), "unstable": un, "pixels": n})
    return {
        "path": path,
        "sample": f"{px_per_eye} random pixels per eye x 2 eyes x {n_poses} poses (0..{n_poses - 1}), "
                  f"launches of {per_batch} poses; stable = oracle moves <= 1e-2 under a +-1e-3 px ray shift",
        "bound": 2.0 / 255,
        "max_abs_stable": max(r["max_abs_stable"] for r in rows),
        "max_abs_all": max(r["max_abs_all"] for r in rows),
        "psnr_db_min": min(r["psnr_db"] for r in rows),
        "psnr_db_mean": float(np.mean([r["psnr_db"] for r in rows])),
        "unstable_frac": sum(r["unstable"] for r in rows) / sum(r["pixels"] for r in rows),
        "within_bound": all(r["max_abs_stable"] <= 2.0 / 255 for r in rows),
        "oracle_s": t_oracle,
        "per_frame": rows,
    }


def time_batched(lf, torch, ctx, w, steps, warmup, per_batch, profile=False):
    """Stereo frames rendered per_batch at a time with lf_render_batch: at
    least MIN_LAUNCHES launches and at least `steps` frames, each launch with
    its own poses (poses 0, 1, ... in order); the warm-up launches take poses
    from the end of the list, so no timed launch repeats a warm-up pose. Each
    launch is bracketed by HIP events on the render stream (p50 / p99 per
    launch); the value is the pixels of all timed launches over the wall
    time of the timed region. Where `steps` frames and the warm-up do not fit
    in the pose list together, the timed frames are cut to the poses the
    warm-up leaves (every pose at most once)."""
    P = len(w.head_pos)
    nw = max(1, -(-warmup // per_batch))
    nb = max(MIN_LAUNCHES, -(-steps // per_batch))
    if (nb + nw) * per_batch > P:
        fit = P // per_batch - nw
        if fit < MIN_LAUNCHES:
            raise SystemExit(f"{MIN_LAUNCHES + nw} launches of {per_batch} poses need more than the {P} poses")
        print(f"[bench] {steps} frames + warm-up exceed the {P} poses: timing {fit * per_batch} frames",
              file=sys.stderr, flush=True)
        nb = fit
    res = np.array([[EYE_W, EYE_H]] * (2 * per_batch), np.int32)
    timed = [batch_poses(w, b * per_batch, per_batch) for b in range(nb)]
    warm = [batch_poses(w, P - (k + 1) * per_batch, per_batch) for k in range(nw)]
    npx = 2 * per_batch * EYE_W * EYE_H
    out = torch.empty(npx * 3, dtype=torch.float32, device="cuda")
    if profile:
        lf.lf_profile(ctx, True)  # graph captured with timing nodes from the start
        lf.lf_profile(ctx, False)
        lf.lf_profile(ctx, True)
    for k in range(nw):
        lf.lf_render_batch(ctx, warm[k], HFOV, res, out)
    torch.cuda.synchronize()
    if profile:
        lf.lf_profile_read(ctx)  # drop warm-up timings
        lf.lf_profile(ctx, True)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(nb)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for b in range(nb):
        ev[b][0].record()
        lf.lf_render_batch(ctx, timed[b], HFOV, res, out)
        ev[b][1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = lf.lf_profile_read(ctx) if profile else None
    if profile:
        lf.lf_profile(ctx, False)
    launch_ms = np.array([a.elapsed_time(b) for a, b in ev])
    frames = nb * per_batch
    return {
        "mpix_s": npx * nb / (t1 - t0) / 1e6,
        "ms_per_stereo_frame": 1e3 * (t1 - t0) / frames,
        "frames": frames,
        "launches": nb,
        "frames_per_launch": per_batch,
        "launch_ms_p50": float(np.percentile(launch_ms, 50)),
        "launch_ms_p99": float(np.percentile(launch_ms, 99)),
        "p50_ms": float(np.percentile(launch_ms, 50)) / per_batch,
        "p99_ms": float(np.percentile(launch_ms, 99)) / per_batch,
        "timed_poses": [0, frames],
        "prof": prof,
    }


def timed_work(lf, ctx, w, first, frames):
    """Work counters (lf_render_stats) summed over stereo poses [first, first + frames)."""
    acc = {k: 0 for k in lf.STAT_NAMES}
    res = np.array([[EYE_W, EYE_H]] * 2, np.int32)
    for q in range(first, first + frames):
        s = lf.lf_render_stats(ctx, lf.lf_stereo_eyes(w.head_pos[q], w.head_rot[q], IPD), HFOV, res)
        for k in acc:
            acc[k] += s[k]
    return acc


MIXED_SIZES = [(1080, 1200), (1440, 1600), (2160, 2160)]
CORR_FLOP_PER_PX = 2 * 9 * (5 * 32 + 32 * 32 + 32 * 32 + 32 * 3)  # 41,472 multiply-adds x 2
BF16_MFMA_PEAK_TFLOPS = 2500.0


def corrector_leg(lf, torch, ctx_rt, ctx_ref, steps=1250, batch=16, crop=96):
    """Train the residual corrector on pairs the method generates (real-time
    FP16 render vs the offline reference: 4x4 sub-pixel rays, disks of twice
    the radius) from three seeded scenes: the bench's scene (seed 0) and
    scenes 1 and 2, generated the same way (12 textured spheres in a box,
    1024 views of 1024^2); 8 eyes each, 20k random crops by default. PSNR
    and max error on held-out poses of scene 0 and on a held-out scene
    (seed 3); inference time on a stereo frame."""
    import lfsynth
    from paper_1810_08860_amd import corrector

    def eyes(seed, n):
        p, R = lfsynth.poses(seed, n, 0.25)
        out = []
        for k in range(n):
            out += [(np.array(e.pos), np.array(e.rot).reshape(3, 3)) for e in lf.lf_stereo_eyes(p[k], R[k], IPD)]
        return out

    def scene_frames(seed, pose_seed, n_poses):
        V = lfsynth.make_views(1024, 1024, 256, 12, seed=seed)
        rt = lf.lf_load_views(V.centres, V.rot, V.rgba8, V.zdepth, V.src_fov_deg, V.disk_radius,
                              img_fmt="rgba16f", geo_fmt="f32")
        ref = lf.lf_load_views(V.centres, V.rot, V.rgba8, V.zdepth, V.src_fov_deg, V.disk_radius,
                               img_fmt="rgba32f", geo_fmt="f32")
        fr = corrector.make_frames(rt, ref, eyes(pose_seed, n_poses), HFOV, EYE_W, EYE_H)
        rt.close()
        ref.close()
        return fr

    t0 = time.perf_counter()
    train_frames = corrector.make_frames(ctx_rt, ctx_ref, eyes(500, 4), HFOV, EYE_W, EYE_H)
    held_poses = corrector.make_frames(ctx_rt, ctx_ref, eyes(900, 2), HFOV, EYE_W, EYE_H)
    for seed in (1, 2):
        train_frames += scene_frames(seed, 500 + seed, 4)
    held_scene = scene_frames(3, 950, 2)
    t_pairs = time.perf_counter() - t0
    corr = lf.lf_corrector_create(corrector.init_params(0))
    t0 = time.perf_counter()
    log = corrector.train(corr, train_frames, steps=steps, batch=batch, crop=crop, seed=1, log_every=250)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    ev = corrector.evaluate(corr, held_poses)
    ev_scene = corrector.evaluate(corr, held_scene)
    test_frames = held_poses
    # inference timing on one stereo frame (both eyes in one call)
    f0, f1 = test_frames[0], test_frames[1]
    rgb = torch.stack([f0.rgb, f1.rgb]).contiguous()
    ws = torch.stack([f0.wsum, f1.wsum]).contiguous()
    cnt = torch.stack([f0.count, f1.count]).contiguous()
    out = torch.empty_like(rgb)
    for _ in range(3):
        lf.lf_corrector_apply(corr, rgb, ws, cnt, 2, EYE_W, EYE_H, 8.0 / 255.0, out)
    reps = 20
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        lf.lf_corrector_apply(corr, rgb, ws, cnt, 2, EYE_W, EYE_H, 8.0 / 255.0, out)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    tflops = CORR_FLOP_PER_PX * 2 * EYE_W * EYE_H / (ms * 1e-3) / 1e12
    # one training step (forward, loss, backward, Adam) on a fixed batch of
    # crops resident on the device (the training loop above also copies its
    # random crops from the host side each step)
    cr = [train_frames[k % len(train_frames)] for k in range(batch)]
    c_rgb, c_ws, c_cnt, c_ref = (torch.stack([getattr(f, n)[:crop, :crop] for f in cr]).contiguous()
                                 for n in ("rgb", "wsum", "count", "ref"))
    for _ in range(3):
        lf.lf_corrector_train_step(corr, c_rgb, c_ws, c_cnt, c_ref, batch, crop, crop, 0.0, want_loss=False)
    torch.cuda.synchronize()
    a.record()
    for _ in range(50):
        lf.lf_corrector_train_step(corr, c_rgb, c_ws, c_cnt, c_ref, batch, crop, crop, 0.0, want_loss=False)
    b.record()
    torch.cuda.synchronize()
    step_ms = a.elapsed_time(b) / 50
    corr.close()
    return {
        "training_crops": steps * batch,
        "crop": crop,
        "train_scenes": [0, 1, 2],
        "train_eyes": len(train_frames),
        "held_out_eyes": len(test_frames),
        "held_out_scene": {"seed": 3, "eyes": len(held_scene), "psnr_plain_db": ev_scene["psnr_plain"],
                           "psnr_corrected_db": ev_scene["psnr_corrected"], "psnr_gain_db": ev_scene["psnr_gain_db"],
                           "max_err_plain": ev_scene["max_err_plain"],
                           "max_err_corrected": ev_scene["max_err_corrected"],
                           "fallback_frac": ev_scene["fallback_frac"]},
        "pair_generation_s": t_pairs,
        "train_s": t_train,
        "train_step_ms": step_ms,
        "train_step": f"{batch} resident crops of {crop} x {crop}, mean of 50 steps (HIP events)",
        "loss_first_last": [log[0][1], log[-1][1]],
        "psnr_plain_db": ev["psnr_plain"],
        "psnr_corrected_db": ev["psnr_corrected"],
        "psnr_gain_db": ev["psnr_gain_db"],
        "max_err_plain": ev["max_err_plain"],
        "max_err_corrected": ev["max_err_corrected"],
        "fallback_threshold": 8.0 / 255.0,
        "fallback_frac": ev["fallback_frac"],
        "ms_per_stereo_frame": ms,
        "achieved_tflops": tflops,
        "mfma_bf16_peak_tflops": BF16_MFMA_PEAK_TFLOPS,
        "frac_of_peak": tflops / BF16_MFMA_PEAK_TFLOPS,
    }


def prefilter_leg(lf, torch, ctx, V, n_targets=16, n_samples=16, reps=3):
    """Prefilter of Sec. 5 (Eq. (5)) over the full light field: the real-time
    model is every 4th view (disks 1.5 x its mean nearest-neighbour spacing),
    the offline model answering the ray queries is the whole view set; 16 of
    the real-time views are prefiltered at full resolution with 16 Lanczos-2
    samples per pixel."""
    import lfsynth
    rt = np.arange(0, V.n, 4)
    radius = 1.5 * lfsynth.mean_nn(V.centres[rt])
    views = rt[:: max(1, len(rt) // n_targets)][:n_targets]
    dp, po = lfsynth.prefilter_samples(77, n_samples, 2.0)
    npx = V.img_res * V.img_res
    out = torch.empty(len(views) * npx * 3, dtype=torch.float32, device="cuda")
    ws = torch.empty(len(views) * npx, dtype=torch.float32, device="cuda")
    lf.lf_prefilter(ctx, views[:1], radius, dp, po, "lanczos2", out, ws)
    torch.cuda.synchronize()
    best = None
    for _ in range(reps):
        t0 = time.perf_counter()
        lf.lf_prefilter(ctx, views, radius, dp, po, "lanczos2", out, ws)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        best = t if best is None else min(best, t)
    rays = len(views) * npx * n_samples
    return {
        "views": len(views),
        "samples_per_pixel": n_samples,
        "basis": "lanczos2",
        "aperture_radius_m": radius,
        "offline_views": V.n,
        "ms_per_view": 1e3 * best / len(views),
        "mrays_s": rays / best / 1e6,
        "note": "one ray = one (pixel, sample) query of the offline model; real-time model = every 4th view",
    }


def two_level_leg(lf, torch, V, eyes_all, steps=200, avail_frac=0.5):
    """Two-level progressive rendering (Sec. 7.2): fine level = every view,
    coarse level = every 4th capture again with disks for its own spacing;
    a seeded half of the fine views is available per frame, and the coarse
    disks that reach a missing fine centre are drawn with them (FP16 images
    and geometry, per-frame path)."""
    import lfsynth
    coarse = np.arange(0, V.n, 4)
    idx = np.concatenate([np.arange(V.n), coarse])
    ext = np.concatenate([np.full((V.n, 4), V.disk_radius),
                          np.full((len(coarse), 4), 1.5 * lfsynth.mean_nn(V.centres[coarse]))])
    ctx = lf.lf_load_views(V.centres[idx], V.rot[idx], V.rgba8[idx], V.zdepth[idx], V.src_fov_deg, V.disk_radius,
                           img_fmt="rgba16f", geo_fmt="f32", disk_ext=ext)
    avail = (np.random.default_rng(5).uniform(size=V.n) < avail_frac).astype(np.uint8)
    mask = lf.lf_two_level_mask(ctx, V.n, avail)
    lf.lf_set_view_mask(ctx, mask)
    r = time_variant(lf, torch, ctx, eyes_all, steps, 16)
    ctx.close()
    return {"fine_available": int(mask[:V.n].sum()), "coarse_drawn": int(mask[V.n:].sum()),
            "mpix_s": r["mpix_s"], "ms_per_stereo_frame": r["ms_per_stereo_frame"],
            "p50_ms": r["p50_ms"], "p99_ms": r["p99_ms"]}


def streaming_leg(lf, torch, V, head_pos, head_rot, frames=270, budget=128, cache_gb=2.0, yaw_deg_s=60.0):
    """Tile streaming and caching (Sec. 4.2, Sec. 7.2) along a head path:
    fine level = every view, paged (64x64 RGBA8 tiles in pinned host memory,
    a 2 GB device cache of pages, FIFO); coarse level = every 4th capture
    again with disks for its spacing, resident in the cache. Each 90 Hz frame
    runs lf_cache_update (visibility pass, at most `budget` tiles copied in,
    mask = available fine views + coarse fill-in) and then renders the stereo
    frame. The path starts cold (empty fine cache) and turns the head at
    yaw_deg_s while drifting 5 cm/s."""
    import lfsynth
    coarse = np.arange(0, V.n, 4)
    idx = np.concatenate([np.arange(V.n), coarse])
    ext = np.concatenate([np.full((V.n, 4), V.disk_radius),
                          np.full((len(coarse), 4), 1.5 * lfsynth.mean_nn(V.centres[coarse]))])
    ctx = lf.lf_load_views(V.centres[idx], V.rot[idx], V.rgba8[idx], V.zdepth[idx], V.src_fov_deg, V.disk_radius,
                           img_fmt="paged_rgba8", geo_fmt="f32", disk_ext=ext)
    pages = int(cache_gb * (1 << 30)) // (64 * 64 * 4)
    lf.lf_cache_config(ctx, pages, first_resident=V.n)
    res = np.array([[EYE_W, EYE_H], [EYE_W, EYE_H]], np.int32)
    out = torch.empty(2 * EYE_W * EYE_H * 3, dtype=torch.float32, device="cuda")
    up_ms, rd_ms, copied, missing, visible = [], [], [], [], []
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(frames)]
    for f in range(frames):
        a = np.radians(yaw_deg_s) * f / 90.0
        Rz = np.array([[np.cos(a), -np.sin(a), 0], [np.sin(a), np.cos(a), 0], [0, 0, 1.0]])
        pos = head_pos + np.array([0.05 * f / 90.0, 0.0, 0.0])
        eyes = [(np.array(e.pos), np.array(e.rot).reshape(3, 3)) for e in lf.lf_stereo_eyes(pos, Rz @ head_rot, IPD)]
        t0 = time.perf_counter()
        _, _, st = lf.lf_cache_update(ctx, eyes, HFOV, res, budget, n_fine=V.n, want_visible=False)
        up_ms.append(1e3 * (time.perf_counter() - t0))
        ev[f][0].record()
        lf.lf_render(ctx, eyes, HFOV, res, out)
        ev[f][1].record()
        copied.append(st["copied"])
        missing.append(st["views_unavailable"])
        visible.append(st["visible"])
    torch.cuda.synchronize()
    rd_ms = np.array([x.elapsed_time(y) for x, y in ev])
    misses = lf.lf_cache_page_misses(ctx)
    ctx.close()
    up_ms, copied, missing = np.array(up_ms), np.array(copied), np.array(missing)
    warm = int(np.argmax(missing == 0)) if (missing == 0).any() else frames
    steady = slice(warm, frames)
    return {
        "frames": frames, "budget_tiles": budget, "cache_gb": cache_gb, "yaw_deg_s": yaw_deg_s,
        "visible_tiles_mean": float(np.mean(visible)),
        "cold_start_frames": warm,
        "copied_tiles_cold_mean": float(copied[:warm].mean()) if warm else 0.0,
        "copied_tiles_steady_mean": float(copied[steady].mean()) if warm < frames else None,
        "copied_tiles_steady_max": int(copied[steady].max()) if warm < frames else None,
        "fine_views_unavailable_steady_mean": float(missing[steady].mean()) if warm < frames else None,
        "update_ms_p50": float(np.percentile(up_ms, 50)), "update_ms_p99": float(np.percentile(up_ms, 99)),
        "render_ms_p50": float(np.percentile(rd_ms, 50)), "render_ms_p99": float(np.percentile(rd_ms, 99)),
        "page_misses": misses,
        "note": "update = visibility pass + host FIFO + tile copies + mask (synchronous); render = lf_render of the "
                "stereo frame from the cache",
    }


def mixed_batch(lf, torch, ctx, seed, n_poses=64, reps=10):
    """64 stereo poses of uneven per-eye sizes in one persistent launch."""
    import lfsynth
    rng = np.random.default_rng(seed)
    eyes_b, res = [], []
    p, R = lfsynth.poses(seed, n_poses * reps, 0.25)
    sizes = [MIXED_SIZES[rng.integers(0, 3)] for _ in range(n_poses)]
    for r in range(reps):
        eyes = []
        for k in range(n_poses):
            eyes.extend(lf.lf_stereo_eyes(p[r * n_poses + k], R[r * n_poses + k], IPD))
        eyes_b.append(lf.make_eyes([(np.array(e.pos), np.array(e.rot)) for e in eyes]))
    for k in range(n_poses):
        res += [sizes[k], sizes[k]]
    res = np.array(res, np.int32)
    npx = int((res[:, 0].astype(np.int64) * res[:, 1]).sum())
    out = torch.empty(npx * 3, dtype=torch.float32, device="cuda")
    t0 = time.perf_counter()
    best, table = lf.lf_autotune_batch(ctx, eyes_b[0], HFOV, res, out, reps=5)
    tune_s = time.perf_counter() - t0
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    spans = []
    lf.lf_render_batch(ctx, eyes_b[0], HFOV, res, out)
    torch.cuda.synchronize()
    for r in range(reps):
        ev[r][0].record()
        lf.lf_render_batch(ctx, eyes_b[r], HFOV, res, out)
        ev[r][1].record()
        t = lf.lf_batch_frame_times(ctx, 2 * n_poses)
        for k in range(n_poses):
            spans.append(max(t[2 * k + 1, 1], t[2 * k, 1]) - min(t[2 * k, 0], t[2 * k + 1, 0]))
    batch_ms = np.array([a.elapsed_time(b) for a, b in ev])
    spans = np.array(spans) / 1e3
    return {
        "poses": n_poses,
        "pixels_per_batch": npx,
        "eye_sizes": {f"{w}x{h}": int(sum(1 for s in sizes if s == (w, h))) for w, h in MIXED_SIZES},
        "tune": {"tile": f"{best[0]}x{best[1]}", "cap": best[2], "seconds": tune_s,
                 "median_ms": {f"{a}x{b} cap {c}": v for (a, b, c), v in table.items()}},
        "batch_ms_median": float(np.median(batch_ms)),
        "mpix_s": npx / (np.median(batch_ms) * 1e-3) / 1e6,
        "frame_span_ms_p50": float(np.percentile(spans, 50)),
        "frame_span_ms_p99": float(np.percentile(spans, 99)),
        "note": "frame span = device wall-clock from the first tile start to the last tile end of the pose's two "
                "eyes inside the persistent launch",
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3000, help="stereo frames timed per variant")
    ap.add_argument("--warmup", type=int, default=32)
    ap.add_argument("--per-batch", type=int, default=16, help="stereo frames per batched launch")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="CPU time budget of the oracle baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-size batch leg")
    ap.add_argument("--no-corrector", action="store_true", help="skip the learned-corrector leg")
    ap.add_argument("--no-prefilter", action="store_true", help="skip the prefilter leg")
    ap.add_argument("--no-two-level", action="store_true", help="skip the two-level progressive leg")
    ap.add_argument("--no-streaming", action="store_true", help="skip the tile streaming leg")
    ap.add_argument("--corrector-steps", type=int, default=1250)
    ap.add_argument("--variants", default="plain,fp16,rgba8,yuv420,yuv420_rgtc,fp16_batched,fp16geo_batched,"
                                           "u16geo_batched,rgba8_batched,fp16_batched_oval")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "k_render_traffic.json"))
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES five times (HBM counter calibration)")
    ap.add_argument("--traffic-from", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV"),
                    help="only write --traffic from rocprofv3 --pmc CSVs of the batched render (FETCH_SIZE, "
                         "WRITE_SIZE) and of --copy-calibration runs (same counters); no GPU use")
    ap.add_argument("--traffic-copy-bytes", type=int, default=1 << 30)
    ap.add_argument("--traffic-commands", default="", help="the profiler commands, ';'-separated, recorded as-is")
    args = ap.parse_args()
    if args.traffic_from:
        t = write_traffic(*args.traffic_from, args.traffic_copy_bytes, args.traffic,
                          [c.strip() for c in args.traffic_commands.split(";") if c.strip()])
        print(json.dumps(t))
        return
    if args.copy_calibration:
        import torch
        n = args.copy_calibration // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 4 * n, "copies": 5}))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the renderer has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import lfsynth
    from paper_1810_08860_amd import lf

    t0 = time.perf_counter()
    w = lfsynth.make_workload("full", seed=0)
    V = w.views
    log(f"[bench] generated {V.n} views {V.img_res}^2 + {V.mesh_m}^2 depth, {len(w.head_pos)} poses "
        f"in {time.perf_counter() - t0:.1f} s")
    eyes_all = [lf.lf_stereo_eyes(w.head_pos[k], w.head_rot[k], IPD) for k in range(len(w.head_pos))]

    # (images, geometry, disks): "circle" = radius 1.5 x mean nearest-neighbour spacing, the workload's
    # definition; "oval" = the asymmetric Delaunay 1-ring ovals of Sec. 4.4 (a different blending field)
    storage = {"plain": ("rgba32f", "f32", "circle"), "fp16": ("rgba16f", "f16", "circle"),
               "rgba8": ("rgba8", "f16", "circle"), "yuv420": ("yuv420", "f16", "circle"),
               "yuv420_rgtc": ("yuv420_rgtc", "f16", "circle"),
               "fp16_batched": ("rgba16f", "f32", "circle"),
               "fp16geo_batched": ("rgba16f", "f16", "circle"),
               "u16geo_batched": ("rgba16f", "u16", "circle"),
               "rgba8_batched": ("rgba8", "f32", "circle"),
               "fp16_batched_oval": ("rgba16f", "f32", "oval")}
    chosen = [v for v in args.variants.split(",") if v]
    main_name = "fp16_batched" if "fp16_batched" in chosen else chosen[0]
    results, ctxs = {}, {}
    mixed = None
    for name in chosen:
        key = storage[name]
        if key not in ctxs:
            t0 = time.perf_counter()
            ext = lf.lf_disk_extents(V.centres, V.rot) if key[2] == "oval" else None
            ctxs[key] = lf.lf_load_views(V.centres, V.rot, V.rgba8, V.zdepth, V.src_fov_deg, V.disk_radius,
                                         img_fmt=key[0], geo_fmt=key[1], disk_ext=ext)
            log(f"[bench] loaded {key} in {time.perf_counter() - t0:.1f} s")
        ctx = ctxs[key]
        prof = name == main_name
        if "_batched" in name:
            r = time_batched(lf, torch, ctx, w, args.steps, args.warmup, args.per_batch, profile=prof)
        else:
            r = time_variant(lf, torch, ctx, eyes_all, args.steps, args.warmup, profile=prof)
            del r["out"]
        if prof or key[2] == "oval":
            # work counters of exactly the timed frames (outside the timed region)
            n_stat = r.get("frames", min(args.steps, len(eyes_all)))
            acc = timed_work(lf, ctx, w, 0, n_stat)
            r["stats_per_frame"] = {k: v / n_stat for k, v in acc.items()}
            r["stats_frames"] = n_stat
        results[name] = r
        log(f"[bench] {name}: {r['mpix_s']:.0f} Mpix/s, {r['ms_per_stereo_frame']:.4f} ms/stereo frame")
    if not args.no_mixed and ("rgba16f", "f32", "circle") in ctxs:
        log("[bench] mixed-size batch ...")
        mixed = mixed_batch(lf, torch, ctxs[("rgba16f", "f32", "circle")], seed=4242)
        log(f"[bench] mixed: {mixed['mpix_s']:.0f} Mpix/s, tune {mixed['tune']['tile']} cap {mixed['tune']['cap']}, "
            f"p50 {mixed['frame_span_ms_p50']:.3f} ms, p99 {mixed['frame_span_ms_p99']:.3f} ms")

    two = None
    if not args.no_two_level:
        log("[bench] two-level ...")
        two = two_level_leg(lf, torch, V, eyes_all)
        log(f"[bench] two-level: {two['fine_available']} fine + {two['coarse_drawn']} coarse views, "
            f"{two['mpix_s']:.0f} Mpix/s, {two['ms_per_stereo_frame']:.4f} ms/stereo frame")

    stream = None
    if not args.no_streaming:
        log("[bench] tile streaming ...")
        stream = streaming_leg(lf, torch, V, w.head_pos[0], w.head_rot[0])
        log(f"[bench] streaming: cold start {stream['cold_start_frames']} frames, steady "
            f"{stream['copied_tiles_steady_mean']} tiles/frame, update p50 {stream['update_ms_p50']:.3f} ms, "
            f"render p50 {stream['render_ms_p50']:.3f} ms, page misses {stream['page_misses']}")

    pref = None
    if not args.no_prefilter and ("rgba32f", "f32", "circle") in ctxs:
        log("[bench] prefilter ...")
        pref = prefilter_leg(lf, torch, ctxs[("rgba32f", "f32", "circle")], V)
        log(f"[bench] prefilter: {pref['ms_per_view']:.2f} ms per view, {pref['mrays_s']:.0f} Mrays/s")

    corr = None
    if not args.no_corrector and ("rgba16f", "f32", "circle") in ctxs and ("rgba32f", "f32", "circle") in ctxs:
        log("[bench] corrector ...")
        corr = corrector_leg(lf, torch, ctxs[("rgba16f", "f32", "circle")], ctxs[("rgba32f", "f32", "circle")],
                             steps=args.corrector_steps)
        log(f"[bench] corrector, held-out scene: PSNR {corr['held_out_scene']['psnr_plain_db']:.2f} -> "
            f"{corr['held_out_scene']['psnr_corrected_db']:.2f} dB")
        log(f"[bench] corrector: PSNR {corr['psnr_plain_db']:.2f} -> {corr['psnr_corrected_db']:.2f} dB, "
            f"{corr['ms_per_stereo_frame']:.3f} ms / stereo frame, {corr['achieved_tflops']:.0f} TFLOP/s")

    m = results[main_name]
    roofline = None
    if m.get("prof") and m.get("stats_per_frame"):
        p, st = m["prof"], m["stats_per_frame"]
        per_launch = m.get("frames_per_launch", 1)
        render_ms = p["render_ms"] / max(p["render_n"], 1)
        work = {k: v * per_launch for k, v in st.items()}
        flops = sum(FLOPS_PER[k] * work[k] for k in FLOPS_PER)
        achieved = flops / (render_ms * 1e-3) / 1e12
        traffic = load_traffic(args.traffic, main_name)
        roofline = {
            "bound": "alu",
            "achieved": achieved,
            "peak": FP32_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP32_VECTOR_PEAK_TFLOPS,
            "traffic": traffic,
            "kernel": "k_render_persistent" if "_batched" in main_name else "k_render",
            "kernel_ms": render_ms,
            "stereo_frames_per_launch": per_launch,
            "algorithmic_flop_per_launch": flops,
            "work_per_launch": work,
            "output_write_gbs": (per_launch * 2 * EYE_W * EYE_H * 12) / (render_ms * 1e-3) / 1e9,
        }
        hbm = achievable_hbm(lf, torch)
        roofline["hbm_achievable_gbs"] = hbm
        if traffic:
            roofline["traffic_gbs"] = traffic / (render_ms * 1e-3) / 1e9
            roofline["traffic_frac_of_achievable"] = roofline["traffic_gbs"] / hbm
        log(f"[bench] achievable HBM (lf_stream_copy): {hbm:.0f} GB/s")
        fma = achievable_fma(lf, torch)
        roofline["valu_fma_achievable"] = fma
        log(f"[bench] achievable FP32 FMA (lf_fma_rate, 7 waves per SIMD): "
            f"{fma['lanes64']['tflops']:.1f} TFLOP/s with 64 lanes live "
            f"({fma['lanes64']['wave_fma_per_simd_per_s'] / 1e9:.3f} G wave-FMAs per SIMD per s), "
            f"{fma['lanes16']['wave_fma_per_simd_per_s'] / 1e9:.3f} G with 16 lanes live")

    cpu = None
    if not args.no_cpu_baseline and ("rgba32f", "f32", "circle") in ctxs:
        log("[bench] cpu baseline (FP64 oracle) ...")
        cpu = cpu_baseline(lf, torch, V, w.head_pos, w.head_rot, ctxs[("rgba32f", "f32", "circle")],
                           args.cpu_seconds)
        import oracle
        ov = oracle.OracleViews.from_views(V)
        for name, what in (("fp16_batched", "RGBA16F images, FP32 geometry"),
                           ("fp16geo_batched", "RGBA16F images, FP16 geometry"),
                           ("u16geo_batched", "RGBA16F images, 16-bit inverse-depth codes"),
                           ("rgba8_batched", "RGBA8 images, FP32 geometry")):
            if name not in results:
                continue
            log(f"[bench] error table of {name} against the oracle (32 poses) ...")
            t = batched_error_table(lf, torch, ov, ctxs[storage[name]], w, args.per_batch,
                                    f"{name} ({what}, FP32 arithmetic, lf_render_batch)")
            cpu[f"{name}_vs_oracle"] = t
            log(f"[bench] {name} vs oracle: max abs stable {t['max_abs_stable']:.3g} (bound {2 / 255:.3g}), "
                f"all {t['max_abs_all']:.3g}, PSNR min {t['psnr_db_min']:.1f} dB, unstable {t['unstable_frac']:.2%}")
    for c in ctxs.values():
        c.close()

    line = {
        "metric": METRIC,
        "value": m["mpix_s"],
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["ms_per_stereo_frame"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "stereo 2x1440x1600 eye views at 100 deg from 1024 views of 1024^2 RGBA8 with 256^2 "
                        "depth meshes, 12 spheres + box, 3000 seeded head poses",
            "path": main_name,
            "storage": dict(zip(("images", "geometry", "disks"), storage[main_name])),
            "stereo_frames_per_launch": m.get("frames_per_launch", 1),
        },
        "ms_per_stereo_frame": m["ms_per_stereo_frame"],
        "frames_timed": m.get("frames"),
        "variants": {k: {kk: v[kk] for kk in ("mpix_s", "ms_per_stereo_frame", "p50_ms", "p99_ms", "frames",
                                             "launches", "launch_ms_p50", "launch_ms_p99", "stats_per_frame",
                                             "stats_frames") if kk in v} for k, v in results.items()},
        "speedup_vs_plain_fp32": (m["mpix_s"] / results["plain"]["mpix_s"]) if "plain" in results else None,
        "batched_vs_oracle": ({k[:-len("_vs_oracle")]: {kk: vv for kk, vv in v.items() if kk != "per_frame"}
                               for k, v in cpu.items() if k.endswith("_vs_oracle") and isinstance(v, dict)}
                              if cpu else None),
        "mixed_batch": mixed,
        "corrector": corr,
        "prefilter": pref,
        "two_level": two,
        "streaming": stream,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
