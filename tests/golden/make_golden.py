"""Writes oracle_tiny_rays.json: the FP64 oracle's values for 96 seeded pixels
of the tiny workload's eye (plain RGBA8 sampling, YUV420, RGTC, oval disks).
Calls only the oracle and the seeded input generator. The stored values pin
the oracle against silent drift: any change to its arithmetic must come with a
regenerated file and the passage of the paper that justifies the change.

    python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import lfsynth  # noqa: E402
import oracle  # noqa: E402

W = H = 256
N_PIX = 96


def cases():
    w = lfsynth.make_workload("tiny", seed=0)
    ov = oracle.OracleViews.from_views(w.views)
    ext, _ = oracle.disk_extents(w.views.centres, w.views.rot)
    return w, {"rgba8": ov, "yuv420": ov.with_yuv420(), "yuv420_rgtc": ov.with_yuv420_rgtc(),
               "oval": ov.with_disk_extents(ext)}


def pixels():
    return np.sort(np.random.default_rng(2024).choice(W * H, N_PIX, replace=False))


def render_all():
    w, cs = cases()
    idx = pixels()
    out = {}
    for name, ov in cs.items():
        r = oracle.render(ov, w.head_pos[0], w.head_rot[0], w.hfov_deg, W, H, idx)
        out[name] = {"rgb": r["rgb"].tolist(), "wsum": r["wsum"].tolist(), "count": r["count"].tolist()}
    return idx, out


if __name__ == "__main__":
    idx, out = render_all()
    with open(os.path.join(HERE, "oracle_tiny_rays.json"), "w") as f:
        json.dump({"workload": "tiny, seed 0, eye 256x256", "pixels": idx.tolist(), "cases": out}, f)
    print("wrote", len(idx), "pixels x", len(out), "cases")
