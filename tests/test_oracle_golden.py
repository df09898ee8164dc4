"""The oracle reproduces its stored values for seeded pixels of the tiny
workload (tests/golden/oracle_tiny_rays.json, written by
tests/golden/make_golden.py from the oracle alone): plain, YUV420, RGTC and
oval-disk queries. A regression guard: the oracle's arithmetic may change
only together with a regenerated file."""
import json
import os
import sys

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_oracle_matches_stored_values():
    sys.path.insert(0, GOLDEN)
    try:
        import make_golden
    finally:
        sys.path.remove(GOLDEN)
    with open(os.path.join(GOLDEN, "oracle_tiny_rays.json")) as f:
        want = json.load(f)
    idx, got = make_golden.render_all()
    assert idx.tolist() == want["pixels"]
    for name, w in want["cases"].items():
        g = got[name]
        assert np.array_equal(np.array(g["count"]), np.array(w["count"])), name
        assert np.abs(np.array(g["rgb"]) - np.array(w["rgb"])).max() <= 1e-12, name
        assert np.abs(np.array(g["wsum"]) - np.array(w["wsum"])).max() <= 1e-12, name
        assert (np.array(w["count"]) > 0).mean() > 0.9, name
