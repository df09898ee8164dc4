"""The oracle's pins catch plausible mistakes: each case below plants one
mistake in a copy of oracle/oracle.c (a dropped half-pixel, a wrong sign or
index, a transposed frame, a wrong triangle split, a missing test, a wrong
weight), builds that copy into its own library and runs the pins that cover
the changed part against it in a separate process; at least one pin must fail.
The real oracle is never modified."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")
PINS = "tests/test_oracle_pins.py"

# name: (pin file, [(text in oracle.c, replacement), ...])
MUTATIONS = {
    "eye ray through the pixel corner": (PINS, [(
        "double X = (2.0 * pxy[2 * k] / W - 1.0) * tx;",
        "double X = (2.0 * (pxy[2 * k] - 0.5) / W - 1.0) * tx;")]),
    "eye ray Y axis flipped": (PINS, [(
        "double Y = (1.0 - 2.0 * pxy[2 * k + 1] / H) * ty;",
        "double Y = (2.0 * pxy[2 * k + 1] / H - 1.0) * ty;")]),
    "falloff in the squared radius": (PINS, [(
        "*rho_out = 1.0 - sqrt(uu * uu + vv * vv) / V->disk_radius;",
        "*rho_out = 1.0 - (uu * uu + vv * vv) / (V->disk_radius * V->disk_radius);")]),
    "view frame transposed": (PINS, [
        ("o[0] = R[0] * x[0] + R[3] * x[1] + R[6] * x[2];", "o[0] = R[0] * x[0] + R[1] * x[1] + R[2] * x[2];"),
        ("o[1] = R[1] * x[0] + R[4] * x[1] + R[7] * x[2];", "o[1] = R[3] * x[0] + R[4] * x[1] + R[5] * x[2];"),
        ("o[2] = R[2] * x[0] + R[5] * x[1] + R[8] * x[2];", "o[2] = R[6] * x[0] + R[7] * x[1] + R[8] * x[2];")]),
    "cells split along the other diagonal": (PINS, [
        ("if (tri_hit(o, e, v00, v10, v11, &t) && t > 0.0 && t < *best) *best = t;",
         "if (tri_hit(o, e, v00, v10, v01, &t) && t > 0.0 && t < *best) *best = t;"),
        ("if (tri_hit(o, e, v00, v11, v01, &t) && t > 0.0 && t < *best) *best = t;",
         "if (tri_hit(o, e, v10, v11, v01, &t) && t > 0.0 && t < *best) *best = t;")]),
    "back-facing disks accepted": (PINS, [(
        "if (!(a > 0.0)) { *u_out = *v_out = *rho_out = NAN; return; }",
        "if (!(a != 0.0)) { *u_out = *v_out = *rho_out = NAN; return; }")]),
    "bilinear weight of the wrong axis": (PINS, [(
        "double top = p00[a] + fx * ((double)p10[a] - p00[a]);",
        "double top = p00[a] + fy * ((double)p10[a] - p00[a]);")]),
    "denominator counts views instead of weights": (PINS, [("ws += r.rho;", "ws += 1.0;")]),
    "mesh vertices at depth-pixel corners": (PINS, [(
        "double X = (2.0 * (j + 0.5) / M - 1.0) * ts;",
        "double X = (2.0 * j / M - 1.0) * ts;")]),
    "texel centres at integers": (PINS, [(
        "double px = (Xs / ts + 1.0) * 0.5 * W - 0.5;",
        "double px = (Xs / ts + 1.0) * 0.5 * W;")]),
    "traversal without dilation": (PINS, [
        ("for (int64_t kk = ck - 1; kk <= ck + 1; ++kk)", "for (int64_t kk = ck; kk <= ck; ++kk)"),
        ("for (int64_t jj = cj - 1; jj <= cj + 1; ++jj)", "for (int64_t jj = cj; jj <= cj; ++jj)")]),
    "traversal steps x without advancing": (PINS, [("cj += sx; tmx += tdx;", "cj += sx;")]),
    "chroma mean truncated": ("tests/test_oracle_yuv.py", [
        ("ci[2 * ((int64_t)by * (W / 2) + bx)] = (uint8_t)((sb + 2) >> 2);",
         "ci[2 * ((int64_t)by * (W / 2) + bx)] = (uint8_t)(sb >> 2);")]),
    "RGTC codes off by one": ("tests/test_oracle_rgtc.py", [(
        "const uint64_t code = p == 0 ? 0 : (p == 7 ? 1 : (uint64_t)(p + 1));",
        "const uint64_t code = p == 0 ? 0 : (p == 7 ? 1 : (uint64_t)p);")]),
    "RGTC texel codes read in the wrong order": ("tests/test_oracle_rgtc.py", [(
        "const int32_t c = (int32_t)((bits >> (3 * t)) & 7u);",
        "const int32_t c = (int32_t)((bits >> (3 * (15 - t))) & 7u);")]),
    "tile of the second tap column ignored": ("tests/test_oracle_paging.py", [(
        "tiles[1] = (y0 / P) * tw + x1 / P;", "tiles[1] = (y0 / P) * tw + x0 / P;")]),
    "prefilter aperture without falloff": ("tests/test_oracle_prefilter.py", [(
        "const double rho = 1.0 - sqrt(du * du + dv * dv);", "const double rho = 1.0;")]),
    "oval prefilter aperture without the quadrant area factor": ("tests/test_oracle_prefilter.py", [(
        "const double wgt = ext ? rho * sigma * su * sv : rho * sigma;", "const double wgt = rho * sigma;")]),
    "oval prefilter aperture maps u by the opposite quadrant": ("tests/test_oracle_prefilter.py", [(
        "const double su = ext ? (du >= 0.0 ? ext[0] : ext[1]) : radius;",
        "const double su = ext ? (du >= 0.0 ? ext[1] : ext[0]) : radius;")]),
}


@pytest.mark.parametrize("name", list(MUTATIONS))
def test_planted_mistake_fails_a_pin(name, tmp_path):
    pins, edits = MUTATIONS[name]
    with open(os.path.join(ORACLE, "oracle.c")) as f:
        src = f.read()
    for old, new in edits:
        assert src.count(old) == 1, f"mutation site not found once: {old}"
        src = src.replace(old, new)
    mutated = tmp_path / "oracle.c"
    mutated.write_text(src)
    so = tmp_path / "liboracle.so"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-D_GNU_SOURCE", str(mutated),
                    os.path.join(ORACLE, "conv_oracle.c"), "-o", str(so), "-lm"], check=True)
    env = dict(os.environ, LF_ORACLE_LIB=str(so), OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu", pins],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    tail = r.stdout.strip().splitlines()[-1] if r.stdout.strip() else r.stderr[-300:]
    print(f"{name}: {tail}")
    assert r.returncode == 1 and "failed" in tail, r.stdout[-2000:] + r.stderr[-2000:]
