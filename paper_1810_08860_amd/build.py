"""Build liblf.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SO = os.path.join(HERE, "liblf.so")
HOSTCHECK_SO = os.path.join(HERE, "liblf_hostcheck.so")

SOURCES = ["lf_kernels.hip", "lf_corrector.hip", "lf_probe.hip", "lf_noalloc.hip", "lf_api.cpp", "lf_corrector_api.cpp",
           "lf_disks.cpp"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-function",
    # keep the compiler from emitting packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build(verbose: bool = False, jobs: int = 4) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    procs, objs = [], []
    for s in srcs:
        obj = os.path.join(objdir, s + ".o")
        objs.append(obj)
        cmd = [hipcc, *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), "-c", os.path.join(CSRC, s), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((s, subprocess.Popen(cmd)))
        if len(procs) >= jobs:
            _wait(procs.pop(0))
    for p in procs:
        _wait(p)
    link = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", SO + ".tmp"]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(SO + ".tmp", SO)
    # host build of the per-ray arithmetic, for CPU tests against the oracle
    hc = [hipcc, *HIPCC_FLAGS, "-shared", "-I", os.path.join(ROOT, "include"),
          os.path.join(CSRC, "lf_hostcheck.cpp"), "-o", HOSTCHECK_SO + ".tmp"]
    if verbose:
        print(" ".join(hc), flush=True)
    subprocess.run(hc, check=True)
    os.replace(HOSTCHECK_SO + ".tmp", HOSTCHECK_SO)
    return SO


def _wait(p):
    name, proc = p
    if proc.wait() != 0:
        raise RuntimeError(f"hipcc failed on {name}")


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(SO)
