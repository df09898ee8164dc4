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


# host-code sanitizers for a checking build (sanitized_build): each -fsanitize=
# is preceded by -Xarch_host, so device code is compiled as usual
SANITIZE_HOST_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
                       "-shared-libsan"]


def sanitized_build(out_dir: str, jobs: int = 4) -> tuple[str, str]:
    """liblf.so and liblf_hostcheck.so built into out_dir with AddressSanitizer
    and UBSan on their host code (for CPU tests of argument checking, the oval
    disk extents and the per-ray host arithmetic); returns their paths."""
    return build(jobs=jobs, out_dir=out_dir, extra=SANITIZE_HOST_FLAGS)


def build(verbose: bool = False, jobs: int = 4, out_dir: str | None = None, extra: list | None = None) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    extra = list(extra or [])
    so = os.path.join(out_dir, "liblf.so") if out_dir else SO
    hostcheck_so = os.path.join(out_dir, "liblf_hostcheck.so") if out_dir else HOSTCHECK_SO
    objdir = os.path.join(out_dir, "_build") if out_dir else os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    procs, objs = [], []
    for s in srcs:
        obj = os.path.join(objdir, s + ".o")
        objs.append(obj)
        cmd = [hipcc, *HIPCC_FLAGS, *extra, "-I", os.path.join(ROOT, "include"), "-c", os.path.join(CSRC, s), "-o",
               obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((s, subprocess.Popen(cmd)))
        if len(procs) >= jobs:
            _wait(procs.pop(0))
    for p in procs:
        _wait(p)
    link = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *extra, *objs, "-o", so + ".tmp"]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(so + ".tmp", so)
    # host build of the per-ray arithmetic, for CPU tests against the oracle
    hc = [hipcc, *HIPCC_FLAGS, *extra, "-shared", "-I", os.path.join(ROOT, "include"),
          os.path.join(CSRC, "lf_hostcheck.cpp"), "-o", hostcheck_so + ".tmp"]
    if verbose:
        print(" ".join(hc), flush=True)
    subprocess.run(hc, check=True)
    os.replace(hostcheck_so + ".tmp", hostcheck_so)
    return (so, hostcheck_so) if out_dir else so


def _wait(p):
    name, proc = p
    if proc.wait() != 0:
        raise RuntimeError(f"hipcc failed on {name}")


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(SO)
