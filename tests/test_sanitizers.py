"""The host code under AddressSanitizer and UBSan, on the CPU: the FP64
oracle (oracle.c, conv_oracle.c, built with gcc) runs its pins, and the
library's host code (argument checks of every entry point, the oval disk
extents, the per-ray arithmetic's host build; built with hipcc, sanitizers on
the host side only) runs the ABI, extent and host-ray tests, each in a
subprocess with its sanitizer runtime preloaded (the Python interpreter is not
instrumented). A canary library with a planted heap overflow shows each setup
catches one."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")
GCC_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fPIC", "-shared", "-std=c11", "-D_GNU_SOURCE"]
GCC_SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]
ENV = {"ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1", "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}

CANARY = r"""
#include <stdlib.h>
#ifdef __cplusplus
extern "C"
#endif
int canary(int n) { int *p = (int *)malloc(sizeof(int) * n); p[n] = 1; int r = p[0]; free(p); return r; }
"""


def _gcc_runtime():
    out = []
    for lib in ("libasan.so", "libubsan.so"):
        p = subprocess.run(["gcc", f"-print-file-name={lib}"], capture_output=True, text=True).stdout.strip()
        if not os.path.isabs(p) or not os.path.exists(p):
            pytest.skip(f"gcc's {lib} is not installed")
        out.append(p)
    return ":".join(out)


def _clang_runtime():
    import glob
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not hits:
        pytest.skip("clang's AddressSanitizer runtime is not installed")
    return hits[-1]


def _run(args, env_extra, timeout=900):
    env = dict(os.environ, **ENV, **env_extra)
    return subprocess.run(args, cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)


def _canary_caught(so, preload):
    code = f"import ctypes; ctypes.CDLL({so!r}).canary(4)"
    r = _run([sys.executable, "-c", code], {"LD_PRELOAD": preload}, timeout=120)
    return r.returncode != 0 and "AddressSanitizer" in r.stderr and "heap-buffer-overflow" in r.stderr


def test_oracle_pins_under_asan_and_ubsan(tmp_path):
    rt = _gcc_runtime()
    src = tmp_path / "canary.c"
    src.write_text(CANARY)
    canary = tmp_path / "libcanary.so"
    subprocess.run(["gcc", *GCC_FLAGS, *GCC_SAN, str(src), "-o", str(canary)], check=True)
    assert _canary_caught(str(canary), rt)
    so = tmp_path / "liboracle.so"
    subprocess.run(["gcc", *GCC_FLAGS, *GCC_SAN, "-fopenmp", os.path.join(ORACLE, "oracle.c"),
                    os.path.join(ORACLE, "conv_oracle.c"), "-o", str(so), "-lm"], check=True)
    pins = ["tests/test_oracle_pins.py", "tests/test_oracle_prefilter.py", "tests/test_oracle_paging.py",
            "tests/test_oracle_yuv.py", "tests/test_oracle_rgtc.py", "tests/test_oracle_ovals.py",
            "tests/test_conv_oracle.py"]
    r = _run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu", *pins],
             {"LD_PRELOAD": rt, "LF_ORACLE_LIB": str(so), "OMP_NUM_THREADS": "8"})
    tail = r.stdout.strip().splitlines()[-1] if r.stdout.strip() else ""
    print("oracle under ASan/UBSan:", tail)
    assert r.returncode == 0 and "passed" in tail, r.stdout[-3000:] + r.stderr[-3000:]


def test_library_host_code_under_asan_and_ubsan(tmp_path):
    rt = _clang_runtime()
    from paper_1810_08860_amd import build
    src = tmp_path / "canary.cpp"
    src.write_text(CANARY)
    canary = tmp_path / "libcanary.so"
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    subprocess.run([hipcc, "-shared", "-fPIC", *build.SANITIZE_HOST_FLAGS, "-x", "c++", str(src), "-o", str(canary)],
                   check=True, capture_output=True)
    r = _run([sys.executable, "-c", "import ctypes; ctypes.CDLL(%r).canary(4)" % str(canary)], {"LD_PRELOAD": rt},
             timeout=120)
    assert r.returncode != 0 and "AddressSanitizer" in r.stderr, r.stderr[-2000:]
    lib, hostcheck = build.sanitized_build(str(tmp_path / "san"))
    tests = ["tests/test_abi.py", "tests/test_disk_extents.py", "tests/test_host_ray.py"]
    r = _run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu", *tests],
             {"LD_PRELOAD": rt, "LF_LIB": lib, "LF_HOSTCHECK_LIB": hostcheck})
    tail = r.stdout.strip().splitlines()[-1] if r.stdout.strip() else ""
    print("library host code under ASan/UBSan:", tail)
    assert r.returncode == 0 and "passed" in tail, r.stdout[-3000:] + r.stderr[-3000:]
