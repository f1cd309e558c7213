"""Host-sanitizer build of libhlb: AddressSanitizer and UndefinedBehaviorSanitizer on the HOST
code only (argument checks, planner, tuning table, workspace and batch bookkeeping); device
code is compiled exactly as in the normal build.

``python -m paper_2503_16080_amd._sanitize`` writes ``libhlb_asan.so`` next to the package.
Load it by setting ``HLB_LIBRARY`` to its path and preloading the compiler's shared ASan
runtime (``asan_runtime()``) into the process, e.g. for the CPU-only ABI tests.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

from . import _build

OBJDIR = os.path.join(_build.HERE, "_build_asan")
LIB = os.path.join(_build.HERE, "libhlb_asan.so")

# every sanitizer flag applies to the host compilation only
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
            "-Xarch_host", "-g"]


def asan_runtime() -> str:
    """The clang shared ASan runtime matching hipcc (to LD_PRELOAD into a Python process)."""
    llvm = os.path.join(os.path.dirname(os.path.dirname(os.path.realpath(_build.HIPCC))), "llvm")
    cands = sorted(glob.glob(os.path.join(llvm, "lib", "clang", "*", "lib", "linux", "libclang_rt.asan-x86_64.so")))
    cands += sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not cands:
        raise FileNotFoundError("libclang_rt.asan-x86_64.so not found next to hipcc")
    return cands[-1]


def _compile(src: str) -> str:
    obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
    cmd = [_build.HIPCC, *_build.COMMON, *HOST_SAN, "-c", os.path.join(_build.CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(jobs: int | None = None) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = jobs or min(len(_build.SOURCES), os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, _build.SOURCES))
    tmp = LIB + ".tmp"
    # link line: no device compilation happens here, and the sanitizer runtimes are host-only
    cmd = [_build.HIPCC, "-shared", "-fPIC", f"--offload-arch={_build.ARCH}", "-fno-gpu-sanitize",
           "-fsanitize=address,undefined", "-shared-libasan", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
    sys.exit(0)
