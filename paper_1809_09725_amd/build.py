"""Build librt4d.so for gfx950 with hipcc (in-tree, no JIT cache).

Usage: python -m paper_1809_09725_amd.build [--jobs N] [--sanitize]

--sanitize also writes _build/sanitize/librt4d.so: the host sources (plan,
ABI, solver, timing, out-of-core driver) built with AddressSanitizer and
UndefinedBehaviorSanitizer (host code only: each -fsanitize= follows
-Xarch_host), linked with the regular device objects.  Load it in a process
with the clang ASan runtime preloaded and RT4D_LIBRARY pointing at it.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build", "rt4d")
LIB = os.path.join(HERE, "librt4d.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

SOURCES = ["plan.cpp", "abi.cpp", "solve.cpp", "timing.cpp", "proj_pf.hip", "backproject.hip", "proj_sf.hip", "tv.hip",
           "reduce.hip", "fbp.hip", "ooc.cpp", "calib.hip"]

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-I", os.path.join(ROOT, "include"), "-I", CSRC,
          # packed FP32 instructions stay off (v_pk_{add,mul,fma}_f32)
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-function"]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, *COMMON, "-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd[1:1] = ["-ffp-contract=off"]   # host tables: plain IEEE operations
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-6000:]}")
    if r.stderr.strip():
        sys.stderr.write(r.stderr)
    return obj


def build(jobs: int = 6, verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


SANITIZE_DIR = os.path.join(ROOT, "_build", "sanitize")
SANITIZE_LIB = os.path.join(SANITIZE_DIR, "librt4d.so")
SANITIZE_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer",
                  "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]


def asan_runtime() -> str | None:
    """The clang ASan runtime that a sanitized library needs preloaded."""
    import glob
    hits = glob.glob("/opt/rocm*/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    return sorted(hits)[-1] if hits else None


def build_sanitized(jobs: int = 6) -> str:
    """The host sources with ASan + UBSan, linked with build()'s device
    objects (built first if any is missing)."""
    if not all(os.path.exists(os.path.join(BUILD, s + ".o")) for s in SOURCES):
        build(jobs, verbose=False)
    os.makedirs(SANITIZE_DIR, exist_ok=True)
    host = [s for s in SOURCES if s.endswith(".cpp")]

    def one(src: str) -> str:
        obj = os.path.join(SANITIZE_DIR, src + ".o")
        flags = [f for f in COMMON if f != "-O3"]
        cmd = [HIPCC, "-ffp-contract=off", *SANITIZE_FLAGS, *flags, "-c",
               os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-6000:]}")
        return obj

    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(one, host))
    dev = [os.path.join(BUILD, s + ".o") for s in SOURCES if not s.endswith(".cpp")]
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-Xarch_host", "-fsanitize=address",
           "-Xarch_host", "-fsanitize=undefined", "-shared-libasan", "-o", SANITIZE_LIB, *objs, *dev]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"sanitized link failed:\n{r.stderr[-4000:]}")
    return SANITIZE_LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=6)
    ap.add_argument("--sanitize", action="store_true")
    a = ap.parse_args()
    build(a.jobs)
    if a.sanitize:
        print(f"built {build_sanitized(a.jobs)}")
