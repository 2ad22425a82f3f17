"""Build libcurldiv.so (HIP, gfx950) in the package directory.

Objects go to ``_build/`` at the repository root; the shared library is
written atomically next to this file so that a failed build never leaves a
half-written library behind.
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libcurldiv.so")
SOURCES = ["csrc/setup.cpp", "csrc/kernels.hip", "csrc/coarse.hip", "csrc/loadvec.hip", "csrc/solver.hip"]
# the operator kernels: one object per (source, precision, half bandwidth)
APPLY_SOURCES = ["csrc/apply2d.hip", "csrc/apply3d.hip"]
APPLY_VARIANTS = [(t, hb) for t in ("double", "float") for hb in range(1, 7)]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    "-I", os.path.join(ROOT, "include"),
]


def _compile(job):
    src, defs = job
    tag = "".join(f"_{v}" for _, v in defs)
    obj = os.path.join(BUILD, os.path.basename(src) + tag + ".o")
    cmd = [HIPCC] + FLAGS + [f"-D{k}={v}" for k, v in defs] + ["-c", os.path.join(HERE, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    jobs = [(src, [("CD_T", t), ("CD_HB", hb)]) for src in APPLY_SOURCES for t, hb in APPLY_VARIANTS]
    jobs += [(src, []) for src in SOURCES]
    workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(_compile, jobs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    shutil.move(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
