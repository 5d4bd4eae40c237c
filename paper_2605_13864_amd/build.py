"""Builds libxtr.so (the HIP kernels and the C ABI) for gfx950 with hipcc.

    python -m paper_2605_13864_amd.build [--jobs N] [--save-temps DIR]

Every source under csrc/ is compiled to an object file in _build/ and the
objects are linked into paper_2605_13864_amd/libxtr.so next to this file.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libxtr.so")
ARCH = os.environ.get("XTR_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for c in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"),
              shutil.which("hipcc") or ""):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found (set ROCM_PATH)")


FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-fno-gpu-rdc",
    "-ffp-contract=off", "-Wall", "-Wno-unused-function",
    # packed fp32 instructions off: some of their forms have given silently wrong results
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    f"-I{os.path.join(ROOT, 'include')}",
]


def compile_one(src: str, extra=()) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [hipcc(), *FLAGS, *extra, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    if r.stderr.strip():
        # hipcc's host pass warns about the device-only target feature; keep real warnings
        lines = [ln for ln in r.stderr.splitlines() if "packed-fp32-ops" not in ln]
        if any(ln.strip() for ln in lines):
            sys.stderr.write("\n".join(lines) + "\n")
    return obj


def build(jobs: int = 8, save_temps: str | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    # longest compiles first (the transpose units), so the pool stays busy
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")), key=lambda f: -os.path.getsize(f))
    srcs.sort(key=lambda f: not os.path.basename(f).startswith("tpose_"))
    extra = []
    if save_temps:
        os.makedirs(save_temps, exist_ok=True)
        extra = ["-save-temps"]      # intermediates land in the current directory
    cwd = os.getcwd()
    if save_temps:
        os.chdir(save_temps)
    try:
        with cf.ThreadPoolExecutor(max(1, jobs)) as ex:
            objs = list(ex.map(lambda s: compile_one(s, extra), srcs))
    finally:
        os.chdir(cwd)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs,
           f"-Wl,-rpath,{os.path.join(os.environ.get('ROCM_PATH', '/opt/rocm'), 'lib')}"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=8)
    ap.add_argument("--save-temps", default=None)
    a = ap.parse_args()
    print(build(a.jobs, a.save_temps))
