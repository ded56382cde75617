"""Build libgpe.so for gfx950 with hipcc (objects compiled in parallel).

    python paper_1504_02891_amd/csrc/build.py [--jobs N]

The shared library lands next to the Python binding
(paper_1504_02891_amd/libgpe.so); objects go to <repo>/_build/.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libgpe.so")

ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # kernel arguments arrive in scalar registers at dispatch (no load round
    # trip before the first descriptor read); older firmware runs the
    # compiler's fallback prologue instead
    "-mllvm", "-amdgpu-kernarg-preload-count=16",
    "-I", os.path.join(ROOT, "include"), "-I", HERE,
    "-Wno-unused-result",
]


def units():
    out = []
    for role in range(4):
        for prec in (0, 1):
            out.append(("k_solver_role.hip", f"solver_r{role}_p{prec}",
                        [f"-DGPE_ROLE={role}", f"-DGPE_PREC64={prec}"]))
            out.append(("k_apply_role.hip", f"apply_r{role}_p{prec}",
                        [f"-DGPE_ROLE={role}", f"-DGPE_FP64={prec}"]))
    for name in ("k_step", "k_dispatch", "k_noalloc", "api"):
        out.append((f"{name}.hip", name, []))
    return out


def hipcc():
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found (ROCm toolchain required)")
    return exe


def compile_one(cc, src, obj, extra):
    cmd = [cc, *FLAGS, *extra, "-c", os.path.join(HERE, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src} {extra}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(jobs: int | None = None, verbose: bool = True) -> str:
    cc = hipcc()
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or max(1, min(16, os.cpu_count() or 4))
    t0 = time.time()
    objs = []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = []
        for src, tag, extra in units():
            obj = os.path.join(BUILD, tag + ".o")
            futs.append(ex.submit(compile_one, cc, src, obj, extra))
        for f in futs:
            objs.append(f.result())
    tmp = LIB + ".tmp"
    r = subprocess.run([cc, "-shared", f"--offload-arch={ARCH}", "-fPIC", "-o", tmp, *objs],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} in {time.time() - t0:.1f}s", flush=True)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    a = ap.parse_args()
    try:
        build(a.jobs)
    except RuntimeError as e:
        print(e, file=sys.stderr)
        sys.exit(1)
