"""Compile the HIP library ``libdpvr.so`` in-tree for gfx950 with hipcc.

Usage: ``python -m paper_2501_01628_amd.build`` (or ``__graft_entry__.build()``).
Every call recompiles.  Objects go to ``_build/`` next to this file.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libdpvr.so")
BUILD = os.path.join(HERE, "_build")
ROOT = os.path.dirname(HERE)

ARCH = os.environ.get("DPVR_OFFLOAD_ARCH", "gfx950")
KERNEL_SOURCES = ["march.hip", "adjoint.hip", "composite.hip", "ingest.hip", "static_scratch.hip", "rqc.hip", "tets.hip"]
HOST_SOURCES = ["api.cpp", "tet_build.cpp"]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libdpvr.so)")


def _common():
    # code object v5: loadable by the HIP runtime torch ships as well as /opt/rocm's
    return ["-O3", "-fPIC", "-std=c++17", "-Wall", "-mcode-object-version=5",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _compile(args):
    cmd, src = args
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return r.stderr


def build(verbose: bool = False) -> str:
    hipcc = _hipcc()
    os.makedirs(BUILD, exist_ok=True)
    jobs, objs = [], []
    for src in KERNEL_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        cmd = [hipcc, "-x", "hip", f"--offload-arch={ARCH}", *_common(),
               # packed FP32 (v_pk_*_f32) is kept out of every kernel
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-munsafe-fp-atomics", "-c", os.path.join(CSRC, src), "-o", obj]
        jobs.append((cmd, src))
        objs.append(obj)
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        cmd = [hipcc, *_common(), "-ffp-contract=off", "-c", os.path.join(CSRC, src), "-o", obj]
        jobs.append((cmd, src))
        objs.append(obj)
    with ThreadPoolExecutor(min(8, len(jobs))) as ex:
        for err in ex.map(_compile, jobs):
            if verbose and err.strip():
                print(err, file=sys.stderr)
    tmp = OUT + ".tmp"
    link = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    _compile((link, "libdpvr.so"))
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
