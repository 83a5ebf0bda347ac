"""Compiles the HIP library ``libgp_ssm.so`` in-tree for gfx950.

Usage: ``python -m paper_2601_02527_amd.build`` (or ``build()`` from Python).
Every call recompiles.  Objects go to ``_build/`` at the repository root.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libgp_ssm.so")
BUILD = os.path.join(ROOT, "_build")

ARCH = os.environ.get("GP_SSM_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")

DEVICE_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]
HOST_FLAGS = ["-O3", "-std=c++17", "-fPIC"]

HIP_SOURCES = ["capi.hip", "scan.hip", "kernels_m1.hip", "kernels_m2.hip", "kernels_m3.hip", "kernels_m4.hip",
               "kernels_m1i.hip", "kernels_m2i.hip", "kernels_m3i.hip", "kernels_m4i.hip",
               "kernels_m1x.hip", "kernels_m2x.hip", "kernels_m3x.hip", "kernels_m4x.hip"]
CPP_SOURCES = ["plan.cpp"]


def build(verbose: bool = True, jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    t0 = time.time()
    procs = []
    objs = []
    for src in CPP_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        cmd = ["g++"] + HOST_FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((src, cmd))
        objs.append(obj)
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        cmd = [HIPCC] + DEVICE_FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((src, cmd))
        objs.append(obj)
    jobs = jobs or max(1, min(len(procs), os.cpu_count() or 4))
    running = []
    errors = []
    queue = list(procs)
    while queue or running:
        while queue and len(running) < jobs:
            src, cmd = queue.pop(0)
            p = subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
            running.append((src, cmd, p))
        src, cmd, p = running.pop(0)
        out, _ = p.communicate()
        if p.returncode != 0:
            errors.append((src, " ".join(cmd), out))
        elif verbose and out.strip():
            lines = [ln for ln in out.splitlines() if "packed-fp32-ops" not in ln and "unknown target feature" not in ln
                     and ln.strip() and not ln.strip().startswith("1 warning")]
            if lines:
                print("\n".join(lines[:40]), file=sys.stderr)
    if errors:
        for src, cmd, out in errors:
            print(f"--- compile failed: {src}\n{cmd}\n{out}", file=sys.stderr)
        raise RuntimeError("HIP build failed: " + ", ".join(e[0] for e in errors))
    tmp = OUT + ".tmp%d" % os.getpid()
    link = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs + ["-lpthread"]
    r = subprocess.run(link, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + " ".join(link) + "\n" + r.stdout)
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT} in {time.time() - t0:.1f}s", file=sys.stderr)
    return OUT


if __name__ == "__main__":
    build()
