"""Compile libaop.so (gfx950) in place with hipcc.

Every HIP source is built with packed-FP32 instructions disabled; the library
is written next to this file so that it travels with the source tree.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libaop.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

SOURCES = ["aop_solver.hip", "aop_plain.hip", "aop_approx.hip", "aop_api.cpp", "aop_serve.cpp"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-I", INCLUDE, "-I", CSRC]
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _compile(src: str, obj: str) -> None:
    cmd = [HIPCC] + COMMON + DEVICE + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed on %s" % os.path.basename(src))


CPU_SRC = os.path.join(CSRC, "aop_cpu.cpp")
CPU_LIB = os.path.join(HERE, "libaop_cpu.so")


def build_cpu(verbose: bool = False) -> str:
    """Compile libaop_cpu.so (the host multicore form of the method) with g++ and OpenMP."""
    tmp = CPU_LIB + ".tmp%d" % os.getpid()
    cmd = ["g++", "-O3", "-std=c++17", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared", "-Wall",
           "-I", INCLUDE, "-o", tmp, CPU_SRC]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("g++ failed on aop_cpu.cpp")
    os.replace(tmp, CPU_LIB)
    if verbose:
        print("built", CPU_LIB)
    return CPU_LIB


def build(verbose: bool = False) -> str:
    """Compile every source and link libaop.so, and libaop_cpu.so; always rebuilds."""
    build_cpu(verbose)
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    jobs = []
    for s in SOURCES:
        src = os.path.join(CSRC, s)
        if not os.path.exists(src):
            continue
        jobs.append((src, os.path.join(objdir, s + ".o")))
    with ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        list(ex.map(lambda j: _compile(*j), jobs))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + [o for _, o in jobs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link failed")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
