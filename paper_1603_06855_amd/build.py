"""Builds libphx.so in-tree: the HIP sources under csrc/ for gfx950 with hipcc, the plain
C++ host module (no GPU code) with the host compiler, linked by hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = ["dense.hip", "physics.hip", "small.hip", "design.hip", "runtime.hip"]
HOST_SOURCES = ["host.cpp"]
LIB = os.path.join(HERE, "libphx.so")


def build(verbose: bool = False, jobs: int = 4) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    flags = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(HERE, "csrc")]
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        objs.append(obj)
        cmd = [hipcc, *flags, "-c", os.path.join(HERE, "csrc", src), "-o", obj]
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
        while len([p for _, p in procs if p.poll() is None]) >= jobs:
            procs[[i for i, (_, p) in enumerate(procs) if p.poll() is None][0]][1].wait()
    cxx = os.environ.get("CXX", "g++")
    for src in HOST_SOURCES:
        obj = os.path.join(objdir, src.replace(".cpp", ".o"))
        objs.append(obj)
        cmd = [cxx, "-O2", "-std=c++17", "-fPIC", "-Wall", "-I" + os.path.join(ROOT, "include"),
               "-c", os.path.join(HERE, "csrc", src), "-o", obj]
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
        while len([p for _, p in procs if p.poll() is None]) >= jobs:
            procs[[i for i, (_, p) in enumerate(procs) if p.poll() is None][0]][1].wait()
    for cmd, p in procs:
        out, _ = p.communicate()
        msgs = [ln for ln in out.splitlines() if "packed-fp32-ops" not in ln]
        if p.returncode != 0:
            raise RuntimeError("compile failed:\n" + " ".join(cmd) + "\n" + "\n".join(msgs))
        if verbose and msgs:
            print("\n".join(msgs), file=sys.stderr)
    tmp = LIB + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
