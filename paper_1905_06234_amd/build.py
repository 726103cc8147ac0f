"""Compile the HIP library (liblife.so) for gfx950, in-tree."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "liblife.so")
SOURCES = ["life_plan.cpp", "life_device.hip", "life_plan_gpu.hip"]

# Packed FP32 instructions are kept out of the generated code on purpose.
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-command-line-argument"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(out: str = LIB, extra=(), quiet: bool = True) -> str:
    """Compile every source to an object (in parallel), then link liblife.so."""
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tag = f".tmp{os.getpid()}"
    objs = [out + f".{i}{tag}.o" for i in range(len(srcs))]
    flags = [f for f in HIP_FLAGS if f != "-shared"]
    procs = [subprocess.Popen([hipcc(), *flags, *extra, "-I", INCLUDE, "-I", CSRC, "-c", src, "-o", obj],
                              stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)
             for src, obj in zip(srcs, objs)]
    errs = []
    for src, p in zip(srcs, procs):
        so, se = p.communicate()
        if p.returncode != 0:
            errs.append(f"{src}:\n{so}{se}")
        elif not quiet:
            sys.stderr.write(se)
    try:
        if errs:
            sys.stderr.write("\n".join(errs))
            raise RuntimeError("hipcc failed to compile " + ", ".join(SOURCES))
        tmp = out + tag
        cmd = [hipcc(), *HIP_FLAGS, *extra, *objs, "-o", tmp]
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("hipcc failed: " + " ".join(cmd))
        os.replace(tmp, out)
    finally:
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
    return out


if __name__ == "__main__":
    print(build(quiet=False))
