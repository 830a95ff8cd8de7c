"""Build libsht.so (HIP kernels for gfx950 + host plan + C ABI) in-tree.

    python -m paper_1110_4874_amd.build

Every HIP source is compiled with packed FP32 disabled
(-Xclang -target-feature -Xclang -packed-fp32-ops); host-only sources are
compiled as plain C++ by the same driver.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libsht.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
HIP_SOURCES = ["legendre.hip", "ring.hip", "adjoint.hip", "butterfly.hip", "butterfly_adjoint.hip",
               "analysis.hip", "noalloc.hip", "interp.hip", "pol.hip"]
CXX_SOURCES = ["plan.cpp", "plan_io.cpp", "interp_plan.cpp", "api.cpp", "butterfly_plan.cpp", "batch.cpp", "queue.cpp", "pol_plan.cpp"]
COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-I", os.path.join(ROOT, "include"), "-I", CSRC]
HIP_FLAGS = ["-x", "hip", f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops", "-munsafe-fp-atomics"]
CXX_FLAGS = ["-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include", "-march=x86-64-v3"]


def _compile(src: str, obj: str, flags):
    cmd = [HIPCC] + COMMON + flags + ["-c", os.path.join(CSRC, src), "-o", obj]
    return subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True), cmd


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    objs = []
    for src in HIP_SOURCES + CXX_SOURCES:
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        flags = HIP_FLAGS if src.endswith(".hip") else CXX_FLAGS
        jobs.append((src,) + _compile(src, obj, flags))
    failed = []
    for src, proc, cmd in jobs:
        out, _ = proc.communicate()
        if verbose or proc.returncode != 0:
            sys.stderr.write(" ".join(cmd) + "\n" + (out or ""))
        if proc.returncode != 0:
            failed.append(src)
    if failed:
        raise RuntimeError("HIP build failed for: " + ", ".join(failed))
    tmp = LIB + ".tmp%d" % os.getpid()
    link = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs + ["-lpthread"]
    r = subprocess.run(link, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(link) + "\n" + r.stdout)
        raise RuntimeError("link of libsht.so failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
