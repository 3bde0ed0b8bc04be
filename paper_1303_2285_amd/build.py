"""Build libcovest.so (HIP for gfx950) in-tree with hipcc.

    python -m paper_1303_2285_amd.build        # or build() from Python

Every HIP source is compiled for gfx950 only, without fast-math (IEEE division
and no reassociation), with packed FP32 instructions disabled.  The library is
written next to this file, where the Python binding loads it.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libcovest.so")
ARCH = "gfx950"

HIP_SOURCES = ["rec_kernels.hip", "rec_mfma.hip", "hankel_kernels.hip", "adj_kernels.hip", "capon_kernels.hip", "noalloc.hip",
               "lane_kernels.hip"]
CPP_SOURCES = ["plan.cpp", "abi.cpp"]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libcovest)")


def _common_flags():
    return ["-O3", "-std=c++17", "-fPIC", "-Wall", "-I", INCLUDE, "-I", CSRC]


def _host_cxx() -> list[str]:
    """Host-only C++ (no device code): ROCm's clang with the HIP headers."""
    rocm = os.path.dirname(os.path.dirname(os.path.realpath(_hipcc())))
    clang = os.path.join(rocm, "lib", "llvm", "bin", "clang++")
    if not os.path.exists(clang):
        clang = shutil.which("clang++") or "g++"
    return [clang, "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(rocm, "include")]


def build(verbose: bool = False, jobs: int = 4) -> str:
    hipcc = _hipcc()
    with tempfile.TemporaryDirectory(prefix="covest_build_") as tmp:
        cmds = []
        objs = []
        for src in HIP_SOURCES:
            obj = os.path.join(tmp, src + ".o")
            objs.append(obj)
            cmds.append([hipcc, *_common_flags(), f"--offload-arch={ARCH}",
                         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                         "-c", os.path.join(CSRC, src), "-o", obj])
        for src in CPP_SOURCES:
            obj = os.path.join(tmp, src + ".o")
            objs.append(obj)
            cmds.append([*_host_cxx(), *_common_flags(),
                         "-c", os.path.join(CSRC, src), "-o", obj])
        procs = []
        for cmd in cmds:
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                                stderr=subprocess.STDOUT, text=True)))
            if len(procs) >= jobs:
                _drain(procs.pop(0), verbose)
        while procs:
            _drain(procs.pop(0), verbose)
        tmp_lib = os.path.join(tmp, "libcovest.so")
        link = [hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp_lib]
        if verbose:
            print(" ".join(link), flush=True)
        _run(link, verbose)
        shutil.copyfile(tmp_lib, LIB + ".tmp")
        os.replace(LIB + ".tmp", LIB)
    return LIB


def _drain(item, verbose):
    cmd, p = item
    out, _ = p.communicate()
    if p.returncode != 0:
        raise RuntimeError(f"build failed: {' '.join(cmd)}\n{out}")
    if verbose and out.strip():
        print(out, flush=True)


def _run(cmd, verbose):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if p.returncode != 0:
        raise RuntimeError(f"build failed: {' '.join(cmd)}\n{p.stdout}")
    if verbose and p.stdout.strip():
        print(p.stdout, flush=True)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
