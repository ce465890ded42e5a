"""Builds liblst.so (HIP for gfx950) in-tree.

Usage: python -m paper_2407_18231_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblst.so")
PROBE = os.path.join(HERE, "sync_probe")
LINK_PROBE = os.path.join(HERE, "link_probe")
SOURCES = ["geometry.cpp", "kernels.hip", "api.hip"]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # IEEE binary32 cut arithmetic: no FMA contraction, correctly rounded
    # division and square root, denormals kept
    "-ffp-contract=off", "-fhip-fp32-correctly-rounded-divide-sqrt",
    "-fno-gpu-flush-denormals-to-zero",
    # no packed-FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def _torch_hip_dir():
    """Directory of the HIP runtime PyTorch ships, if PyTorch is installed.

    A process holds one HIP runtime: linking against the one PyTorch loads
    lets torch tensors (device memory, streams) and this library share a
    process."""
    try:
        import importlib.util
        spec = importlib.util.find_spec("torch")
    except Exception:
        spec = None
    if spec is None or not spec.origin:
        return None
    d = os.path.join(os.path.dirname(spec.origin), "lib")
    return d if os.path.exists(os.path.join(d, "libamdhip64.so")) else None


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc, *FLAGS, "-c", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
               os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp"
    tdir = _torch_hip_dir()
    if tdir:
        link = ["g++", "-shared", "-o", tmp, *objs, "-L" + tdir, "-l:libamdhip64.so",
                "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx",
                "-Wl,-rpath," + tdir + ":/opt/rocm/lib", "-lpthread"]
    else:
        link = [hipcc, "--offload-arch=gfx950", "-shared", "-o", tmp, *objs, "-L/opt/rocm/lib",
                "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib", "-lpthread"]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.check_call(link)
    os.replace(tmp, LIB)
    # the stage-boundary probe (a program of its own; bench.py runs it)
    probe = [hipcc, "--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops", os.path.join(CSRC, "sync_probe.hip"), "-o", PROBE + ".tmp"]
    if verbose:
        print(" ".join(probe), flush=True)
    subprocess.check_call(probe)
    os.replace(PROBE + ".tmp", PROBE)
    # the host-link probe (bench.py runs it too)
    link = [hipcc, "--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
            "-packed-fp32-ops", os.path.join(CSRC, "link_probe.hip"), "-o", LINK_PROBE + ".tmp"]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.check_call(link)
    os.replace(LINK_PROBE + ".tmp", LINK_PROBE)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
