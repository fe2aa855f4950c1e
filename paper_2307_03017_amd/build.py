"""Build libhsgd.so in-tree for gfx950 with hipcc.

    python -m paper_2307_03017_amd.build        # or: from paper_2307_03017_amd.build import build

Objects go to _build/ at the repository root; the shared library lands next to this file
(paper_2307_03017_amd/libhsgd.so), where the Python binding loads it from.
"""

from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libhsgd.so")
# a plain-C program driving the library through include/hsgd.h alone (run by the GPU tests)
C_SMOKE_SRC = os.path.join(ROOT, "tests", "hsgd_c_smoke.c")
C_SMOKE = os.path.join(PKG, "hsgd_c_smoke")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

# Device code: wave64 gfx950; packed-FP32 instructions disabled; FP32 denormals kept (the
# selection scores are specified in exact IEEE float32); hardware float atomics.
DEVICE_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fno-gpu-flush-denormals-to-zero", "-munsafe-fp-atomics",
    "-Wall", "-Wno-unused-function",
]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-D__HIP_PLATFORM_AMD__"]

SOURCES = [
    ("hsgd_kernels.hip", "device"),
    ("hsgd_psv.hip", "device"),
    ("hsgd_noalloc.hip", "device"),
    ("hsgd_api.cpp", "host"),
    ("hsgd_host.cpp", "host"),
    ("hsgd_profile.cpp", "host"),
    ("hsgd_batch.cpp", "host"),
]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + r.stdout)
    return r.stdout


def build(verbose: bool = False) -> str:
    """Compile every source and link libhsgd.so; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    for src, kind in SOURCES:
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        path = os.path.join(CSRC, src)
        if kind == "device":
            cmd = [HIPCC, *DEVICE_FLAGS, "-I", INCLUDE, "-c", path, "-o", obj]
        else:
            cmd = [HIPCC, "-x", "c++", *HOST_FLAGS, "-I", INCLUDE, "-I", "/opt/rocm/include",
                   "-c", path, "-o", obj]
        jobs.append((cmd, obj))
    with ThreadPoolExecutor(max_workers=min(4, len(jobs))) as ex:
        outs = list(ex.map(lambda j: _run(j[0]), jobs))
    if verbose:
        for o in outs:
            if o.strip():
                print(o)
    tmp = LIB + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp,
          *[o for _, o in jobs], "-L/opt/rocm/lib", "-lamdhip64"])
    os.replace(tmp, LIB)
    if os.path.exists(C_SMOKE_SRC):
        _run(["gcc", "-std=c11", "-O2", "-Wall", "-Wextra", "-D__HIP_PLATFORM_AMD__", "-I", INCLUDE,
              "-I", "/opt/rocm/include", C_SMOKE_SRC, "-L", PKG, "-lhsgd", "-L/opt/rocm/lib", "-lamdhip64",
              "-lm", "-Wl,-rpath,$ORIGIN", "-Wl,-rpath,/opt/rocm/lib", "-o", C_SMOKE])
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
