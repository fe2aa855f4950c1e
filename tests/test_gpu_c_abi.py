"""The C ABI on its own: tests/hsgd_c_smoke.c (built next to libhsgd.so by the package's build
step) allocates device memory with the HIP runtime and drives warps, render, select, the
gradient step and a two-level refine through include/hsgd.h, checking status codes and
closed-form results (see the program's header). Run as a child process."""

import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

BIN = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2307_03017_amd",
                   "hsgd_c_smoke")


def test_c_program_through_the_abi():
    assert os.path.exists(BIN), "build the package first (it also builds the C program)"
    print("running", BIN, flush=True)
    r = subprocess.run([BIN], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=120)
    print(r.stdout, flush=True)
    assert r.returncode == 0, r.stdout
    assert r.stdout.strip().endswith("ok")
