"""Build step of the HIP library: ``python -m paper_2410_09739_amd.build``.

Compiles ``csrc/lbm.hip`` and ``csrc/closure.hip`` for gfx950 into ``liblbm.so`` next to this file.
Packed FP32 instructions are disabled for all device code
(``-target-feature -packed-fp32-ops``).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, "csrc", "lbm.hip"), os.path.join(HERE, "csrc", "closure.hip")]
OUT = os.path.join(HERE, "liblbm.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


HOST_CHECK_SRC = os.path.join(os.path.dirname(HERE), "tests", "native", "collide_host.hip")
HOST_CHECK_OUT = os.path.join(os.path.dirname(HERE), "tests", "native", "libcollide_host.so")


def build_host_check() -> str:
    """Host-only build of the kernels' per-node arithmetic, used by CPU tests."""
    tmp = HOST_CHECK_OUT + ".tmp"
    cmd = [HIPCC, "-O2", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
           "-Wno-unused-command-line-argument", "-o", tmp, HOST_CHECK_SRC]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed for " + HOST_CHECK_SRC)
    os.replace(tmp, HOST_CHECK_OUT)
    return HOST_CHECK_OUT


C_ABI_CHECK_SRC = os.path.join(os.path.dirname(HERE), "tests", "native", "c_abi_channel.c")
C_ABI_CHECK_OUT = os.path.join(os.path.dirname(HERE), "tests", "native", "c_abi_channel")


def build_c_abi_check() -> str:
    """A plain C99 program linked against liblbm.so through include/lbm.h only
    (a GPU test runs it): the boundary is usable without Python."""
    tmp = C_ABI_CHECK_OUT + ".tmp"
    inc = os.path.join(os.path.dirname(HERE), "include")
    cmd = ["gcc", "-std=c99", "-O2", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I", inc, "-o", tmp,
           C_ABI_CHECK_SRC, "-L", HERE, "-llbm", "-Wl,-rpath,$ORIGIN/../../paper_2410_09739_amd"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("gcc failed for " + C_ABI_CHECK_SRC)
    os.replace(tmp, C_ABI_CHECK_OUT)
    return C_ABI_CHECK_OUT


def build(verbose: bool = False) -> str:
    tmp = OUT + ".tmp"
    cmd = [HIPCC, *FLAGS, "-o", tmp, *SRCS]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed for " + " ".join(SRCS))
    if verbose:
        sys.stderr.write(res.stderr)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
    if os.path.exists(HOST_CHECK_SRC):
        print(build_host_check())
    if os.path.exists(C_ABI_CHECK_SRC):
        print(build_c_abi_check())
