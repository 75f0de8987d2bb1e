"""The library's host code (the C ABI: argument checks, the rate table,
context set-up and clean-up) built with AddressSanitizer and
UndefinedBehaviorSanitizer and driven, without a GPU, by a plain C++ program
(tests/native/abi_host_sanitized.cpp) through include/lbm.h: any out-of-bounds
access, use after free, leak or undefined behaviour on those paths aborts it.
The device code is compiled unoptimised (it is never launched here)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang++"
SRCS = [os.path.join(ROOT, "paper_2410_09739_amd", "csrc", f) for f in ("lbm.hip", "closure.hip")]
DRIVER = os.path.join(ROOT, "tests", "native", "abi_host_sanitized.cpp")


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="no ROCm clang toolchain")
def test_c_abi_host_code_is_clean_under_address_and_ub_sanitizers(tmp_path):
    lib = tmp_path / "liblbm_san.so"
    host_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-O0", "-Xarch_host", "-O1", "-Xarch_host", "-g",
                           "-std=c++17", "-fPIC", "-shared", *host_san,
                           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                           "-Wno-unused-command-line-argument", "-o", str(lib), *SRCS],
                          stderr=subprocess.DEVNULL)
    exe = tmp_path / "drive"
    subprocess.check_call([CLANG, "-std=c++17", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-I", os.path.join(ROOT, "include"), "-o", str(exe), DRIVER, "-L", str(tmp_path),
                           "-llbm_san", f"-Wl,-rpath,{tmp_path}"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "0 unexpected results" in r.stdout
