"""The FP64 oracle (test infrastructure, plain C) built with AddressSanitizer
and UndefinedBehaviorSanitizer and run on every boundary set, the LES, the
Maxwellian model and the node-sampling entry point, in a separate process:
any out-of-bounds access or undefined behaviour in the C code aborts it."""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "fpc_oracle.c")


def _libasan():
    out = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    return out if os.path.isabs(out) and os.path.exists(out) else None


@pytest.mark.skipif(_libasan() is None, reason="gcc without AddressSanitizer runtime")
def test_oracle_is_clean_under_address_and_ub_sanitizers(tmp_path):
    lib = tmp_path / "liboracle_asan.so"
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]
    subprocess.check_call(["gcc", "-O1", "-g", *san, "-fPIC", "-shared", "-o", str(lib), SRC, "-lm"])
    script = tmp_path / "drive.py"
    script.write_text(textwrap.dedent(f"""
        import ctypes, numpy as np
        lib = ctypes.CDLL({str(lib)!r})
        dp = ctypes.POINTER(ctypes.c_double)
        i64p = ctypes.POINTER(ctypes.c_int64)
        def d(a):
            return None if a is None else a.ctypes.data_as(dp)
        nx, ny, nz = 5, 4, 3
        N = nx * ny * nz
        rng = np.random.default_rng(0)
        w = np.zeros(27); lib.orc_feq(ctypes.c_double(1.0), d(np.zeros(3)), d(w))
        g = (w[:, None] * (1 + 0.1 * rng.standard_normal((27, N)))).copy()
        om = np.full(27, 1.0); om[4:10] = 1.7
        F = np.array([1e-4, 0.0, 2e-5])
        lid = np.array([0.02, 0.0, 0.0])
        les = np.array([0.2, 3.0, 26.0])
        lib.orc_run.argtypes = [ctypes.c_int] * 4 + [dp, dp, dp, dp, ctypes.c_int, ctypes.c_int, dp]
        lib.orc_stream_push.argtypes = [ctypes.c_int] * 4 + [dp, dp, dp]
        lib.orc_step_nodes.argtypes = [ctypes.c_int] * 4 + [dp, dp, dp, dp, i64p, ctypes.c_int64, dp, ctypes.c_int, dp]
        for walls, l, model, le in [(0, None, 0, None), (1, lid, 1, None), (7, lid, 0, les), (9, None, 0, les),
                                    (11, None, 1, None)]:
            h = g.copy()
            assert lib.orc_run(nx, ny, nz, walls, d(l), d(om), d(F), d(h), 3, model, d(le)) == 0
            f = np.zeros_like(h)
            lib.orc_stream_push(nx, ny, nz, walls, d(l), d(h), d(f))
            sel = np.arange(0, N, 7, dtype=np.int64)
            out = np.zeros((27, sel.size))
            lib.orc_step_nodes(nx, ny, nz, walls, d(l), d(om), d(F), d(h), sel.ctypes.data_as(i64p), sel.size,
                               d(out), model, d(le))
            assert np.isfinite(out).all()
        print("ok")
    """))
    env = dict(os.environ, LD_PRELOAD=_libasan(), ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, str(script)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout[-2000:] + r.stderr[-4000:]
