"""The C ABI used from plain C (tests/native/c_abi_channel.c, built by
__graft_entry__.build() against include/lbm.h and liblbm.so only): a forced
FP64 channel from rest, whose printed profile, mass and momentum match the
FP64 oracle's run of the same steps (Step 7 fields, 1e-12)."""
import os
import subprocess

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "tests", "native", "c_abi_channel")


def test_plain_c_program_matches_oracle():
    if not os.path.exists(EXE):
        pytest.fail("tests/native/c_abi_channel is not built: run __graft_entry__.build()")
    nx, ny, nz, steps = 32, 16, 8, 100
    r = subprocess.run([EXE, str(nx), str(ny), str(nz), str(steps)], capture_output=True, text=True, timeout=100)
    assert r.returncode == 0, r.stderr
    vals = np.array([float(v) for v in r.stdout.split()])
    assert vals.size == ny + 2
    F = (1e-5, 0.0, 0.0)
    g0 = O.init(np.ones((nz, ny, nx)), np.zeros((3, nz, ny, nx)))
    g = O.run(g0, O.omega_table(0.02), F, walls_y=True, steps=steps)
    rho, u = O.macroscopic(g, F)
    prof = u[0].mean(axis=(0, 2))
    np.testing.assert_allclose(vals[:ny], prof, rtol=1e-12, atol=1e-17)
    assert vals[ny] == pytest.approx(rho.sum(), rel=1e-13)
    assert vals[ny + 1] == pytest.approx((rho * u[0]).sum(), rel=1e-12)
    assert prof[ny // 2] > 0  # the force has driven the flow
