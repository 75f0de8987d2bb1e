"""The kernels' per-node arithmetic (fpc_collide.hpp), compiled for the host,
against the FP64 oracle on the CPU: catches transform or collision mistakes in
the HIP path before any GPU run.  FP64: 1e-13 relative to max(|f|, w_alpha);
FP32: the per-step FP32 bound of the GPU parity tests (4e-7 w_alpha)."""
import ctypes
import os

import numpy as np
import pytest

import oracle as O
from paper_2410_09739_amd import workloads as W

LIB = os.path.join(os.path.dirname(__file__), "native", "libcollide_host.so")
_dp = ctypes.POINTER(ctypes.c_double)


@pytest.fixture(scope="module")
def host():
    if not os.path.exists(LIB):
        from paper_2410_09739_amd import build
        build.build_host_check()
    lib = ctypes.CDLL(LIB)
    for n in ("host_collide_f64", "host_collide_f32", "host_collide_maxwell_f64", "host_collide_maxwell_f32"):
        getattr(lib, n).argtypes = [_dp, _dp, _dp, _dp]
    lib.host_feq_f64.argtypes = [ctypes.c_double, _dp, _dp]
    _fp = ctypes.POINTER(ctypes.c_float)
    for n in ("host_collide_dev_f32", "host_collide_units_f32"):
        getattr(lib, n).argtypes = [_fp, _dp, _dp, ctypes.c_int, _fp]
    for n in ("host_collide_unit_f64", "host_collide_unit_f32"):
        getattr(lib, n).argtypes = [_dp, _dp, _dp]
    for n in ("host_collide_unit_dev_f32", "host_collide_unit_units_f32"):
        getattr(lib, n).argtypes = [_fp, _dp, _fp]
    return lib


def _call(fn, f, om, F):
    out = np.zeros(27)
    a = [np.ascontiguousarray(x, dtype=np.float64) for x in (f, om, F)]
    fn(*(x.ctypes.data_as(_dp) for x in a), out.ctypes.data_as(_dp))
    return out


WA = O.feq(1.0, [0, 0, 0])


@pytest.mark.parametrize("attractor", ["fpc", "maxwell"])
@pytest.mark.parametrize("seed", range(12))
def test_host_collision_matches_oracle(host, seed, attractor):
    rng = np.random.default_rng(100 + seed)
    u = 0.1 * rng.uniform(-1, 1, 3)
    f = O.feq(1 + 0.05 * rng.uniform(-1, 1), u) * W.random_factors(27, seed, 0.2)
    mode = ["paper", "order_scaled", "explicit"][seed % 3]
    om = O.omega_table(10 ** rng.uniform(-5, -0.5), omega_bulk=rng.uniform(0.5, 1.9),
                       omega_higher=rng.uniform(0.5, 1.9), mode=mode, explicit=rng.uniform(0.1, 1.99, 27))
    F = 1e-4 * rng.uniform(-1, 1, 3) if seed % 2 else np.zeros(3)
    ref = O.collide_node(f, om, F, attractor=attractor)
    tag = "" if attractor == "fpc" else "maxwell_"
    got = _call(getattr(host, f"host_collide_{tag}f64"), f, om, F)
    err = np.max(np.abs(got - ref) / np.maximum(np.abs(ref), WA))
    assert err <= 1e-13, err
    got32 = _call(getattr(host, f"host_collide_{tag}f32"), f, om, F)
    assert np.all(np.abs(got32 - ref) <= 4e-7 * WA), np.max(np.abs(got32 - ref) / WA)


@pytest.mark.parametrize("rho,u", [(1.0, (0, 0, 0)), (1.04, (0.06, -0.02, 0.09)), (0.95, (-0.2, 0.15, 0.05))])
def test_host_equilibrium_matches_oracle(host, rho, u):
    out = np.zeros(27)
    uu = np.ascontiguousarray(u, dtype=np.float64)
    host.host_feq_f64(rho, uu.ctypes.data_as(_dp), out.ctypes.data_as(_dp))
    np.testing.assert_allclose(out, O.feq(rho, u), rtol=0, atol=4e-16)


def _call_dev(fn, dev, om, F, maxwell):
    fp = ctypes.POINTER(ctypes.c_float)
    out = np.zeros(27, dtype=np.float32)
    d = np.ascontiguousarray(dev, dtype=np.float32)
    a = [np.ascontiguousarray(x, dtype=np.float64) for x in (om, F)]
    fn(d.ctypes.data_as(fp), *(x.ctypes.data_as(_dp) for x in a), int(maxwell), out.ctypes.data_as(fp))
    return out


@pytest.mark.parametrize("maxwell", [False, True])
@pytest.mark.parametrize("seed", range(16))
def test_storage_unit_collision_is_bitwise_the_deviation_one(host, seed, maxwell):
    """The FP16/BF16 kernels run the collision on the stored numbers (each
    deviation times its power-of-two storage scale, moments times 2^18);
    every factor is an exact power of two, so the post-collision deviations
    must be bitwise those of the same FP32 arithmetic on plain deviations,
    from deviations of 1e-9 w up to w."""
    rng = np.random.default_rng(700 + seed)
    u = 0.1 * rng.uniform(-1, 1, 3)
    f = O.feq(1 + 0.05 * rng.uniform(-1, 1), u) * W.random_factors(27, seed, 0.2)
    amp = 10.0 ** rng.uniform(-9, 0)  # overall size of the non-equilibrium part
    dev = ((f - WA) * amp).astype(np.float32)
    om = O.omega_table(10 ** rng.uniform(-5, -0.5), omega_bulk=rng.uniform(0.5, 1.9),
                       omega_higher=rng.uniform(0.5, 1.9), mode="paper")
    F = 1e-4 * rng.uniform(-1, 1, 3) * amp
    a = _call_dev(host.host_collide_dev_f32, dev, om, F, maxwell)
    b = _call_dev(host.host_collide_units_f32, dev, om, F, maxwell)
    assert np.all(np.isfinite(a))
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), np.max(np.abs(a - b))


@pytest.mark.parametrize("seed", range(16))
def test_host_unit_rate_collision_matches_oracle(host, seed):
    """The step kernels' collision for the paper's rates (bulk omega_7 and every
    rate of orders 3-6 equal to 1) without a force computes only the
    second-order moments before relaxing; it must equal the oracle's full
    Appendix D collision (explicit matrices, every moment relaxed) to the same
    bounds as the general path, for shear viscosities from 1e-5 to 0.3 and
    states far from equilibrium."""
    rng = np.random.default_rng(900 + seed)
    u = 0.15 * rng.uniform(-1, 1, 3)
    f = O.feq(1 + 0.08 * rng.uniform(-1, 1), u) * W.random_factors(27, seed + 50, 0.3)
    om = O.omega_table(10 ** rng.uniform(-5, -0.5))
    assert om[7] == 1.0 and np.all(om[10:] == 1.0)
    ref = O.collide_node(f, om)
    out = np.zeros(27)
    a = [np.ascontiguousarray(x, dtype=np.float64) for x in (f, om)]
    host.host_collide_unit_f64(*(x.ctypes.data_as(_dp) for x in a), out.ctypes.data_as(_dp))
    err = np.max(np.abs(out - ref) / np.maximum(np.abs(ref), WA))
    assert err <= 1e-13, err
    out32 = np.zeros(27)
    host.host_collide_unit_f32(*(x.ctypes.data_as(_dp) for x in a), out32.ctypes.data_as(_dp))
    assert np.all(np.abs(out32 - ref) <= 4e-7 * WA), np.max(np.abs(out32 - ref) / WA)
    # and the general path (every moment relaxed at rate 1) agrees with it
    gen = _call(host.host_collide_f64, f, om, np.zeros(3))
    assert np.max(np.abs(gen - out) / np.maximum(np.abs(ref), WA)) <= 1e-13


@pytest.mark.parametrize("seed", range(12))
def test_unit_rate_collision_in_storage_units_is_bitwise_the_deviation_one(host, seed):
    """As for the general collision: the storage-unit form of the unit-rate
    collision (the 16-bit kernels' arithmetic) is bitwise the FP32 arithmetic on
    plain deviations, for deviations from 1e-9 w to w."""
    fp = ctypes.POINTER(ctypes.c_float)
    rng = np.random.default_rng(950 + seed)
    u = 0.1 * rng.uniform(-1, 1, 3)
    f = O.feq(1 + 0.05 * rng.uniform(-1, 1), u) * W.random_factors(27, seed + 70, 0.2)
    dev = ((f - WA) * 10.0 ** rng.uniform(-9, 0)).astype(np.float32)
    om = np.ascontiguousarray(O.omega_table(10 ** rng.uniform(-5, -0.5)))
    outs = []
    for fn in (host.host_collide_unit_dev_f32, host.host_collide_unit_units_f32):
        o = np.zeros(27, dtype=np.float32)
        fn(dev.ctypes.data_as(fp), om.ctypes.data_as(_dp), o.ctypes.data_as(fp))
        outs.append(o)
    assert np.all(np.isfinite(outs[0]))
    assert np.array_equal(outs[0].view(np.uint32), outs[1].view(np.uint32))
