"""The entry point that allocates nothing (lbm_get_f_nodes_noalloc) against
lbm_get_f_nodes, through the C ABI: the same populations, bit for bit, on two
calls in a row (the second with fewer nodes), for every storage form; the size
limit is enforced; two contexts on one GPU use the shared staging array one
after the other."""
import numpy as np
import pytest

import oracle as O
from paper_2410_09739_amd import lbm as L
from paper_2410_09739_amd import workloads as W

pytestmark = pytest.mark.gpu

MAXN = 4096  # LBM_NOALLOC_MAX_NODES of include/lbm.h


def _lattice(shape, storage, seed):
    nx, ny, nz = shape
    rho, u = W.random_fields(nx, ny, nz, seed=seed, u_amp=0.05)
    g0 = O.init(rho, u) * W.random_factors((27, nz, ny, nx), seed=seed + 1, amplitude=0.05)
    lat = L.Lattice(L.Config(nx, ny, nz, storage=storage, walls_y=True, nu=0.02, force=(1e-5, 0, 0)))
    lat.set_f(g0)
    lat.step(3)
    return lat


def _noalloc(lat, nodes):
    nodes = np.ascontiguousarray(nodes, dtype=np.int64)
    f = np.full(27 * max(nodes.size, 1), np.nan)
    L.lbm_get_f_nodes_noalloc(lat.ctx, nodes, f)
    return f[: 27 * nodes.size].reshape(27, nodes.size)


@pytest.mark.parametrize("storage", ["f64", "f32", "f16dev", "bf16dev"])
def test_noalloc_node_read_equals_the_allocating_one(storage):
    shape = (70, 9, 11)
    n = np.prod(shape)
    rng = np.random.default_rng(5)
    with _lattice(shape, storage, 71) as lat:
        for count in (3000, 17):  # two calls in a row, the second smaller
            nodes = rng.integers(0, n, count)
            ref = lat.get_f_nodes(nodes)
            got = _noalloc(lat, nodes)
            assert np.array_equal(got, ref), (storage, count)
        # the full maximum, with the first and last node
        nodes = np.concatenate([[0, n - 1], rng.integers(0, n, MAXN - 2)])
        assert np.array_equal(_noalloc(lat, nodes), lat.get_f_nodes(nodes))


def test_noalloc_rejects_too_many_nodes_and_bad_indices():
    with _lattice((20, 6, 5), "f32", 81) as lat:
        with pytest.raises(L.LBMError) as ei:
            _noalloc(lat, np.zeros(MAXN + 1, dtype=np.int64))
        assert ei.value.code == L.LBM_EINVAL and "maximum" in str(ei.value)
        with pytest.raises(L.LBMError) as ei:
            _noalloc(lat, np.array([0, 600]))
        assert ei.value.code == L.LBM_EINVAL
        assert _noalloc(lat, np.zeros(0, dtype=np.int64)).shape == (27, 0)
        # the context stays usable
        nodes = np.arange(0, 600, 7)
        assert np.array_equal(_noalloc(lat, nodes), lat.get_f_nodes(nodes))


def test_two_contexts_share_the_staging_array_in_turn():
    a = _lattice((33, 7, 5), "f64", 91)
    b = _lattice((64, 4, 3), "f16dev", 93)
    try:
        na = np.arange(0, 33 * 7 * 5, 3)
        nb = np.arange(0, 64 * 4 * 3, 5)
        for _ in range(2):
            ga = _noalloc(a, na)
            gb = _noalloc(b, nb)
            assert np.array_equal(ga, a.get_f_nodes(na))
            assert np.array_equal(gb, b.get_f_nodes(nb))
    finally:
        a.close()
        b.close()
