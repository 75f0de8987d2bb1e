"""Pins of the closure oracle: calculus (finite differences), an independent
automatic differentiation (torch, FP64, CPU), the Adam update's closed form,
exact identities of the feature map, the box filter and the strain stencil."""
import numpy as np
import pytest

import oracle as O
from oracle import closure_oracle as C


def _data(seed, B=37):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((B, C.NIN))
    Y = rng.standard_normal((B, C.NOUT))
    return C.init_params(seed), X, Y


def test_param_count_and_layout():
    assert C.NPARAM == 6342
    p = np.arange(C.NPARAM, dtype=float)
    W1, b1, W2, b2, W3, b3 = C.unpack(p)
    assert W1[0, 0] == 0 and b1[0] == 64 * 27 and W3.shape == (6, 64) and b3[-1] == C.NPARAM - 1
    np.testing.assert_array_equal(C.pack(*C.unpack(p)), p)


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_matches_central_differences(seed):
    p, X, Y = _data(seed)
    _, g = C.loss_and_grad(p, X, Y)
    rng = np.random.default_rng(seed + 10)
    idx = rng.choice(C.NPARAM, 60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros(C.NPARAM)
        e[i] = h
        fd = (C.loss(p + e, X, Y) - C.loss(p - e, X, Y)) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-6, abs=1e-9), i


def test_gradient_matches_torch_autograd():
    torch = pytest.importorskip("torch")
    p, X, Y = _data(3)
    L, g = C.loss_and_grad(p, X, Y)
    pt = torch.tensor(p, dtype=torch.float64, requires_grad=True)
    sizes = [64 * 27, 64, 64 * 64, 64, 6 * 64, 6]
    parts = torch.split(pt, sizes)
    W1, b1, W2, b2, W3, b3 = (parts[0].view(64, 27), parts[1], parts[2].view(64, 64), parts[3],
                              parts[4].view(6, 64), parts[5])
    Xt, Yt = torch.tensor(X), torch.tensor(Y)
    h = torch.relu(Xt @ W1.T + b1)
    h = torch.relu(h @ W2.T + b2)
    lt = torch.mean((h @ W3.T + b3 - Yt) ** 2)
    lt.backward()
    assert L == pytest.approx(lt.item(), rel=1e-14)
    np.testing.assert_allclose(g, pt.grad.numpy(), rtol=1e-12, atol=1e-15)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(0)
    p = rng.standard_normal(10)
    g = rng.standard_normal(10)
    p1, m, v = C.adam_step(p, g, np.zeros(10), np.zeros(10), 1, lr=1e-3)
    # bias-corrected m = g, v = g^2 on the first step
    np.testing.assert_allclose(p1, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_folded_normalisation_is_exact():
    p, X, _ = _data(5)
    rng = np.random.default_rng(6)
    mu = rng.standard_normal(27)
    sigma = rng.uniform(0.5, 2.0, 27)
    sigma[3] = 0.0  # a dropped (constant) feature
    s_y = 3.7e-4
    Xr = X * np.where(sigma > 0, sigma, 1.0) + mu
    Xstd = np.where(sigma > 0, (Xr - mu) / np.where(sigma > 0, sigma, 1.0), 0.0)
    o_std, _ = C.forward(p, Xstd)
    o_raw, _ = C.forward(C.fold_normalisation(p, mu, sigma, s_y), Xr)
    np.testing.assert_allclose(o_raw, s_y * o_std, rtol=1e-10, atol=1e-16)


def test_features_vanish_at_equilibrium_except_density():
    e, _, _ = O.lattice()
    for rho, u in [(1.02, (0.05, -0.03, 0.01)), (0.97, (0.0, 0.0, 0.0))]:
        f = O.feq(rho, u)
        kap = C.central_moments(f[:, None], np.array(u)[:, None], e)[:, 0]
        x = C.features(kap, np.array(rho))
        assert x[0] == pytest.approx(rho - 1, abs=1e-15)
        np.testing.assert_allclose(x[1:], 0.0, atol=1e-14)


def test_box_filter_conserves_mass_momentum_and_stress_is_a_covariance():
    rng = np.random.default_rng(1)
    rho = 1 + 0.01 * rng.standard_normal((4, 6, 8))
    u = 0.05 * rng.standard_normal((3, 4, 6, 8))
    rb, ut, tau = C.box_filter(rho, u)
    assert rb.shape == (2, 3, 4)
    assert rb.sum() * 8 == pytest.approx(rho.sum(), rel=1e-14)
    for d in range(3):
        assert (rb * ut[d]).sum() * 8 == pytest.approx((rho * u[d]).sum(), rel=1e-12)
    # tau is rho-weighted covariance of u within each box: positive semidefinite
    T = np.zeros((2, 3, 4, 3, 3))
    for k, (i, j) in enumerate([(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]):
        T[..., i, j] = tau[k]
        T[..., j, i] = tau[k]
    assert np.linalg.eigvalsh(T).min() > -1e-15
    # a velocity that is uniform in each box has no sub-filter stress
    uu = np.repeat(np.repeat(np.repeat(ut, 2, 1), 2, 2), 2, 3)
    _, _, tau0 = C.box_filter(np.ones_like(rho), uu)
    np.testing.assert_allclose(tau0, 0.0, atol=1e-17)


def test_strain_of_a_shear_wave_is_the_centred_difference():
    ny = 16
    k = 2 * np.pi / ny
    y = np.arange(ny)
    u = np.zeros((3, 2, ny, 3))
    u[0] = np.sin(k * y)[None, :, None]
    S = C.strain(u, walls_y=False)
    np.testing.assert_allclose(S[3, 0, :, 0], 0.5 * np.sin(k) * np.cos(k * y), atol=1e-15)
    np.testing.assert_allclose(S[[0, 1, 2, 4, 5]], 0.0, atol=1e-15)
    # walls: u = 0 at y = -1/2 and ny - 1/2 -> antisymmetric ghost
    u[0] = (y + 0.5)[None, :, None] * 0.01
    Sw = C.strain(u, walls_y=True)
    assert Sw[3, 0, 0, 0] == pytest.approx(0.5 * 0.5 * (0.015 + 0.005))
    assert Sw[3, 0, 5, 0] == pytest.approx(0.5 * 0.01)


def test_targets_recover_an_exact_eddy_viscosity():
    rng = np.random.default_rng(2)
    S = rng.standard_normal((6, 3, 4, 5))
    rho = 1 + 0.01 * rng.standard_normal((3, 4, 5))
    nu0 = 2.5e-4
    tau = -2 * rho[None] * nu0 * S
    nu = C.targets(rho, tau, S, eps_rel=0.0)
    np.testing.assert_allclose(nu[[0, 1, 2, 4, 5]], nu0, rtol=1e-12)
    np.testing.assert_array_equal(nu[3], 0.0)
    # anti-diffusive stress is clipped to zero viscosity
    assert np.all(C.targets(rho, -tau, S, eps_rel=0.0) == 0.0)
