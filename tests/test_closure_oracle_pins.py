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


def test_first_order_central_moments_are_minus_half_the_force():
    """About the Step 7 velocity (rho u = sum f e + F/2) the first-order central
    moments of any state are -F/2: they carry nothing about the node, which is
    why the feature map sets x_100 = x_010 = x_001 = 0."""
    rng = np.random.default_rng(4)
    e, _, _ = O.lattice()
    F = np.array([3e-5, -2e-5, 1e-5])
    f = O.feq(1.0, [0, 0, 0])[:, None] * (1 + 0.2 * rng.standard_normal((27, 50)))
    rho, u = O.macroscopic(f, tuple(F), post_collision=False)
    kap = C.central_moments(f, u, e)
    for d in range(3):
        np.testing.assert_allclose(kap[1 + d], -0.5 * F[d], rtol=0, atol=1e-16)
    x = C.features(kap, rho)
    assert np.all(x[:, 1:4] == 0.0)
    assert np.all(np.abs(x[:, 4:]) > 0)


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
    """A sub-filter stress that is exactly -2 rho nu0 S, with the filtered fine
    strain equal to the coarse one, is nu0 on the off-diagonal groups; the trace
    and the normal-stress differences get no eddy viscosity."""
    rng = np.random.default_rng(2)
    S = rng.standard_normal((6, 3, 4, 5))
    rho = 1 + 0.01 * rng.standard_normal((3, 4, 5))
    nu0 = 2.5e-4
    tau = -2 * rho[None] * nu0 * S
    nu = C.targets(rho, tau, S, S, 1e-3, eps_rel=0.0)
    np.testing.assert_allclose(nu[[0, 1, 2]], nu0, rtol=1e-12)
    np.testing.assert_array_equal(nu[3:], 0.0)
    # anti-diffusive stress is clipped to zero viscosity
    assert np.all(C.targets(rho, -tau, S, S, 1e-3, eps_rel=0.0) == 0.0)
    np.testing.assert_allclose(C.targets(rho, -tau, S, S, 1e-3, eps_rel=0.0, clip=False)[:3], -nu0, rtol=1e-12)


def test_targets_recover_the_missing_viscous_stress():
    """No sub-filter stress, but the filtered fine strain is (1 + a) times the
    coarse strain: the coarse node needs the viscosity nu (1 + a), so
    nu* = a nu per group (each group with its own nu)."""
    rng = np.random.default_rng(3)
    S = rng.standard_normal((6, 2, 3, 4))
    rho = 1 + 0.01 * rng.standard_normal((2, 3, 4))
    a = np.array([0.3, 0.1, 0.25])
    Sbar = S.copy()
    Sbar[3:] *= (1 + a)[:, None, None, None]
    nus = np.array([4e-4, 5e-4, 6e-4])
    nu = C.targets(rho, np.zeros_like(S), S, Sbar, nus, eps_rel=0.0)
    for j in range(3):
        np.testing.assert_allclose(nu[j], a[j] * nus[j], rtol=1e-12)
    # with eps > 0 the least-squares fit shrinks by S^2 / (S^2 + eps^2)
    nu_e = C.targets(rho, np.zeros_like(S), S, Sbar, nus, eps_rel=0.5)
    eps2 = 0.25 * np.mean(S[:3] ** 2 + 2 * S[3:] ** 2)
    np.testing.assert_allclose(nu_e[0], a[0] * nus[0] * S[3] ** 2 / (S[3] ** 2 + eps2), rtol=1e-12)


def _profile_field(ny, fn):
    """u_x = fn(y) on fine rows y = 0..ny-1, uniform in x and z; rho = 1."""
    y = np.arange(ny, dtype=np.float64)
    u = np.zeros((3, 4, ny, 4))
    u[0] = fn(y)[None, :, None]
    return np.ones((4, ny, 4)), u


def test_filtered_strain_of_polynomial_profiles():
    """Centred differences are exact for quadratics, so for u_x = A y + B y^2 the
    filtered fine strain equals the coarse strain of the filtered velocity away
    from the walls; for u_x = C y^3 both stencils are off by a known amount and
    Sbar_xy - S_xy = -3 C on every interior coarse row (worked by hand: fine
    S_xy = C (3 y^2 + 1) / 2, filtered and doubled C (12 k^2 + 6 k + 5/2); the
    filtered velocity C (16 k^3 + 12 k^2 + 6 k + 1) / 2 gives
    S_xy = C (12 k^2 + 6 k + 11/2))."""
    ny = 12
    rows = slice(1, ny // 2 - 1)  # coarse rows whose stencils stay off the walls
    for walls in (False, True):
        rho, u = _profile_field(ny, lambda y: 0.01 * y + 0.002 * y * y)
        rb, ut, _ = C.box_filter(rho, u)
        Sb = C.filtered_strain(rho, u, walls)
        Sc = C.strain(ut, walls)
        np.testing.assert_allclose(Sb[3][:, rows], Sc[3][:, rows], rtol=1e-13)
        k = np.arange(ny // 2)[rows]
        np.testing.assert_allclose(Sb[3][0, rows, 0], 0.01 + 0.002 * (4 * k + 1), rtol=1e-13)
        Cc = 1e-4
        rho, u = _profile_field(ny, lambda y: Cc * y ** 3)
        rb, ut, _ = C.box_filter(rho, u)
        Sb = C.filtered_strain(rho, u, walls)
        Sc = C.strain(ut, walls)
        np.testing.assert_allclose(Sb[3][0, rows, 0], Cc * (12 * k * k + 6 * k + 2.5), rtol=1e-13)
        np.testing.assert_allclose(Sc[3][0, rows, 0], Cc * (12 * k * k + 6 * k + 5.5), rtol=1e-13)
        np.testing.assert_allclose((Sb[3] - Sc[3])[:, rows], -3 * Cc, rtol=1e-12)
        np.testing.assert_allclose(Sb[[0, 1, 2, 4, 5]], 0.0, atol=1e-18)


def test_filtered_strain_matches_a_loop_over_boxes():
    """Brute force on a tiny grid with varying density: for every coarse node,
    loop over its eight fine nodes, difference u by explicit neighbour indices
    (periodic, or the mirrored value with flipped sign across a y wall), weight
    by rho, average, and double."""
    rng = np.random.default_rng(9)
    nz, ny, nx = 4, 6, 4
    rho = 1 + 0.05 * rng.standard_normal((nz, ny, nx))
    u = 0.03 * rng.standard_normal((3, nz, ny, nx))
    pairs = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
    for walls in (False, True):
        def uval(c, z, y, x):
            x %= nx
            z %= nz
            if walls and (y < 0 or y >= ny):
                return -u[c, z, min(max(y, 0), ny - 1), x]
            return u[c, z, y % ny, x]

        ref = np.zeros((6, nz // 2, ny // 2, nx // 2))
        for Z in range(nz // 2):
            for Y in range(ny // 2):
                for X in range(nx // 2):
                    acc = np.zeros(6)
                    rsum = 0.0
                    for z in (2 * Z, 2 * Z + 1):
                        for y in (2 * Y, 2 * Y + 1):
                            for x in (2 * X, 2 * X + 1):
                                g = np.zeros((3, 3))  # g[i][j] = d_i u_j
                                for c in range(3):
                                    g[0][c] = 0.5 * (uval(c, z, y, x + 1) - uval(c, z, y, x - 1))
                                    g[1][c] = 0.5 * (uval(c, z, y + 1, x) - uval(c, z, y - 1, x))
                                    g[2][c] = 0.5 * (uval(c, z + 1, y, x) - uval(c, z - 1, y, x))
                                for k, (i, j) in enumerate(pairs):
                                    acc[k] += rho[z, y, x] * 0.5 * (g[i][j] + g[j][i])
                                rsum += rho[z, y, x]
                    ref[:, Z, Y, X] = 2.0 * acc / rsum
        np.testing.assert_allclose(C.filtered_strain(rho, u, walls), ref, rtol=1e-12, atol=1e-16)


def test_bf16_rounding_equals_torch_cpu_cast():
    """round_bf16 against an independent implementation of the same rounding:
    torch's CPU float32 -> bfloat16 conversion (round to nearest, ties to even).
    Inputs cover random magnitudes, exact ties (low 16 bits 0x8000) with even and
    odd kept halves, values next to ties, subnormals, the overflow edge, signed
    zeros and infinities."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(123)
    mant = rng.integers(0, 1 << 23, 4000, dtype=np.uint64)
    expo = rng.integers(1, 255, 4000, dtype=np.uint64)
    sign = rng.integers(0, 2, 4000, dtype=np.uint64)
    bits = (sign << 31) | (expo << 23) | mant
    ties = (bits & ~np.uint64(0xFFFF)) | np.uint64(0x8000)
    near = np.concatenate([ties - 1, ties + 1])
    sub = rng.integers(1, 1 << 23, 500, dtype=np.uint64)
    edge = np.array([0x7F7F7FFF, 0x7F7F8000, 0x7F7FFFFF, 0x80000000, 0x00000000, 0x7F800000, 0xFF800000,
                     0x00008000, 0x00018000, 0x3F808000, 0x3F818000], dtype=np.uint64)
    allbits = np.concatenate([bits, ties, near, sub, edge]).astype(np.uint32)
    x = allbits.view(np.float32)
    ref = torch.from_numpy(x.copy()).to(torch.bfloat16).to(torch.float32).numpy().astype(np.float64)
    got = C.round_bf16(x)
    np.testing.assert_array_equal(np.signbit(got), np.signbit(ref))
    np.testing.assert_array_equal(got, ref)


def test_splitmix64_output_function_reproduces_the_published_sequence():
    """The generator's mixing function is SplitMix64's (Steele, Lea and Flood,
    2014).  Stepping the state by the golden gamma 0x9E3779B97F4A7C15 from the
    seed 1234567 gives the sequence published with the reference implementation
    (Vigna's splitmix64.c test values)."""
    M = (1 << 64) - 1
    s, out = 1234567, []
    for _ in range(5):
        s = (s + 0x9E3779B97F4A7C15) & M
        out.append(C._mix64(s))
    assert out == [6457827717110365317, 3203168211198807973, 9817491932198370423,
                   4593380528125082431, 16408922859458223821]


def test_minibatch_indices_follow_their_definition_and_are_uniform():
    """sample_indices: slot j of step t is mix64(seed ^ mix64(t gamma + j)) mod n,
    checked against the published-sequence generator above for the inner word;
    the indices stay in [0, n), differ between steps and seeds, and a large
    draw is uniform over n bins (chi-square at the 1e-4 level)."""
    M = (1 << 64) - 1
    gamma = 0x9E3779B97F4A7C15
    for seed, t, n in [(7, 0, 1000), (123456789, 41, 17), (2**63 + 5, 9999, 1 << 20)]:
        idx = C.sample_indices(seed, t, 64, n)
        for j in (0, 1, 63):
            inner = C._mix64((t * gamma + j) & M)
            assert idx[j] == C._mix64(seed ^ inner) % n
        assert idx.min() >= 0 and idx.max() < n
    assert not np.array_equal(C.sample_indices(1, 0, 64, 1 << 30), C.sample_indices(1, 1, 64, 1 << 30))
    assert not np.array_equal(C.sample_indices(1, 0, 64, 1 << 30), C.sample_indices(2, 0, 64, 1 << 30))
    n = 50
    draws = np.concatenate([C.sample_indices(99, t, 500, n) for t in range(40)])
    counts = np.bincount(draws, minlength=n)
    expect = draws.size / n
    chi2 = float(((counts - expect) ** 2 / expect).sum())
    from scipy.stats import chi2 as chi2dist
    assert chi2dist.sf(chi2, n - 1) > 1e-4


def _hidden(p, x):
    """Pre-activations and bf16 activations of the oracle's quantised network."""
    W1, b1, W2, b2, W3, b3 = C.unpack(p)
    xq = C.round_bf16(x)
    z1 = xq @ C.round_bf16(W1).T + b1.astype(np.float32)
    h1 = C.round_bf16(np.maximum(z1, 0.0))
    z2 = h1 @ C.round_bf16(W2).T + b2.astype(np.float32)
    return z1, h1, z2, C.round_bf16(np.maximum(z2, 0.0))


def test_acceptance_of_one_hidden_rounding_flip_rejects_planted_mistakes():
    """The GPU inference check accepts a node's outputs when they are the
    oracle's network with one hidden activation rounded to its other bf16
    neighbour, where that activation may sit on a rounding boundary.  Planted
    on the CPU: such a flip next to a boundary is accepted; the same flip on a
    unit far from any boundary, an output offset by 1e-4, the outputs of another
    node, or the outputs with W3's rows swapped are rejected."""
    from closure_checks import explained_by_one_hidden_flip as ok
    rng = np.random.default_rng(4)
    W1, b1, W2, b2, W3, b3 = C.unpack(C.init_params(2))
    p = C.pack(W1, b1 + 0.1 * rng.standard_normal(64), W2, b2 + 0.1 * rng.standard_normal(64), W3,
               b3 + 0.1 * rng.standard_normal(6)).astype(np.float32).astype(np.float64)
    W3q, b3f = C.round_bf16(C.unpack(p)[4]), C.unpack(p)[5].astype(np.float32).astype(np.float64)
    X = rng.standard_normal((3000, 27)).astype(np.float32).astype(np.float64)
    ref = C.forward_bf16(p, X)
    tol = 1e-6
    near = far = None
    for n in range(X.shape[0]):
        z1, h1, z2, h2 = _hidden(p, X[n])
        up = C.round_bf16(np.maximum(z2, 0.0) * (1 + 2.0 ** -8))  # the next bf16 value up (positive units)
        rel = np.abs(np.maximum(z2, 0.0) - 0.5 * (h2 + up)) / np.maximum(np.abs(z2), 1e-30)
        k_near, k_far = int(np.argmin(np.where(z2 > 0, rel, np.inf))), int(np.argmax(np.where(z2 > 1.0, rel, -1)))
        if near is None and z2[k_near] > 0 and rel[k_near] < 1e-7:
            h = h2.copy()
            h[k_near] = C.round_bf16([2 * z2[k_near] - h2[k_near]])[0]  # the other neighbour
            near = (n, h @ W3q.T + b3f)
        if far is None and z2[k_far] > 1.0 and rel[k_far] > 1e-3:
            h = h2.copy()
            h[k_far] = C.round_bf16([2 * z2[k_far] - h2[k_far]])[0]
            if np.abs(h @ W3q.T + b3f - ref[n]).max() > 10 * tol:
                far = (n, h @ W3q.T + b3f)
        if near and far:
            break
    assert near is not None and far is not None
    n, got = near
    assert np.abs(got - ref[n]).max() > 10 * tol  # the flip is visible
    assert ok(p, X[n], got, tol)
    n, got = far
    assert not ok(p, X[n], got, tol)
    assert not ok(p, X[0], ref[0] + 1e-4, tol)
    assert not ok(p, X[0], ref[1], tol)
    assert not ok(p, X[0], ref[0][[1, 0, 2, 3, 4, 5]], tol) or np.allclose(ref[0][0], ref[0][1])


def test_feature_rounding_alternatives_cover_exactly_the_near_boundary_features():
    """The fused-step check may take a feature rounded to its other bf16
    neighbour only where the feature lies within the stated distance of a
    rounding boundary: a feature planted on a boundary gets the alternative,
    features far from any boundary get none."""
    from closure_checks import bf16_alternatives
    X = np.full((3, 27), 1.0 + 2.0 ** -8)  # 1 + half a bf16 ulp (2^-7 in [1, 2)): a tie
    X[1] = 1.0 + 2.0 ** -9                 # a quarter ulp from 1: far from the boundaries
    X[2] = 1.0 + 2.0 ** -9
    X[2, 5] = 1.0 + 2.0 ** -8 + 1e-9      # just above the tie
    alts = bf16_alternatives(X, np.full(X.shape, 1e-7))
    assert set(alts) == {0, 2}
    assert all(len(a) == 2 ** 4 - 1 for a in [alts[0]])  # ties in every column: the first four flipped
    (only,) = alts[2]
    assert np.flatnonzero(only != C.round_bf16(X[2])).tolist() == [5]
    assert {C.round_bf16(X[2])[5], only[5]} == {1.0, 1.0 + 2.0 ** -7}
