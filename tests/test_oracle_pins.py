"""Pins of the FP64 CPU oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: printed tables
of Appendix D (fixtures under tests/golden/), exact rational arithmetic, brute
force definitions, closed forms printed in Sec. 3.4, conservation laws,
symmetry of the lattice, and the viscosity law of Eq. (transportcoeff3DFPCLBM).
"""
import itertools
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from paper_2410_09739_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")
ORDER = ["000", "100", "010", "001", "110", "101", "011", "200", "020", "002", "120", "102",
         "210", "012", "201", "021", "111", "220", "202", "022", "211", "121", "112", "122",
         "212", "221", "222"]
IX = {k: i for i, k in enumerate(ORDER)}


def _rows(name):
    with open(os.path.join(GOLD, name)) as fh:
        return [ln.split() for ln in fh if ln.strip() and not ln.startswith("#")]


def _state(seed, rho=1.0, u=(0.04, -0.03, 0.02), amp=0.1):
    fe = O.feq(rho, u)
    return fe * W.random_factors(27, seed, amp)


# ------------------------------------------------------------------ lattice
def test_velocity_set_is_full_cube_and_opposites_pair():
    e, opp, mnp = O.lattice()
    assert sorted(map(tuple, e.tolist())) == sorted(itertools.product([-1, 0, 1], repeat=3))
    assert (e[opp] == -e).all() and (opp[opp] == np.arange(27)).all()
    # moment exponents in the printed order of the moment vectors (Sec. 3.5)
    assert ["".join(map(str, r)) for r in mnp.tolist()] == ORDER


def test_P_rows_equal_printed_step1():
    rows = _rows("app_d_step1_raw_moment_rows.txt")
    P, _, _, _ = O.matrices([0, 0, 0])
    assert [r[0] for r in rows] == ORDER
    A = np.array([[int(x) for x in r[1:]] for r in rows], dtype=float)
    np.testing.assert_array_equal(P, A)


def _exact_inverse(M):
    n = len(M)
    a = [[Fraction(int(M[i][j])) for j in range(n)] + [Fraction(int(i == j)) for j in range(n)] for i in range(n)]
    for c in range(n):
        piv = next(r for r in range(c, n) if a[r][c] != 0)
        a[c], a[piv] = a[piv], a[c]
        d = a[c][c]
        a[c] = [x / d for x in a[c]]
        for r in range(n):
            if r != c and a[r][c] != 0:
                s = a[r][c]
                a[r] = [x - s * y for x, y in zip(a[r], a[c])]
    return [[a[i][n + j] for j in range(n)] for i in range(n)]


def _exact_det(M):
    n = len(M)
    a = [[Fraction(int(M[i][j])) for j in range(n)] for i in range(n)]
    det = Fraction(1)
    for c in range(n):
        piv = next((r for r in range(c, n) if a[r][c] != 0), None)
        if piv is None:
            return Fraction(0)
        if piv != c:
            a[c], a[piv] = a[piv], a[c]
            det = -det
        det *= a[c][c]
        for r in range(c + 1, n):
            s = a[r][c] / a[c][c]
            a[r] = [x - s * y for x, y in zip(a[r], a[c])]
    return det


def test_P_inverse_is_exact_and_matches_printed_step5_except_f4_sign():
    P, Pinv, _, _ = O.matrices([0, 0, 0])
    assert _exact_det(P.astype(int).tolist()) == -(2 ** 27)
    exact = np.array([[float(x) for x in r] for r in _exact_inverse(P.astype(int).tolist())])
    np.testing.assert_allclose(Pinv, exact, rtol=0, atol=1e-14)
    rows = _rows("app_d_step5_population_rows.txt")
    printed = np.array([[int(x) for x in r[2:]] for r in rows], float) / np.array([int(r[1]) for r in rows])[:, None]
    diff = np.abs(printed - exact) > 1e-14
    # Reading R6: the only disagreement is the sign of kappa~'_010 in f~_4 (e_4 = (0,-1,0)).
    assert list(zip(*np.nonzero(diff))) == [(4, IX["010"])]
    assert printed[4, IX["010"]] == 0.5 and exact[4, IX["010"]] == -0.5


# ------------------------------------------------------------------ frame shift
@pytest.mark.parametrize("u", [(0.0, 0.0, 0.0), (0.07, -0.02, 0.11), (-0.3, 0.25, -0.1)])
def test_frame_shift_is_the_central_moment_definition(u):
    e, _, mnp = O.lattice()
    P, _, Fu, Fi = O.matrices(u)
    f = _state(1)
    # brute force: kappa_mnp = sum_a f_a (e_ax - ux)^m (e_ay - uy)^n (e_az - uz)^p
    brute = np.array([np.sum(f * np.prod((e - np.array(u)) ** mnp[k], axis=1)) for k in range(27)])
    np.testing.assert_allclose(Fu @ (P @ f), brute, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(Fu @ Fi, np.eye(27), atol=1e-15)
    # lower triangular in the sense of the binomial expansion: only lower exponents enter
    for k in range(27):
        for j in range(27):
            if np.any(mnp[j] > mnp[k]):
                assert Fu[k, j] == 0.0


# ------------------------------------------------------------------ equilibrium
def test_rest_equilibrium_gives_standard_d3q27_weights():
    e, _, _ = O.lattice()
    w = O.feq(1.0, [0, 0, 0])
    expect = {0: 8 / 27, 1: 2 / 27, 2: 1 / 54, 3: 1 / 216}
    for a in range(27):
        assert w[a] == pytest.approx(expect[int(np.abs(e[a]).sum())], abs=1e-15)


@pytest.mark.parametrize("rho,u", [(1.0, (0.0, 0.0, 0.0)), (1.03, (0.05, -0.04, 0.02)), (0.97, (-0.2, 0.1, 0.15))])
def test_equilibrium_moments(rho, u):
    e, _, mnp = O.lattice()
    fe = O.feq(rho, u)
    assert fe.sum() == pytest.approx(rho, abs=1e-14)
    np.testing.assert_allclose(fe @ e, rho * np.array(u), atol=1e-15)
    c = np.array([1.0, 0.0, 1.0 / 3.0])
    kap = np.array([np.sum(fe * np.prod((e - np.array(u)) ** mnp[k], axis=1)) for k in range(27)])
    np.testing.assert_allclose(kap, rho * c[mnp].prod(1), atol=1e-14)
    # product form phi(0)=2/3-u^2, phi(+-1)=(1/3+u^2+-u)/2 in each direction
    def phi(ea, ud):
        return 2.0 / 3.0 - ud * ud if ea == 0 else (1.0 / 3.0 + ud * ud + ea * ud) / 2.0
    prod = np.array([rho * phi(e[a, 0], u[0]) * phi(e[a, 1], u[1]) * phi(e[a, 2], u[2]) for a in range(27)])
    np.testing.assert_allclose(fe, prod, atol=1e-15)


# ------------------------------------------------------------------ attractors
def _printed_attractors(k, rho):
    """Closed forms printed in Sec. 3.4 (continuous list) for orders 4-6."""
    return {
        "220": (k["200"] * k["020"] + 2 * k["110"] ** 2) / rho,
        "202": (k["200"] * k["002"] + 2 * k["101"] ** 2) / rho,
        "022": (k["020"] * k["002"] + 2 * k["011"] ** 2) / rho,
        "211": (k["200"] * k["011"] + 2 * k["110"] * k["101"]) / rho,
        "121": (k["020"] * k["101"] + 2 * k["110"] * k["011"]) / rho,
        "112": (k["002"] * k["110"] + 2 * k["101"] * k["011"]) / rho,
        "122": 2 / (5 * rho) * (k["020"] * k["102"] + k["002"] * k["120"] + 4 * k["011"] * k["111"]
                                + 2 * (k["101"] * k["021"] + k["110"] * k["012"])),
        "212": 2 / (5 * rho) * (k["200"] * k["012"] + k["002"] * k["210"] + 4 * k["101"] * k["111"]
                                + 2 * (k["110"] * k["102"] + k["011"] * k["201"])),
        "221": 2 / (5 * rho) * (k["200"] * k["021"] + k["020"] * k["201"] + 4 * k["110"] * k["111"]
                                + 2 * (k["011"] * k["210"] + k["101"] * k["120"])),
        "222": 1 / (3 * rho) * (k["200"] * k["022"] + k["020"] * k["202"] + k["002"] * k["220"]
                                + 4 * (k["110"] * k["112"] + k["101"] * k["121"] + k["011"] * k["211"])),
    }


def test_general_attractor_reproduces_printed_closed_forms():
    rng = np.random.default_rng(7)
    for _ in range(20):
        pi = rng.standard_normal(27)
        rho = 1.0 + 0.1 * rng.random()
        pi[0] = rho
        pi[1:4] = 0.0
        k = {name: pi[i] for i, name in enumerate(ORDER)}
        D = np.array([k["200"], k["020"], k["002"], k["110"], k["011"], k["101"]]) / rho
        printed = _printed_attractors(k, rho)
        for name, val in printed.items():
            m, n, p = map(int, name)
            assert O.attractor(m, n, p, D, pi) == pytest.approx(val, rel=1e-13, abs=1e-15), name
        # Reading R3: the discrete list prints kappa_011 kappa_012 in kappa^Mv_122;
        # the general formula gives kappa_110 kappa_012 (as the continuous list does).
        typo = printed["122"] - 2 / (5 * rho) * 2 * (k["110"] - k["011"]) * k["012"]
        assert abs(O.attractor(1, 2, 2, D, pi) - typo) > 1e-9


def test_low_order_attractors_with_equilibrium_diffusion_tensor():
    pi = np.zeros(27)
    pi[0] = 1.3
    D = np.array([1 / 3, 1 / 3, 1 / 3, 0, 0, 0])
    for name, expect in [("200", 1.3 / 3), ("020", 1.3 / 3), ("002", 1.3 / 3), ("110", 0.0), ("100", 0.0)]:
        m, n, p = map(int, name)
        assert O.attractor(m, n, p, D, pi) == pytest.approx(expect, abs=1e-15)


# ------------------------------------------------------------------ collision
@pytest.mark.parametrize("seed", range(4))
def test_mass_conserved_and_momentum_gains_force(seed):
    e, _, _ = O.lattice()
    rng = np.random.default_rng(seed)
    f = _state(seed, rho=1 + 0.05 * rng.random(), u=tuple(0.08 * rng.uniform(-1, 1, 3)))
    om = rng.uniform(0.2, 1.95, 27)
    F = 1e-3 * rng.uniform(-1, 1, 3)
    ft, kpre, kpost = O.collide_node(f, om, F, return_moments=True)
    assert ft.sum() == pytest.approx(f.sum(), rel=0, abs=1e-15)
    np.testing.assert_allclose(ft @ e, f @ e + F, rtol=0, atol=1e-16)
    # first-order central moments: -F/2 before, +F/2 after, for any omega_1..3
    np.testing.assert_allclose(kpre[1:4], -F / 2, atol=1e-16)
    np.testing.assert_allclose(kpost[1:4], F / 2, atol=1e-16)


@pytest.mark.parametrize("seed", range(3))
def test_equilibrium_is_fixed_point_without_force(seed):
    rng = np.random.default_rng(10 + seed)
    u = 0.1 * rng.uniform(-1, 1, 3)
    fe = O.feq(1 + 0.1 * rng.random(), u)
    om = rng.uniform(0.05, 1.99, 27)
    np.testing.assert_allclose(O.collide_node(fe, om), fe, rtol=0, atol=1e-15)


def test_unit_rates_collapse_to_equilibrium():
    e, _, _ = O.lattice()
    f = _state(3, amp=0.3)
    rho = f.sum()
    u = (f @ e) / rho
    np.testing.assert_allclose(O.collide_node(f, np.ones(27)), O.feq(rho, u), atol=1e-15)


def test_each_group_relaxes_at_its_own_rate():
    """Without force, second- and third-order groups relax linearly:
    kappa~ = kappa + omega (kappa^eq - kappa) with the group's own omega."""
    f = _state(5, amp=0.2)
    base = np.ones(27)
    _, kpre, k1 = O.collide_node(f, base, return_moments=True)
    rho = kpre[0]
    groups = {
        4: lambda k: k[IX["110"]], 5: lambda k: k[IX["101"]], 6: lambda k: k[IX["011"]],
        7: lambda k: k[IX["200"]] + k[IX["020"]] + k[IX["002"]],
        8: lambda k: k[IX["200"]] - k[IX["020"]], 9: lambda k: k[IX["200"]] - k[IX["002"]],
        10: lambda k: k[IX["120"]] + k[IX["102"]], 11: lambda k: k[IX["120"]] - k[IX["102"]],
        12: lambda k: k[IX["210"]] + k[IX["012"]], 13: lambda k: k[IX["210"]] - k[IX["012"]],
        14: lambda k: k[IX["201"]] + k[IX["021"]], 15: lambda k: k[IX["201"]] - k[IX["021"]],
        16: lambda k: k[IX["111"]],
    }
    eq = {7: rho}
    for j, g in groups.items():
        om = base.copy()
        om[j] = 0.3
        _, kp, kt = O.collide_node(f, om, return_moments=True)
        target = eq.get(j, 0.0)
        assert g(kt) == pytest.approx(g(kp) + 0.3 * (target - g(kp)), rel=1e-12, abs=1e-16), j
        # every other group is unaffected by omega_j
        for i, h in groups.items():
            if i != j:
                assert h(kt) == pytest.approx(h(k1), abs=1e-15), (j, i)


# Combined moments of orders 4-6 and the rate that relaxes each one
# (Appendix D Step 3): omega_17..19 the fourth-order combinations 4s1, 4d1,
# 4d2; omega_20..22 the moments 211, 121, 112; omega_23..25 122, 212, 221;
# omega_26 the sixth-order moment 222.
HIGH_GROUPS = {
    17: lambda k: k[IX["220"]] + k[IX["202"]] + k[IX["022"]],
    18: lambda k: k[IX["220"]] + k[IX["202"]] - k[IX["022"]],
    19: lambda k: k[IX["220"]] - k[IX["202"]],
    20: lambda k: k[IX["211"]], 21: lambda k: k[IX["121"]], 22: lambda k: k[IX["112"]],
    23: lambda k: k[IX["122"]], 24: lambda k: k[IX["212"]], 25: lambda k: k[IX["221"]],
}


@pytest.mark.parametrize("j", sorted(HIGH_GROUPS) + [26])
def test_each_higher_order_group_relaxes_at_its_own_rate(j):
    """Orders 4-6, one rate at a time.  With F = 0 and every other rate 1, the
    post-collision orders 2 and 3 are at equilibrium (kappa~_200 = rho c_s^2,
    off-diagonal and third-order moments 0), so the attractors built from them
    (Sec. 3.5, Eq. Mvcmattractor3D) take closed forms: kappa^Mv_220 = kappa^Mv_202
    = kappa^Mv_022 = rho c_s^4 (4s1 -> rho/3, 4d1 -> rho/9, 4d2 -> 0), the mixed
    fourth- and fifth-order attractors vanish, and kappa^Mv_222 =
    (c_s^2 / 3) (kappa~_220 + kappa~_202 + kappa~_022) with the post-collision
    fourth order.  The group relaxed with omega_j must move by
    omega_j (kappa^Mv - kappa) and every other group must keep its unit-rate
    value; a swap of two rates (e.g. omega_20 with omega_23) fails here."""
    f = _state(7 + j, amp=0.25)
    base = np.ones(27)
    _, _, k1 = O.collide_node(f, base, return_moments=True)
    om = base.copy()
    om[j] = 0.35
    _, kp, kt = O.collide_node(f, om, return_moments=True)
    rho = kp[0]
    cs2 = 1.0 / 3.0
    eq4 = {17: 3 * rho * cs2 * cs2, 18: rho * cs2 * cs2, 19: 0.0}
    if j == 26:
        target = cs2 / 3.0 * (kt[IX["220"]] + kt[IX["202"]] + kt[IX["022"]])
        assert target == pytest.approx(rho / 27.0, rel=1e-14)  # fourth order at equilibrium here
        got, pre = kt[IX["222"]], kp[IX["222"]]
    else:
        target = eq4.get(j, 0.0)
        got, pre = HIGH_GROUPS[j](kt), HIGH_GROUPS[j](kp)
    assert got == pytest.approx(pre + 0.35 * (target - pre), rel=1e-12, abs=1e-16), j
    for i, h in HIGH_GROUPS.items():
        if i != j:
            assert h(kt) == pytest.approx(h(k1), abs=1e-15), (j, i)
    if j not in (17, 18, 19, 26):
        # the sixth-order moment sees the fourth-order combinations only
        assert kt[IX["222"]] == pytest.approx(k1[IX["222"]], abs=1e-15), j


@pytest.mark.parametrize("j", [17, 18, 19])
def test_sixth_order_attractor_uses_the_post_collision_fourth_order(j):
    """A fourth-order rate away from 1 leaves the fourth order off equilibrium
    after the collision; with omega_26 = 1, kappa~_222 must equal the attractor
    (c_s^2 / 3)(kappa~_220 + kappa~_202 + kappa~_022) of those post-collision
    values (orders 2 and 3 at equilibrium), not of the pre-collision ones."""
    f = _state(31 + j, amp=0.3)
    om = np.ones(27)
    om[j] = 1.7
    _, kp, kt = O.collide_node(f, om, return_moments=True)
    post = kt[IX["220"]] + kt[IX["202"]] + kt[IX["022"]]
    pre = kp[IX["220"]] + kp[IX["202"]] + kp[IX["022"]]
    assert abs(post - pre) > 1e-4 * kp[0]
    assert kt[IX["222"]] == pytest.approx(post / 9.0, rel=1e-13)
    assert abs(kt[IX["222"]] - pre / 9.0) > 1e-6


def _moment_order(j):
    """Order of the moments relaxed with omega_j, read off the lattice's moment
    exponents of one member of the group (Appendix D Step 3)."""
    member = {4: "110", 5: "101", 6: "011", 7: "200", 8: "200", 9: "200", 10: "120", 11: "120",
              12: "210", 13: "210", 14: "201", 15: "201", 16: "111", 17: "220", 18: "220", 19: "220",
              20: "211", 21: "121", 22: "112", 23: "122", 24: "212", 25: "221", 26: "222"}[j]
    _, _, mnp = O.lattice()
    return int(mnp[IX[member]].sum())


@pytest.mark.parametrize("nu", [1e-6, 1e-3, 0.01, 1.0 / 6.0, 0.5, 10.0])
def test_order_scaled_rates_are_the_trapezoidal_discretisation_of_order_times_omega_fp(nu):
    """Eq. (FPcoll3d): the continuous model relaxes a moment of order n = m+n+p at
    n omega_FP.  Second order: 2 omega_FP, and the shear viscosity fixes the
    discrete omega_2 through Eq. (transportcoeff3DFPCLBM).  The lattice rates are
    the Henon (trapezoidal, Crank-Nicolson) integration of a linear relaxation at
    rate lambda over one step: omega = lambda / (1 + lambda / 2).  So omega_FP
    follows from omega_2 and every higher group must carry lambda = n omega_FP
    with n its moments' order; all rates stay in (0, 2)."""
    om = O.omega_table(nu, mode="order_scaled")
    w2 = om[4]
    lam2 = w2 / (1.0 - w2 / 2.0)  # inverse of the trapezoidal map
    omega_fp = lam2 / 2.0
    assert nu == pytest.approx((1.0 / 3.0) / (2.0 * omega_fp), rel=1e-12)  # nu = c_s^2 / lambda_2
    for j in range(10, 27):
        n = _moment_order(j)
        lam = n * omega_fp
        assert om[j] == pytest.approx(lam / (1.0 + lam / 2.0), rel=1e-13), (j, n)
        assert 0.0 < om[j] < 2.0
    # bulk and shear rates are not order-scaled
    assert om[7] == 1.0 and np.all(om[[4, 5, 6, 8, 9]] == w2)


def test_order_scaled_rates_approach_the_continuous_ratio_for_slow_relaxation():
    """For slow relaxation (omega_2 -> 0, large viscosity) the discrete rates tend
    to the continuous ones, omega_n / omega_2 -> n / 2 (Eq. FPcoll3d), with an
    O(omega_2) deviation; for fast relaxation they stay below 2."""
    for nu in [1e3, 1e5, 1e7]:
        om = O.omega_table(nu, mode="order_scaled")
        w2 = om[4]
        for j in range(10, 27):
            n = _moment_order(j)
            assert om[j] / w2 == pytest.approx(n / 2.0, rel=2 * w2 * n), (nu, j)
    om = O.omega_table(1e-9, mode="order_scaled")
    assert np.all(om < 2.0) and np.all(om[10:] > om[4] - 1e-9)


def _cube_maps():
    e, _, _ = O.lattice()
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product([1, -1], repeat=3):
            R = np.zeros((3, 3), int)
            for i in range(3):
                R[i, perm[i]] = signs[i]
            Re = e @ R.T
            yield R, np.array([int(np.nonzero((e == Re[a]).all(1))[0][0]) for a in range(27)])


@pytest.mark.parametrize("variant", ["paper", "order_scaled", "grouped"])
def test_collision_is_equivariant_under_the_48_cube_symmetries(variant):
    om = O.omega_table(0.004, mode="order_scaled" if variant == "order_scaled" else "paper")
    if variant == "grouped":
        om[7] = 1.3
        om[[10, 12, 14]] = 1.2
        om[[11, 13, 15]] = 1.5
        om[16] = 1.45
        om[17:20] = 1.25  # 4s1/4d1/4d2 are only isotropic with one common rate
        om[20:23] = 1.6
        om[23:26] = 0.9
        om[26] = 1.7
    f = _state(11, amp=0.15)
    F = np.array([1e-3, 2e-3, -3e-3])
    g = O.collide_node(f, om, F)
    for R, idx in _cube_maps():
        fr = np.zeros(27)
        fr[idx] = f
        ref = np.zeros(27)
        ref[idx] = g
        np.testing.assert_allclose(O.collide_node(fr, om, R @ F), ref, rtol=0, atol=5e-16)


def test_output_central_moments_are_the_relaxed_moments():
    e, _, mnp = O.lattice()
    f = _state(13, amp=0.2)
    F = np.array([2e-3, -1e-3, 5e-4])
    ft, kpre, kpost = O.collide_node(f, O.omega_table(0.01), F, return_moments=True)
    rho = f.sum()
    u = (f @ e + F / 2) / rho
    brute_pre = np.array([np.sum(f * np.prod((e - u) ** mnp[k], axis=1)) for k in range(27)])
    brute_post = np.array([np.sum(ft * np.prod((e - u) ** mnp[k], axis=1)) for k in range(27)])
    np.testing.assert_allclose(kpre, brute_pre, atol=1e-15)
    np.testing.assert_allclose(kpost, brute_post, atol=1e-15)


def test_sources_enter_with_half_weight_factor():
    """sigma enters as (1 - omega/2) sigma: with a force and omega=1 for the shear
    group, kappa~_120 + kappa~_102 picks up (1/2) sigma_3s1 on top of relaxing to 0,
    sigma_120 = (Fx/rho) kappa_020 + 2 (Fy/rho) kappa_110 (Eq. cmupdatesourceD3Q27)."""
    f = _state(17, amp=0.1)
    F = np.array([3e-3, -2e-3, 1e-3])
    om = np.ones(27)
    om[10] = 0.4
    _, kp, kt = O.collide_node(f, om, F, return_moments=True)
    rho = f.sum()
    s120 = F[0] / rho * kp[IX["020"]] + 2 * F[1] / rho * kp[IX["110"]]
    s102 = F[0] / rho * kp[IX["002"]] + 2 * F[2] / rho * kp[IX["101"]]
    k3s1 = kp[IX["120"]] + kp[IX["102"]]
    expect = k3s1 + 0.4 * (0.0 - k3s1) + (1 - 0.2) * (s120 + s102)
    assert kt[IX["120"]] + kt[IX["102"]] == pytest.approx(expect, rel=1e-12)


# ------------------------------------------------------------------ streaming
def test_stream_pull_definition_brute_force():
    e, opp, _ = O.lattice()
    nx, ny, nz = 5, 4, 3
    g = np.random.default_rng(0).random((27, nz, ny, nx))
    f = O.stream(g, walls_y=False)
    fw = O.stream(g, walls_y=True)
    for a in range(27):
        for z in range(nz):
            for y in range(ny):
                for x in range(nx):
                    xs, ys, zs = (x - e[a, 0]) % nx, (y - e[a, 1]) % ny, (z - e[a, 2]) % nz
                    assert f[a, z, y, x] == g[a, zs, ys, xs]
                    yraw = y - e[a, 1]
                    if 0 <= yraw < ny:
                        assert fw[a, z, y, x] == g[a, zs, yraw, xs]
                    else:  # halfway bounce-back: own node, opposite direction
                        assert fw[a, z, y, x] == g[opp[a], z, y, x]


def test_stream_is_a_permutation_of_each_direction_and_bounce_back_keeps_mass():
    g = np.random.default_rng(1).random((27, 4, 6, 5))
    f = O.stream(g)
    np.testing.assert_allclose(f.sum((1, 2, 3)), g.sum((1, 2, 3)), rtol=1e-14)
    fw = O.stream(g, walls_y=True)
    assert fw.sum() == pytest.approx(g.sum(), rel=1e-14)


# ------------------------------------------------------------------ physics
@pytest.mark.parametrize("nu", [0.01, 0.05, 0.15])
def test_shear_wave_decay_gives_the_chapman_enskog_viscosity(nu):
    """Eq. (transportcoeff3DFPCLBM): nu = c_s^2 (1/omega - 1/2)."""
    nx = 64
    rho, u = W.shear_wave(nx, 1, 1, amp=1e-4)
    g = O.init(rho, u)
    om = O.omega_table(nu)
    k = 2 * np.pi / nx
    x = np.arange(nx)
    amps, t0, t1 = [], 20, 20 + int(0.5 / (nu * k * k))
    g = O.run(g, om, steps=t0)
    for steps in (0, t1 - t0):
        g = O.run(g, om, steps=steps) if steps else g
        _, uu = O.macroscopic(g)
        amps.append(2 * np.mean(uu[1, 0, 0] * np.cos(k * x)))
    nu_meas = -np.log(amps[1] / amps[0]) / (k * k * (t1 - t0))
    assert nu_meas == pytest.approx(nu, rel=0.01)


def test_taylor_green_small_amplitude_decay_rate():
    """Linear limit: velocity amplitude decays as exp(-3 nu k^2 t), KE as exp(-6 nu k^2 t)."""
    n = 16
    nu = 0.05
    rho, u = W.taylor_green(n, u0=1e-4)
    g = O.init(rho, u)
    om = O.omega_table(nu)
    k = 2 * np.pi / n

    def ke(state):
        r, uu = O.macroscopic(state)
        return 0.5 * np.sum(r * (uu ** 2).sum(0))

    g = O.run(g, om, steps=10)
    e0 = ke(g)
    T = 60
    g = O.run(g, om, steps=T)
    rate = -np.log(ke(g) / e0) / T
    assert rate == pytest.approx(6 * nu * k * k, rel=0.02)


def test_poiseuille_steady_state_with_halfway_bounce_back():
    """Steady force-driven channel: interior second differences equal -F/(rho nu)
    (exact for a parabola), zero crossing near the half-link wall position, and the
    wall momentum exchange balances the body force."""
    ny, nu, Fx = 16, 0.1, 1e-5
    e, opp, _ = O.lattice()
    rho, u = W.channel_at_rest(1, ny, 1)
    g = O.init(rho, u)
    om = O.omega_table(nu)
    F = (Fx, 0.0, 0.0)
    g = O.run(g, om, F, walls_y=True, steps=6000)
    _, uu = O.macroscopic(g, F)
    ux = uu[0, 0, :, 0]
    d2 = ux[2:] - 2 * ux[1:-1] + ux[:-2]
    np.testing.assert_allclose(d2, -Fx / nu, rtol=2e-3)
    y = np.arange(ny) + 0.5
    analytic = Fx / (2 * nu) * y * (ny - y)
    assert np.max(np.abs(ux - analytic)) / analytic.max() < 0.02
    # momentum exchange with the walls: links leaving y=0 downward and y=ny-1 upward
    wall = 0.0
    for a in range(27):
        if e[a, 1] == -1:
            wall += 2 * g[a, 0, 0, 0] * e[a, 0]
        if e[a, 1] == 1:
            wall += 2 * g[a, 0, ny - 1, 0] * e[a, 0]
    assert wall == pytest.approx(Fx * ny, rel=1e-3)  # force of the fluid on the walls


# ------------------------------------------------------------------ Maxwellian comparison model
def test_markovian_attractors_at_equilibrium_are_the_maxwellian_central_moments():
    """Sec. 1 and Sec. 3: with the lower moments at their equilibrium values the
    Markovian attractors coincide with the Maxwellian's central moments.  Built
    up order by order from the general formula, the attractor of every moment
    equals the central moment of f^eq (the discrete Maxwellian of reading R2)."""
    e, _, mnp = O.lattice()
    rho = 1.17
    fe = O.feq(rho, (0.0, 0.0, 0.0))
    maxwell = np.array([fe @ np.prod(e ** m, axis=1) for m in mnp])
    pi = np.zeros(27)
    pi[0] = rho
    D = np.array([1 / 3, 1 / 3, 1 / 3, 0, 0, 0])
    for order in range(2, 7):
        for q, m in enumerate(mnp):
            if sum(m) == order:
                pi[q] = O.attractor(*m, D, pi)
    np.testing.assert_allclose(pi, maxwell, rtol=0, atol=1e-15)


@pytest.mark.parametrize("seed", range(3))
def test_maxwellian_model_relaxes_higher_orders_to_fixed_values(seed):
    """MCM comparison model (reading R22): with unit rates for orders >= 4 the
    post-collision moments of orders >= 4 are rho c_a c_b c_c whatever the
    second-order state; the FPC model's are not (they follow the post-collision
    second order)."""
    rng = np.random.default_rng(40 + seed)
    f = _state(60 + seed, amp=0.3)
    om = np.ones(27)
    om[4:10] = rng.uniform(1.2, 1.9, 6)
    _, kpre, kpost = O.collide_node(f, om, return_moments=True, attractor="maxwell")
    rho = kpre[0]
    c = {0: 1.0, 1: 0.0, 2: 1 / 3}
    for q, name in enumerate(ORDER):
        if sum(map(int, name)) >= 4:
            a, b, d = map(int, name)
            assert kpost[q] == pytest.approx(rho * c[a] * c[b] * c[d], abs=1e-15), name
    _, _, kfpc = O.collide_node(f, om, return_moments=True)
    assert abs(kfpc[IX["220"]] - rho / 9) > 1e-6
    # orders <= 3 are the same in both models
    np.testing.assert_allclose(kfpc[:17], kpost[:17], rtol=0, atol=1e-16)


def test_maxwellian_model_keeps_the_conservation_laws_and_fixed_point():
    e, _, _ = O.lattice()
    f = _state(71, amp=0.2)
    rng = np.random.default_rng(71)
    om = rng.uniform(0.3, 1.9, 27)
    F = (2e-4, -1e-4, 3e-4)
    ft = O.collide_node(f, om, F, attractor="maxwell")
    assert ft.sum() == pytest.approx(f.sum(), rel=0, abs=1e-15)
    np.testing.assert_allclose(ft @ e, f @ e + np.array(F), rtol=0, atol=1e-16)
    fe = O.feq(1.05, (0.03, -0.02, 0.05))
    np.testing.assert_allclose(O.collide_node(fe, om, attractor="maxwell"), fe, rtol=0, atol=1e-15)


def _crossing_shear_wave_amplitudes(attractor, marks, nx=30, ny=2, nz=30, amp=1e-5, nu=1e-7):
    x, z = np.arange(nx), np.arange(nz)
    Z, _, X = np.meshgrid(z, np.arange(ny), x, indexing="ij")
    k = 2 * np.pi / nx
    mode = np.cos(k * X) * np.cos(k * Z)
    u = np.zeros((3, nz, ny, nx))
    u[1] = amp * mode
    g = O.init(np.ones((nz, ny, nx)), u)
    om = O.omega_table(nu)
    out, done = [], 0
    for m in marks:
        g = O.run(g, om, steps=m - done, attractor=attractor)
        done = m
        _, uu = O.macroscopic(g)
        out.append((uu[1] * mode).sum() / (mode * mode).sum() / amp)
    return np.array(out), 2 * k * k * nu


def test_crossing_shear_waves_show_hyperviscosity_only_with_maxwellian_attractors():
    """Sec. 4 (orthogonal crossing shear waves, nu = 1e-7, L = 30): the wave
    should hardly decay (the exact rate nu (k_x^2 + k_z^2) is 8.8e-9 per step).
    With Maxwellian attractors for the higher moments it decays at a rate that
    is orders of magnitude larger (numerical hyperviscosity); with the
    Markovian attractors of FPC-LBM it does not.  Rates are measured after the
    initial odd-even transient of omega ~ 2 has settled."""
    marks = [300, 2300]
    a_fpc, exact = _crossing_shear_wave_amplitudes("fpc", marks)
    a_mcm, _ = _crossing_shear_wave_amplitudes("maxwell", marks)
    rate_fpc = np.log(a_fpc[0] / a_fpc[1]) / (marks[1] - marks[0])
    rate_mcm = np.log(a_mcm[0] / a_mcm[1]) / (marks[1] - marks[0])
    assert rate_mcm > 1000 * exact
    assert rate_mcm > 50 * rate_fpc
    assert abs(a_fpc[1] - 1.0) < 0.02 and a_mcm[1] < 0.92


# ------------------------------------------------------------------ walls on every face, moving lid
@pytest.mark.parametrize("nu", [0.1, 0.02])
def test_moving_wall_bounce_back_gives_exact_plane_couette_flow(nu):
    """Sec. 4 cavity boundary (reading R23): halfway bounce-back with the
    moving-wall momentum correction.  Between a resting wall half a link below
    y = 0 and a wall moving at U half a link above y = ny - 1 the steady
    solution is u_x = U (y + 1/2) / ny, which the scheme reproduces to
    rounding."""
    nx, ny, nz, U = 2, 8, 2, 0.02
    g = O.init(np.ones((nz, ny, nx)), np.zeros((3, nz, ny, nx)))
    g = O.run(g, O.omega_table(nu), walls="y", lid=(U, 0, 0), steps=int(12 * ny * ny / nu))
    _, u = O.macroscopic(g)
    exact = U * (np.arange(ny) + 0.5) / ny
    np.testing.assert_allclose(u[0], np.broadcast_to(exact[None, :, None], u[0].shape), rtol=0, atol=1e-12 * U)
    assert np.abs(u[1]).max() < 1e-14 and np.abs(u[2]).max() < 1e-14


def _cavity(n, lid, steps, nu=0.05):
    g = O.init(np.ones((n, n, n)), np.zeros((3, n, n, n)))
    return O.run(g, O.omega_table(nu), walls="xyz", lid=lid, steps=steps)


def test_lid_driven_cavity_is_mirror_symmetric_and_keeps_mass():
    """Cubic cavity with the lid moving along x: the flow is symmetric under
    z -> nz - 1 - z (u_z odd), and a tangential lid changes no mass."""
    n, U = 8, 0.05
    g = _cavity(n, (U, 0, 0), 150)
    rho, u = O.macroscopic(g)
    m = rho[::-1]
    np.testing.assert_allclose(rho, m, rtol=0, atol=1e-14)
    np.testing.assert_allclose(u[0], u[0][::-1], rtol=0, atol=1e-15)
    np.testing.assert_allclose(u[1], u[1][::-1], rtol=0, atol=1e-15)
    np.testing.assert_allclose(u[2], -u[2][::-1], rtol=0, atol=1e-15)
    assert rho.sum() == pytest.approx(n ** 3, rel=1e-13)
    assert u[0][:, -1].mean() > 0.1 * U  # the lid drives the top layer


def test_lid_driven_cavity_rotates_with_the_lid_direction():
    """The lid moving along z gives the x <-> z mirror image of the lid moving
    along x (walls on every face, cubic box): checks the x- and z-wall paths
    against each other."""
    n, U = 7, 0.05
    rx, ux = O.macroscopic(_cavity(n, (U, 0, 0), 60))
    rz, uz = O.macroscopic(_cavity(n, (0, 0, U), 60))
    sw = lambda a: np.swapaxes(a, 0, 2)  # [z, y, x] -> [x, y, z]
    np.testing.assert_allclose(rz, sw(rx), rtol=0, atol=1e-14)
    np.testing.assert_allclose(uz[2], sw(ux[0]), rtol=0, atol=1e-15)
    np.testing.assert_allclose(uz[0], sw(ux[2]), rtol=0, atol=1e-15)
    np.testing.assert_allclose(uz[1], sw(ux[1]), rtol=0, atol=1e-15)


def test_specular_symmetry_plane_reproduces_the_lower_half_of_the_full_channel():
    """Sec. 4 half channel (reading R24): a wall below y = 0 and a specular
    symmetry plane above y = H - 1 evolve exactly like the lower half of the
    full channel of height 2H with walls on both sides, started from a state
    that is mirror-symmetric about the mid-plane (equivariance of the
    collision under the y mirror, exact to rounding)."""
    nx, H, nz = 6, 5, 4
    e, _, _ = O.lattice()
    mir = np.array([np.where((e[:, 0] == a[0]) & (e[:, 1] == -a[1]) & (e[:, 2] == a[2]))[0][0] for a in e])
    half = O.feq(1.0, (0.0, 0.0, 0.0))[:, None, None, None] * W.random_factors((27, nz, H, nx), seed=8, amplitude=0.2)
    full = np.concatenate([half, half[mir][:, :, ::-1, :]], axis=2)
    om = O.omega_table(0.03)
    F = (2e-5, 0.0, 1e-5)
    gh = O.run(half, om, F, walls="ys", steps=6)
    gf = O.run(full, om, F, walls="y", steps=6)
    np.testing.assert_allclose(gh, gf[:, :, :H, :], rtol=0, atol=1e-15)
    np.testing.assert_allclose(gf[:, :, H:, :], gf[mir][:, :, H - 1::-1, :], rtol=0, atol=1e-15)


@pytest.mark.parametrize("damping", [False, True])
def test_smagorinsky_les_gives_the_model_eddy_viscosity_in_channel_flow(damping):
    """Reading R25 (Sec. 4 LES): in steady force-driven channel flow the shear
    stress balances the force, (nu + nu_t) du/dy = F (y_c - y), and the eddy
    viscosity the scheme develops is the model's nu_t = (C D)^2 |du/dy| with
    the van Driest factor D = 1 - exp(-y+ / 26), y+ counted from the wall half
    a link outside the first layer.  Checked away from the centre line (where
    du/dy -> 0): to 3 % without damping; to 10 % with it, where D changes by a
    factor 2 across the few layers of this 16-layer channel (a y+ offset of
    half a layer either way is off by 15-90 %)."""
    nx, ny, nz, nu = 2, 16, 2, 0.05
    F = 8 * nu * 0.05 / ny ** 2
    C, scale = 0.6, (6.0 if damping else 0.0)
    g = O.init(np.ones((nz, ny, nx)), np.zeros((3, nz, ny, nx)))
    g = O.run(g, O.omega_table(nu), (F, 0, 0), walls="y", steps=int(8 * ny * ny / nu), les=(C, scale, 26.0))
    _, u = O.macroscopic(g, force=(F, 0, 0))
    ux = u[0, 0, :, 0]
    j = np.arange(1, ny - 1)
    gam = (ux[2:] - ux[:-2]) / 2
    yw = np.minimum(j + 0.5, ny - 0.5 - j)
    D = 1 - np.exp(-yw * scale / 26.0) if damping else np.ones_like(yw)
    nut_model = (C * D) ** 2 * np.abs(gam)
    nut_seen = F * ((ny - 1) / 2 - j) / gam - nu
    far = np.abs(j - (ny - 1) / 2) > ny / 4
    assert nut_model[far].max() > 0.01 * nu
    np.testing.assert_allclose(nut_seen[far], nut_model[far], rtol=0.10 if damping else 0.03)


@pytest.mark.parametrize("walls,lid", [("", None), ("y", None), ("xyz", (0.03, 0.0, 0.01)), ("ys", None),
                                       ("xys", None), ("yz", (0.0, 0.0, 0.02))])
def test_pull_and_push_streaming_agree(walls, lid):
    """The pull gather the kernels use and the push scatter give the same
    populations for every boundary set (both written out independently)."""
    g = O.feq(1.0, (0.0, 0.0, 0.0))[:, None, None, None] * W.random_factors((27, 5, 6, 7), seed=4, amplitude=0.3)
    np.testing.assert_array_equal(O.stream(g, walls=walls, lid=lid), O.stream_push(g, walls=walls, lid=lid))


def test_streaming_in_place_without_double_buffer_is_caught():
    """Negative control for the A/B buffers: streaming that overwrites the
    state it reads (a single buffer, nodes visited in order) differs from the
    double-buffered step far beyond any parity tolerance."""
    g = O.feq(1.0, (0.0, 0.0, 0.0))[:, None, None, None] * W.random_factors((27, 4, 5, 6), seed=5, amplitude=0.3)
    e, _, _ = O.lattice()
    _, nz, ny, nx = g.shape
    f = g.copy()  # planted mistake: read and write the same array
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                for a in range(27):
                    f[a, z, y, x] = f[a, (z - e[a, 2]) % nz, (y - e[a, 1]) % ny, (x - e[a, 0]) % nx]
    good = O.stream(g)
    assert np.abs(f - good).max() > 1e-3 * np.abs(good).max()


# ------------------------------------------------------------------ diagnostics
def _grid(nx, ny, nz):
    z, y, x = np.meshgrid(np.arange(nz) + 0.5, np.arange(ny) + 0.5, np.arange(nx) + 0.5, indexing="ij")
    return x, y, z


@pytest.mark.parametrize("n", [8, 12])
def test_enstrophy_of_the_taylor_green_field_is_the_closed_form(n):
    """u = u0 sin kx cos ky cos kz, v = -u0 cos kx sin ky cos kz, w = 0 with
    k = 2 pi / n (cell-centred, periodic).  Its curl is
    (-u0 k cos kx sin ky sin kz, -u0 k sin kx cos ky sin kz, 2 u0 k sin kx sin ky cos kz);
    a centred difference of sin(k x) or cos(k x) equals the derivative times
    sin(k) / k, and the grid means of the squared products are 1/8, so
    1/2 sum |curl u|^2 = (3/8) u0^2 sin(k)^2 n^3."""
    u0, k = 0.05, 2 * np.pi / n
    x, y, z = _grid(n, n, n)
    u = np.stack([u0 * np.sin(k * x) * np.cos(k * y) * np.cos(k * z),
                  -u0 * np.cos(k * x) * np.sin(k * y) * np.cos(k * z), np.zeros_like(x)])
    w = O.vorticity(u)
    s = np.sin(k)
    np.testing.assert_allclose(w[2], 2 * u0 * s * np.sin(k * x) * np.sin(k * y) * np.cos(k * z), atol=1e-15)
    np.testing.assert_allclose(w[0], -u0 * s * np.cos(k * x) * np.sin(k * y) * np.sin(k * z), atol=1e-15)
    ens = 0.5 * float((w ** 2).sum())
    assert ens == pytest.approx(3.0 / 8.0 * u0 ** 2 * s ** 2 * n ** 3, rel=1e-12)
    # through the lattice state: f^eq of the field, rho = 1
    d = O.diagnostics(O.init(np.ones((n, n, n)), u))
    assert d["enstrophy"] == pytest.approx(ens, rel=1e-12)
    assert d["kinetic_energy"] == pytest.approx(0.5 * float((u ** 2).sum()), rel=1e-13)
    assert d["max_speed"] == pytest.approx(float(np.sqrt((u ** 2).sum(0)).max()), rel=1e-13)
    assert d["min_rho"] == pytest.approx(1.0, abs=1e-14)
    assert d["mass"] == pytest.approx(n ** 3, rel=1e-14)


@pytest.mark.parametrize("n", [6, 10])
def test_vorticity_of_the_abc_beltrami_flow_is_sin_k_times_the_velocity(n):
    """The Arnold-Beltrami-Childress field u = (A sin kz + C cos ky,
    B sin kx + A cos kz, C sin ky + B cos kx) has curl u = k u; with centred
    differences every derivative carries sin(k)/k, so the discrete curl is
    sin(k) u, element by element, in all three components (a wrong sign or
    index in any of the six derivatives fails)."""
    A, B, C = 0.03, -0.02, 0.05
    k = 2 * np.pi / n
    x, y, z = _grid(n, n + 0, n)
    u = np.stack([A * np.sin(k * z) + C * np.cos(k * y), B * np.sin(k * x) + A * np.cos(k * z),
                  C * np.sin(k * y) + B * np.cos(k * x)])
    np.testing.assert_allclose(O.vorticity(u), np.sin(k) * u, atol=1e-16)


@pytest.mark.parametrize("case", ["walls", "symmetry"])
def test_enstrophy_of_a_sine_profile_between_walls_and_under_a_symmetry_plane(case):
    """u_x(y) = sin(kappa (y + 1/2)) vanishes at the half-link wall y = -1/2 and is
    odd about it; with kappa = pi / H it also vanishes at the upper wall
    y = H - 1/2, with kappa = pi / (2H) it is even about the symmetry plane
    there.  The ghost layers (-u at a wall, mirrored tangential velocity at the
    plane) are then exact extensions, every centred difference is
    sin(kappa) cos(kappa (y + 1/2)), and the sum over y of cos^2 is H / 2:
    1/2 sum |curl u|^2 = (1/4) nx nz H sin(kappa)^2."""
    nx, ny, nz = 4, 10, 3
    kap = np.pi / ny if case == "walls" else np.pi / (2 * ny)
    walls = "y" if case == "walls" else "ys"
    _, y, _ = _grid(nx, ny, nz)
    u = np.stack([np.sin(kap * y), np.zeros_like(y), np.zeros_like(y)])
    w = O.vorticity(u, walls=walls)
    np.testing.assert_allclose(w[2], -np.sin(kap) * np.cos(kap * y), atol=1e-15)
    assert 0.5 * float((w ** 2).sum()) == pytest.approx(0.25 * nx * nz * ny * np.sin(kap) ** 2, rel=1e-12)
    # the same profile along z between z walls, and along x between x walls
    xg, _, zg = _grid(6, 5, 8)
    kz = np.pi / 8
    uz = np.stack([np.sin(kz * zg), np.zeros_like(zg), np.zeros_like(zg)])
    wz = O.vorticity(uz, walls="z")
    assert 0.5 * float((wz ** 2).sum()) == pytest.approx(0.25 * 6 * 5 * 8 * np.sin(kz) ** 2, rel=1e-12)
    kx = np.pi / 6
    ux = np.stack([np.zeros_like(xg), np.sin(kx * xg), np.zeros_like(xg)])
    wx = O.vorticity(ux, walls="x")
    assert 0.5 * float((wx ** 2).sum()) == pytest.approx(0.25 * 6 * 5 * 8 * np.sin(kx) ** 2, rel=1e-12)


def test_enstrophy_of_plane_couette_flow_under_a_moving_lid():
    """Plane Couette flow u_x = U (y + 1/2) / H between the resting wall at
    y = -1/2 and the lid at y = H - 1/2 moving with U: the ghost values -u (wall)
    and 2U - u (lid) lie on the same line, so every centred difference is U / H
    and the enstrophy is 1/2 nx nz H (U/H)^2.  A resting-wall ghost under the lid
    would give the top row a different slope."""
    nx, ny, nz, U = 5, 9, 4, 0.07
    _, y, _ = _grid(nx, ny, nz)
    u = np.stack([U * y / ny, np.zeros_like(y), np.zeros_like(y)])
    w = O.vorticity(u, walls="y", lid=(U, 0.0, 0.0))
    np.testing.assert_allclose(w[2], -U / ny, rtol=1e-13)
    np.testing.assert_allclose(w[:2], 0.0, atol=1e-17)
    assert 0.5 * float((w ** 2).sum()) == pytest.approx(0.5 * nx * nz * ny * (U / ny) ** 2, rel=1e-12)
    w_rest = O.vorticity(u, walls="y")
    assert abs(w_rest[2, :, -1, :] + U / ny).min() > 0.1 * U / ny


def test_diagnostic_sums_are_the_step7_fields():
    """Mass, momentum (with the F/2 shift of a post-collision state), kinetic
    energy, min rho and the non-finite count against Appendix D Step 7 computed
    by brute force over nodes and directions."""
    e, _, _ = O.lattice()
    rng = np.random.default_rng(3)
    nx, ny, nz = 5, 4, 3
    rho = 1 + 0.05 * rng.standard_normal((nz, ny, nx))
    u = 0.03 * rng.standard_normal((3, nz, ny, nx))
    f = O.init(rho, u) * (1 + 0.02 * rng.standard_normal((27, nz, ny, nx)))
    F = np.array([1e-4, -2e-4, 3e-4])
    d = O.diagnostics(f, F)
    mass = mom = ke = 0.0
    mom = np.zeros(3)
    rmin = np.inf
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                r = sum(f[a, z, y, x] for a in range(27))
                j = sum(f[a, z, y, x] * e[a] for a in range(27)) - F / 2
                mass += r
                mom += j
                ke += 0.5 * float(j @ j) / r
                rmin = min(rmin, r)
    assert d["mass"] == pytest.approx(mass, rel=1e-14)
    np.testing.assert_allclose(d["momentum"], mom, rtol=1e-12, atol=1e-16)
    assert d["kinetic_energy"] == pytest.approx(ke, rel=1e-12)
    assert d["min_rho"] == pytest.approx(rmin, rel=1e-15)
    assert d["n_nonfinite"] == 0
    f[3, 1, 2, 0] = np.nan
    f[5, 1, 2, 0] = np.inf
    f[0, 0, 0, 4] = -np.inf
    assert O.diagnostics(f, F)["n_nonfinite"] == 2
