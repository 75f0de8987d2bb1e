"""Host checks of the experiment drivers' analysis helpers (no GPU)."""
import numpy as np
import pytest

from paper_2410_09739_amd.experiments import closure_channel as CC


@pytest.mark.parametrize("ny", [32, 64])
def test_balance_eddy_viscosity_recovers_a_prescribed_profile(ny):
    """Mean momentum balance of a channel, (nu + nu_t) dU/dy - <u'v'> =
    u_tau^2 (1 - y/h): with U = c (y - y^2 / 2h) (a quadratic, whose centred
    difference is its exact derivative c (1 - y/h)), c = u_tau^2 / (3 nu) and a
    resolved stress <u'v'> = -u_tau^2 (1 - y/h) sin(pi y / 2h) / 2 (negative
    below the centreplane, antisymmetric about it), the eddy viscosity that
    closes the balance is nu_t = 3 nu (1 - sin(pi y / 2h) / 2) - nu at every
    row away from the walls (the wall rows use a ghost value)."""
    nu, ut = 4.4e-4, 0.0025
    h = ny / 2.0
    y = np.arange(ny) + 0.5
    c = ut * ut / (3 * nu)
    U = c * (y - y * y / (2 * h))
    uv = -0.5 * ut * ut * (1 - y / h) * np.sin(np.pi * y / (2 * h))
    got = CC.balance_eddy_viscosity({"uv": uv}, {"U": U}, ut, nu, cap=10 * nu)
    want = 3 * nu * (1 - 0.5 * np.sin(np.pi * y / (2 * h))) - nu
    np.testing.assert_allclose(got[1:-1], want[1:-1], rtol=1e-9, atol=1e-15)
    # no resolved stress and the laminar profile of nu: nothing to add
    lam = CC.balance_eddy_viscosity({"uv": np.zeros(ny)}, {"U": ut * ut / nu * (y - y * y / (2 * h))}, ut, nu,
                                    cap=10 * nu)
    assert np.max(np.abs(lam[1:-1])) <= 1e-12
    # clipped to [0, cap]: a profile steeper than the stress allows asks for no eddy viscosity
    steep = CC.balance_eddy_viscosity({"uv": np.zeros(ny)}, {"U": 10 * U}, ut, nu, cap=10 * nu)
    assert np.all(steep == 0.0)
    capped = CC.balance_eddy_viscosity({"uv": np.zeros(ny)}, {"U": 0.01 * U}, ut, nu, cap=2 * nu)
    assert np.all(capped[1:-1] == 2 * nu)


def test_output_gain_interpolates_the_bulk_velocity_linearly():
    """The closure study's output gain: with U_b(g) = U_plain + g (U_net - U_plain),
    the g that gives the fine U_b; the measured case of the 192 x 96 x 96 grid
    (plain 16.671, network 13.764, fine 15.729 u_tau) gives 0.324; outside
    [0.1, 2] it is clipped, and a network that leaves U_b unchanged keeps g = 1."""
    from paper_2410_09739_amd.experiments.closure_channel import output_gain
    for up, un, uf in [(18.0, 16.0, 16.5), (16.671, 13.764, 15.729), (10.0, 12.0, 11.0)]:
        g = output_gain(up, un, uf)
        assert up + g * (un - up) == pytest.approx(uf, rel=1e-12)
    assert output_gain(16.671, 13.764, 15.729) == pytest.approx(0.324, abs=5e-4)
    assert output_gain(18.0, 17.9, 10.0) == 2.0
    assert output_gain(18.0, 16.0, 18.5) == 0.1
    assert output_gain(18.0, 18.0, 16.0) == 1.0
