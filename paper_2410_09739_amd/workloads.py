"""Seeded synthetic inputs shared by the tests, the benchmark and the examples.

This module holds no arithmetic of the lattice Boltzmann method: it only builds
macroscopic fields (density, velocity) and random numbers on the host, in
float64, with the shapes and statistics of the workloads the library runs:

* 3D Taylor-Green vortex on an n^3 periodic box;
* body-force-driven channel between two walls (at rest, or a laminar profile
  plus a seeded divergence-free perturbation);
* crossing shear waves;
* seeded random positive arrays for perturbing states.

Arrays use the library's layout: scalar fields [nz, ny, nx], vector fields
[3, nz, ny, nx], population arrays [27, nz, ny, nx] (x fastest).
"""
from __future__ import annotations

import numpy as np


def taylor_green(n: int, u0: float = 0.05, rho0: float = 1.0, cell_centred: bool = True,
                 ny: int | None = None, nz: int | None = None):
    """Taylor-Green vortex: u = u0 sin x cos y cos z, v = -u0 cos x sin y cos z, w = 0,
    with the matching pressure p' = rho0 u0^2/16 (cos 2x + cos 2y)(cos 2z + 2),
    stored as a density perturbation rho' = 3 p' (isothermal, c_s^2 = 1/3).

    Coordinates are 2 pi (i + 1/2)/n (cell centred) or 2 pi i/n.
    """
    ny = n if ny is None else ny
    nz = n if nz is None else nz
    off = 0.5 if cell_centred else 0.0
    # separable factors, broadcast over the grid (the same products, in the same
    # order, as on a full coordinate mesh)
    x = (2 * np.pi * (np.arange(n) + off) / n)[None, None, :]
    y = (2 * np.pi * (np.arange(ny) + off) / ny)[None, :, None]
    z = (2 * np.pi * (np.arange(nz) + off) / nz)[:, None, None]
    u = np.zeros((3, nz, ny, n))
    u[0] = u0 * np.sin(x) * np.cos(y) * np.cos(z)
    u[1] = -u0 * np.cos(x) * np.sin(y) * np.cos(z)
    p = rho0 * u0 * u0 / 16.0 * (np.cos(2 * x) + np.cos(2 * y)) * (np.cos(2 * z) + 2.0)
    rho = rho0 + 3.0 * p
    return rho, u


def shear_wave(nx: int, ny: int, nz: int, amp: float, kx_modes: int = 1, kz_modes: int = 0):
    """u_y = amp cos(k_x x) cos(k_z z) (k = 2 pi modes / L), u_x = u_z = 0, rho = 1."""
    x = 2 * np.pi * kx_modes * np.arange(nx) / nx
    z = 2 * np.pi * kz_modes * np.arange(nz) / nz
    Z, Y, X = np.meshgrid(z, np.arange(ny), x, indexing="ij")
    u = np.zeros((3, nz, ny, nx))
    u[1] = amp * np.cos(X) * np.cos(Z)
    return np.ones((nz, ny, nx)), u


def channel_at_rest(nx: int, ny: int, nz: int, rho0: float = 1.0):
    return np.full((nz, ny, nx), rho0), np.zeros((3, nz, ny, nx))


def channel_turbulent_start(nx: int, ny: int, nz: int, u_bulk: float, amp: float = 0.1,
                            seed: int = 1234, kmax: int = 4):
    """Laminar parabola with bulk velocity u_bulk between walls half a link outside
    y = 0 and y = ny-1, plus a seeded divergence-free perturbation u' = curl(psi).

    psi is a sum of random Fourier modes (|k_x|, |k_z| <= kmax) in the periodic
    x and z directions times the wall envelope (1 - eta^2)^2, eta in (-1, 1),
    so u' vanishes at the walls; u' is scaled to rms = amp * u_bulk.  The
    discrete curl uses centred differences (periodic in x, z; one-sided at the
    walls), so it is divergence-free to truncation error only.
    """
    rng = np.random.default_rng(seed)
    H = float(ny)
    yc = np.arange(ny) + 0.5
    prof = 6.0 * u_bulk * yc * (H - yc) / (H * H)  # mean of 6 y(H-y)/H^2 over [0,H] is 1
    eta = 2.0 * yc / H - 1.0
    env = (1.0 - eta * eta) ** 2
    xs = 2 * np.pi * np.arange(nx) / nx
    zs = 2 * np.pi * np.arange(nz) / nz
    Z, Yv, X = np.meshgrid(zs, np.arange(ny), xs, indexing="ij")
    E = env[None, :, None] * np.ones((nz, ny, nx))
    psi = np.zeros((3, nz, ny, nx))
    for c in range(3):
        for kx in range(-kmax, kmax + 1):
            for kz in range(-kmax, kmax + 1):
                if kx == 0 and kz == 0:
                    continue
                a, ph = rng.standard_normal(), rng.uniform(0, 2 * np.pi)
                psi[c] += a * np.cos(kx * X + kz * Z + ph)
        psi[c] *= E

    def d(f, axis):
        if axis == 1:  # y: not periodic
            return np.gradient(f, axis=1)
        return (np.roll(f, -1, axis=axis) - np.roll(f, 1, axis=axis)) * 0.5

    # axes of [nz, ny, nx]: x -> 2, y -> 1, z -> 0
    up = np.zeros((3, nz, ny, nx))
    up[0] = d(psi[2], 1) - d(psi[1], 0)
    up[1] = d(psi[0], 0) - d(psi[2], 2)
    up[2] = d(psi[1], 2) - d(psi[0], 1)
    rms = np.sqrt((up ** 2).sum(0).mean() / 3.0)
    up *= amp * u_bulk / max(rms, 1e-300)
    u = up
    u[0] += prof[None, :, None]
    return np.ones((nz, ny, nx)), u


def random_factors(shape, seed: int, amplitude: float) -> np.ndarray:
    """1 + amplitude * U(-1, 1), seeded; used to perturb population arrays."""
    rng = np.random.default_rng(seed)
    return 1.0 + amplitude * rng.uniform(-1.0, 1.0, size=shape)


def random_fields(nx: int, ny: int, nz: int, seed: int, u_amp: float = 0.05, rho_amp: float = 0.02):
    """Random density and velocity fields (uniform noise), seeded."""
    rng = np.random.default_rng(seed)
    rho = 1.0 + rho_amp * rng.uniform(-1, 1, size=(nz, ny, nx))
    u = u_amp * rng.uniform(-1, 1, size=(3, nz, ny, nx))
    return rho, u
