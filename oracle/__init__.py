"""FP64 CPU oracle of the D3Q27 FPC-LBM (arXiv 2410.09739) -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and its
Python binding) never imports, links or runs anything here, and this package
never imports the product path.

The per-node arithmetic lives in ``fpc_oracle.c`` (plain C, FP64, explicit 27x27
matrices, Appendix D of the paper in its own order); this module only loads it
through ctypes and adds the host-side parameter mapping of the paper:

* shear viscosity -> second-order relaxation rates, Eq. (transportcoeff3DFPCLBM)
  with the Henon correction: nu = c_s^2 (1/omega - 1/2);
* bulk viscosity: zeta = (2/3) c_s^2 (1/omega_2s - 1/2), same equation;
* remaining rates: free parameters in (0, 2); the paper's runs set them to 1
  (Sec. 4, first subsection).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fpc_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

CS2 = 1.0 / 3.0
Q = 27

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_i64p = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = False) -> str:
    """Compile ``fpc_oracle.c`` into ``liboracle.so`` next to it (gcc, -O2, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.orc_collide_node.argtypes = [_dp, _dp, _dp, _dp, _dp, _dp, ctypes.c_int, ctypes.c_double]
        lib.orc_feq.argtypes = [ctypes.c_double, _dp, _dp]
        lib.orc_lattice.argtypes = [_ip, _ip, _ip, _ip, _ip]
        lib.orc_matrices.argtypes = [_dp, _dp, _dp, _dp, _dp]
        lib.orc_attractor.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, _dp]
        lib.orc_attractor.restype = ctypes.c_double
        lib.orc_init.argtypes = [ctypes.c_int] * 3 + [_dp, _dp, _dp]
        lib.orc_collide.argtypes = [ctypes.c_int] * 3 + [_dp, _dp, _dp, _dp, ctypes.c_int, ctypes.c_int, _dp]
        lib.orc_stream.argtypes = [ctypes.c_int] * 4 + [_dp, _dp, _dp]
        lib.orc_stream_push.argtypes = [ctypes.c_int] * 4 + [_dp, _dp, _dp]
        lib.orc_run.argtypes = [ctypes.c_int] * 4 + [_dp, _dp, _dp, _dp, ctypes.c_int, ctypes.c_int, _dp]
        lib.orc_run.restype = ctypes.c_int
        lib.orc_num_threads.restype = ctypes.c_int
        lib.orc_step_nodes.argtypes = [ctypes.c_int] * 4 + [_dp, _dp, _dp, _dp, _i64p, ctypes.c_int64, _dp, ctypes.c_int, _dp]
        _lib = lib
    return _lib


def _d(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


# ---------------------------------------------------------------- parameters
def omega_table(nu: float, omega_bulk: float = 1.0, omega_higher: float = 1.0,
                mode: str = "paper", explicit=None) -> np.ndarray:
    """The 27 relaxation rates omega_0..omega_26 in Appendix D numbering.

    omega_4..6 (110, 101, 011) and omega_8, omega_9 (2d1, 2d2) follow from the
    shear viscosity, Eq. (transportcoeff3DFPCLBM): 1/omega = nu/c_s^2 + 1/2.
    omega_7 (2s1) is the bulk rate.  ``paper``: all other rates equal
    ``omega_higher`` (1 in the paper's runs).  ``order_scaled``: the continuous
    scaling omega_mnp = (m+n+p) omega_FP carried through the Henon correction,
    1/omega_n - 1/2 = (2/n)(1/omega_2 - 1/2) for moments of order n >= 3.
    ``explicit``: the 27 given values.
    """
    if mode == "explicit":
        w = _f64(explicit).copy()
        assert w.shape == (Q,)
        return w
    w_nu = 1.0 / (nu / CS2 + 0.5)
    w = np.full(Q, float(omega_higher))
    w[0:4] = 1.0
    w[4:7] = w_nu
    w[7] = omega_bulk
    w[8:10] = w_nu
    if mode == "order_scaled":
        order = {10: 3, 11: 3, 12: 3, 13: 3, 14: 3, 15: 3, 16: 3,
                 17: 4, 18: 4, 19: 4, 20: 4, 21: 4, 22: 4,
                 23: 5, 24: 5, 25: 5, 26: 6}
        for j, n in order.items():
            w[j] = 1.0 / ((2.0 / n) * (1.0 / w_nu - 0.5) + 0.5)
    elif mode != "paper":
        raise ValueError(mode)
    return w


# ---------------------------------------------------------------- per node
def lattice():
    """(e [27,3], opp [27], mnp [27,3]) as the oracle builds them."""
    lib = _load()
    ex, ey, ez, opp = (np.zeros(Q, np.int32) for _ in range(4))
    mnp = np.zeros(Q * 3, np.int32)
    lib.orc_lattice(*(a.ctypes.data_as(_ip) for a in (ex, ey, ez, opp, mnp)))
    return np.stack([ex, ey, ez], 1), opp, mnp.reshape(Q, 3)


def matrices(u):
    """P, P^-1, F(u), F^-1(u) as 27x27 float64 arrays."""
    lib = _load()
    out = [np.zeros((Q, Q)) for _ in range(4)]
    lib.orc_matrices(_d(_f64(u)), *(_d(a) for a in out))
    return tuple(out)


def attractor(m: int, n: int, p: int, D, pi) -> float:
    """Eq. (Mvcmattractor3D) for moment (m,n,p); D = (D'200, D'020, D'002, D'110, D'011, D'101)."""
    return _load().orc_attractor(m, n, p, _d(_f64(D)), _d(_f64(pi)))


def _model(attractor: str) -> int:
    """0: FPC Markovian attractors; 1: Maxwellian attractors (the MCM comparison model)."""
    return {"fpc": 0, "maxwell": 1}[attractor]


def collide_node(f, omega, force=(0.0, 0.0, 0.0), return_moments: bool = False, attractor: str = "fpc",
                 les_cd: float = 0.0):
    """Appendix D Steps 1-5 at one node (27 populations in, 27 out).  les_cd:
    the Smagorinsky factor C D of reading R25 at this node (0: no LES)."""
    lib = _load()
    f = _f64(f)
    ft, kpre, kpost = np.zeros(Q), np.zeros(Q), np.zeros(Q)
    lib.orc_collide_node(_d(f), _d(_f64(omega)), _d(_f64(force)), _d(ft), _d(kpre), _d(kpost), _model(attractor),
                         float(les_cd))
    return (ft, kpre, kpost) if return_moments else ft


def feq(rho: float, u) -> np.ndarray:
    lib = _load()
    out = np.zeros(Q)
    lib.orc_feq(float(rho), _d(_f64(u)), _d(out))
    return out


# ---------------------------------------------------------------- lattice-wide
def init(rho: np.ndarray, u: np.ndarray) -> np.ndarray:
    """f^eq at every node.  rho: [nz,ny,nx]; u: [3,nz,ny,nx]; returns [27,nz,ny,nx]."""
    lib = _load()
    rho = _f64(rho)
    nz, ny, nx = rho.shape
    u = _f64(u)
    f = np.zeros((Q, nz, ny, nx))
    lib.orc_init(nx, ny, nz, _d(rho), _d(u), _d(f))
    return f


def _les(les):
    """les = (C_s, u_tau / nu, A+) of reading R25, or None."""
    return None if les is None else _f64(les)


def collide(f: np.ndarray, omega, force=(0.0, 0.0, 0.0), attractor: str = "fpc", walls_y: bool = False,
            walls=None, les=None) -> np.ndarray:
    lib = _load()
    f = _f64(f)
    _, nz, ny, nx = f.shape
    g = np.zeros_like(f)
    lib.orc_collide(nx, ny, nz, _d(f), _d(g), _d(_f64(omega)), _d(_f64(force)), _model(attractor),
                    _walls(walls_y, walls), _d(_les(les)))
    return g


def _walls(walls_y: bool, walls) -> int:
    """Wall mask (readings R23, R24): 1 = y faces, 2 = x faces, 4 = z faces,
    8 = the face above y = ny - 1 is a specular symmetry plane.  ``walls``
    overrides ``walls_y`` when given (a mask or a string: "x", "y", "z" walls,
    "s" symmetry plane on top, e.g. "ys" for the half channel)."""
    if walls is None:
        return 1 if walls_y else 0
    if isinstance(walls, str):
        return sum({"y": 1, "x": 2, "z": 4, "s": 8}[c] for c in walls)
    return int(walls)


def _lid(lid):
    return None if lid is None else _f64(lid)


def stream(g: np.ndarray, walls_y: bool = False, walls=None, lid=None) -> np.ndarray:
    lib = _load()
    g = _f64(g)
    _, nz, ny, nx = g.shape
    f = np.zeros_like(g)
    lib.orc_stream(nx, ny, nz, _walls(walls_y, walls), _d(_lid(lid)), _d(g), _d(f))
    return f


def stream_push(g: np.ndarray, walls_y: bool = False, walls=None, lid=None) -> np.ndarray:
    """Streaming in push form (cross-check of ``stream``)."""
    lib = _load()
    g = _f64(g)
    _, nz, ny, nx = g.shape
    f = np.zeros_like(g)
    lib.orc_stream_push(nx, ny, nz, _walls(walls_y, walls), _d(_lid(lid)), _d(g), _d(f))
    return f


def run(g: np.ndarray, omega, force=(0.0, 0.0, 0.0), walls_y: bool = False, steps: int = 1,
        attractor: str = "fpc", walls=None, lid=None, les=None) -> np.ndarray:
    """``steps`` full time steps (stream, then collide) from a post-collision state."""
    lib = _load()
    g = _f64(g).copy()
    _, nz, ny, nx = g.shape
    rc = lib.orc_run(nx, ny, nz, _walls(walls_y, walls), _d(_lid(lid)), _d(_f64(omega)), _d(_f64(force)), _d(g),
                     int(steps), _model(attractor), _d(_les(les)))
    if rc != 0:
        raise MemoryError("oracle run failed")
    return g


def step_nodes(g: np.ndarray, sel, omega, force=(0.0, 0.0, 0.0), walls_y: bool = False,
               attractor: str = "fpc", walls=None, lid=None, les=None) -> np.ndarray:
    """One step evaluated at the flat node indices ``sel`` only; returns [27, len(sel)]."""
    lib = _load()
    g = _f64(g)
    _, nz, ny, nx = g.shape
    sel = np.ascontiguousarray(np.asarray(sel, dtype=np.int64))
    out = np.zeros((Q, sel.size))
    lib.orc_step_nodes(nx, ny, nz, _walls(walls_y, walls), _d(_lid(lid)), _d(_f64(omega)), _d(_f64(force)), _d(g),
                       sel.ctypes.data_as(_i64p), sel.size, _d(out), _model(attractor), _d(_les(les)))
    return out


def num_threads() -> int:
    """OpenMP threads the oracle's lattice loops use."""
    return int(_load().orc_num_threads())


def macroscopic(state: np.ndarray, force=(0.0, 0.0, 0.0), post_collision: bool = True):
    """rho and u from a lattice state, Appendix D Step 7.

    For a pre-collision state rho u = sum f e + F/2.  The collision adds exactly F
    to sum f e, so from a post-collision state rho u = sum f~ e - F/2.
    """
    e, _, _ = lattice()
    f = _f64(state)
    rho = f.sum(0)
    j = np.einsum("a...,ad->d...", f, e.astype(np.float64))
    sgn = -0.5 if post_collision else 0.5
    for d in range(3):
        j[d] += sgn * force[d]
    return rho, j / rho


# ---------------------------------------------------------------- diagnostics
def _ghosted(u: np.ndarray, mask: int, lid) -> np.ndarray:
    """The velocity field [3, nz, ny, nx] with one ghost layer on every side.

    Periodic axes wrap.  Across a half-link wall at rest the ghost holds -u of
    the adjacent fluid node (u = 0 halfway between them); across the moving lid
    above y = ny - 1 it holds 2 U - u (u = U halfway); across the specular
    symmetry plane above y = ny - 1 the tangential components u_x, u_z mirror
    (ghost = u) and the normal one u_y changes sign.  Corners of the ghost layer
    are never read by the centred differences."""
    _, nz, ny, nx = u.shape
    g = np.zeros((3, nz + 2, ny + 2, nx + 2))
    g[:, 1:-1, 1:-1, 1:-1] = u
    # x faces
    if mask & 2:
        g[:, 1:-1, 1:-1, 0] = -u[:, :, :, 0]
        g[:, 1:-1, 1:-1, -1] = -u[:, :, :, -1]
    else:
        g[:, 1:-1, 1:-1, 0] = u[:, :, :, -1]
        g[:, 1:-1, 1:-1, -1] = u[:, :, :, 0]
    # z faces
    if mask & 4:
        g[:, 0, 1:-1, 1:-1] = -u[:, 0]
        g[:, -1, 1:-1, 1:-1] = -u[:, -1]
    else:
        g[:, 0, 1:-1, 1:-1] = u[:, -1]
        g[:, -1, 1:-1, 1:-1] = u[:, 0]
    # y faces
    if mask & 1:
        g[:, 1:-1, 0, 1:-1] = -u[:, :, 0, :]
        top = u[:, :, -1, :]
        if mask & 8:
            g[:, 1:-1, -1, 1:-1] = top * np.array([1.0, -1.0, 1.0])[:, None, None]
        elif lid is not None:
            g[:, 1:-1, -1, 1:-1] = 2.0 * np.asarray(lid, dtype=np.float64)[:, None, None] - top
        else:
            g[:, 1:-1, -1, 1:-1] = -top
    else:
        g[:, 1:-1, 0, 1:-1] = u[:, :, -1, :]
        g[:, 1:-1, -1, 1:-1] = u[:, :, 0, :]
    return g


def vorticity(u: np.ndarray, walls_y: bool = False, walls=None, lid=None) -> np.ndarray:
    """curl u [3, nz, ny, nx] by second-order centred differences,
    d_x q(i) = (q(i+1) - q(i-1)) / 2 (lattice units), with the ghost layers of
    ``_ghosted`` at walls, the lid and the symmetry plane."""
    g = _ghosted(_f64(u), _walls(walls_y, walls), lid)

    def d(c, axis):  # centred difference of component c along axis (0 x, 1 y, 2 z)
        if axis == 0:
            return 0.5 * (g[c, 1:-1, 1:-1, 2:] - g[c, 1:-1, 1:-1, :-2])
        if axis == 1:
            return 0.5 * (g[c, 1:-1, 2:, 1:-1] - g[c, 1:-1, :-2, 1:-1])
        return 0.5 * (g[c, 2:, 1:-1, 1:-1] - g[c, :-2, 1:-1, 1:-1])

    return np.stack([d(2, 1) - d(1, 2), d(0, 2) - d(2, 0), d(1, 0) - d(0, 1)])


def diagnostics(state: np.ndarray, force=(0.0, 0.0, 0.0), walls_y: bool = False, walls=None, lid=None) -> dict:
    """FP64 diagnostics of a post-collision lattice state, from their definitions:
    mass sum rho; momentum sum rho u (Appendix D Step 7, with the F/2 shift);
    kinetic energy 1/2 sum rho |u|^2; enstrophy 1/2 sum |curl u|^2 (``vorticity``);
    max |u|; min rho; nodes with a non-finite population; and the force of the
    fluid on the walls, sum over the bounce-back links of 2 f~_a e_a (a link
    leaves a fluid node towards a wall; the symmetry plane takes no force)."""
    f = _f64(state)
    mask = _walls(walls_y, walls)
    rho, u = macroscopic(f, force)
    e, _, _ = lattice()
    wall = np.zeros(3)
    _, nz, ny, nx = f.shape
    for a in range(Q):
        ex, ey, ez = (int(c) for c in e[a])
        sel = np.zeros((nz, ny, nx), dtype=bool)
        if mask & 1:
            if ey == -1:
                sel[:, 0, :] = True
            if ey == 1 and not mask & 8:
                sel[:, ny - 1, :] = True
        if mask & 2:
            if ex == -1:
                sel[:, :, 0] = True
            if ex == 1:
                sel[:, :, nx - 1] = True
        if mask & 4:
            if ez == -1:
                sel[0] = True
            if ez == 1:
                sel[nz - 1] = True
        wall += 2.0 * f[a][sel].sum() * e[a]
    w = vorticity(u, walls=mask, lid=lid)
    return {
        "mass": float(rho.sum()),
        "momentum": [float((rho * u[d]).sum()) for d in range(3)],
        "kinetic_energy": float(0.5 * (rho * (u ** 2).sum(0)).sum()),
        "enstrophy": float(0.5 * (w ** 2).sum()),
        "max_speed": float(np.sqrt((u ** 2).sum(0)).max()),
        "min_rho": float(rho.min()),
        "n_nonfinite": int((~np.isfinite(f)).any(0).sum()),
        "wall_force": wall.tolist(),
    }
