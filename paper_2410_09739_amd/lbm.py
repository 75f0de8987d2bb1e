"""Thin ctypes binding of the C ABI in ``include/lbm.h`` (``liblbm.so``).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  The shared library is built in-tree (``__graft_entry__.build()`` or
``python -m paper_2410_09739_amd.build``); importing this module fails loudly if
it is missing.  The functions keep the C names (``lbm_create``, ``lbm_init``,
``lbm_step``, ...); ``Lattice`` wraps one context for convenience.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EHIP, LBM_EUNSTABLE, LBM_ESTATE = 0, -1, -2, -3, -4, -5
LBM_F64, LBM_F32, LBM_F16DEV, LBM_BF16DEV, LBM_F16DEV_RNE, LBM_BF16DEV_RNE = 0, 1, 2, 3, 4, 5
LBM_OMEGA_PAPER, LBM_OMEGA_ORDER_SCALED, LBM_OMEGA_EXPLICIT = 0, 1, 2
LBM_ATTRACTOR_FPC, LBM_ATTRACTOR_MAXWELL = 0, 1
Q = 27
CLOSURE_NPARAM = 6342

STORAGE = {"f64": LBM_F64, "f32": LBM_F32, "f16dev": LBM_F16DEV, "bf16dev": LBM_BF16DEV,
           "f16dev_rne": LBM_F16DEV_RNE, "bf16dev_rne": LBM_BF16DEV_RNE}
STORAGE_BYTES = {LBM_F64: 8, LBM_F32: 4, LBM_F16DEV: 2, LBM_BF16DEV: 2, LBM_F16DEV_RNE: 2, LBM_BF16DEV_RNE: 2}
OMEGA_MODE = {"paper": LBM_OMEGA_PAPER, "order_scaled": LBM_OMEGA_ORDER_SCALED, "explicit": LBM_OMEGA_EXPLICIT}
ATTRACTOR = {"fpc": LBM_ATTRACTOR_FPC, "maxwell": LBM_ATTRACTOR_MAXWELL}


class lbm_config(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("storage", ctypes.c_int32), ("walls_y", ctypes.c_int32), ("omega_mode", ctypes.c_int32),
        ("nu", ctypes.c_double), ("omega_bulk", ctypes.c_double), ("omega_higher", ctypes.c_double),
        ("omega", ctypes.c_double * Q), ("force", ctypes.c_double * 3),
        ("hip_stream", ctypes.c_void_p), ("attractor", ctypes.c_int32),
        ("walls_x", ctypes.c_int32), ("walls_z", ctypes.c_int32), ("lid_velocity", ctypes.c_double * 3),
        ("sym_top", ctypes.c_int32), ("les_cs", ctypes.c_double), ("les_wall_units", ctypes.c_double),
        ("les_aplus", ctypes.c_double),
    ]


class lbm_diag(ctypes.Structure):
    _fields_ = [
        ("mass", ctypes.c_double), ("momentum", ctypes.c_double * 3), ("kinetic_energy", ctypes.c_double),
        ("enstrophy", ctypes.c_double), ("wall_force", ctypes.c_double * 3), ("max_speed", ctypes.c_double),
        ("min_rho", ctypes.c_double), ("n_nonfinite", ctypes.c_int64), ("step", ctypes.c_int64),
    ]

    def as_dict(self) -> dict:
        return {
            "mass": self.mass, "momentum": list(self.momentum), "kinetic_energy": self.kinetic_energy,
            "enstrophy": self.enstrophy, "wall_force": list(self.wall_force), "max_speed": self.max_speed,
            "min_rho": self.min_rho, "n_nonfinite": int(self.n_nonfinite), "step": int(self.step),
        }


_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)
_vp = ctypes.c_void_p
_ctx = ctypes.c_void_p
_mlp = ctypes.c_void_p

# name -> (restype, argtypes); the exported C ABI
SIGNATURES = {
    "lbm_config_default": (None, [ctypes.POINTER(lbm_config)]),
    "lbm_omega_table": (ctypes.c_int, [ctypes.POINTER(lbm_config), _dp]),
    "lbm_create": (ctypes.c_int, [ctypes.POINTER(lbm_config), ctypes.POINTER(_ctx)]),
    "lbm_init": (ctypes.c_int, [_ctx, _dp, _dp]),
    "lbm_step": (ctypes.c_int, [_ctx, ctypes.c_int64]),
    "lbm_synchronize": (ctypes.c_int, [_ctx]),
    "lbm_moments": (ctypes.c_int, [_ctx, _dp, _dp]),
    "lbm_moments_device": (ctypes.c_int, [_ctx, _vp, _vp, ctypes.c_int32]),
    "lbm_diagnostics": (ctypes.c_int, [_ctx, ctypes.POINTER(lbm_diag)]),
    "lbm_get_f": (ctypes.c_int, [_ctx, _dp]),
    "lbm_set_f": (ctypes.c_int, [_ctx, _dp]),
    "lbm_get_f_nodes": (ctypes.c_int, [_ctx, ctypes.POINTER(ctypes.c_int64), ctypes.c_int64, _dp]),
    "lbm_get_f_nodes_noalloc": (ctypes.c_int, [_ctx, ctypes.POINTER(ctypes.c_int64), ctypes.c_int64, _dp]),
    "lbm_state_bytes": (ctypes.c_int64, [_ctx]),
    "lbm_get_raw": (ctypes.c_int, [_ctx, _vp, ctypes.c_int64]),
    "lbm_set_raw": (ctypes.c_int, [_ctx, _vp, ctypes.c_int64]),
    "lbm_stream": (_vp, [_ctx]),
    "lbm_step_count": (ctypes.c_int64, [_ctx]),
    "lbm_set_step_count": (ctypes.c_int, [_ctx, ctypes.c_int64]),
    "lbm_destroy": (None, [_ctx]),
    "lbm_last_error": (ctypes.c_char_p, [_ctx]),
    # learned closure
    "lbm_set_closure": (ctypes.c_int, [_ctx, _fp]),
    "lbm_closure_features": (ctypes.c_int, [_ctx, _vp]),
    "lbm_closure_eval": (ctypes.c_int, [_fp, _vp, _vp, ctypes.c_int64, _vp]),
    "lbm_coarsen": (ctypes.c_int, [_ctx, _vp, _vp, _vp, _vp]),
    "lbm_init_device": (ctypes.c_int, [_ctx, _vp, _vp]),
    "lbm_closure_targets": (ctypes.c_int, [_ctx, _vp, _vp, _vp, _vp, ctypes.c_double, _vp]),
    "lbm_mlp_create": (ctypes.c_int, [ctypes.c_uint64, _vp, ctypes.POINTER(_mlp)]),
    "lbm_mlp_set_params": (ctypes.c_int, [_mlp, _fp]),
    "lbm_mlp_get_params": (ctypes.c_int, [_mlp, _fp]),
    "lbm_mlp_set_normalisation": (ctypes.c_int, [_mlp, _fp, _fp, ctypes.c_float]),
    "lbm_mlp_get_normalisation": (ctypes.c_int, [_mlp, _fp, _fp, ctypes.POINTER(ctypes.c_float)]),
    "lbm_mlp_fit_normalisation": (ctypes.c_int, [_mlp, _vp, _vp, ctypes.c_int64]),
    "lbm_mlp_loss_grad": (ctypes.c_int, [_mlp, _vp, _vp, ctypes.c_int64, _dp, _fp]),
    "lbm_mlp_train": (ctypes.c_int, [_mlp, _vp, _vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_float, ctypes.c_uint64, _dp]),
    "lbm_mlp_export": (ctypes.c_int, [_mlp, _fp]),
    "lbm_mlp_destroy": (None, [_mlp]),
    "lbm_mlp_last_error": (ctypes.c_char_p, [_mlp]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load ``liblbm.so``; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"HIP library {path} is missing: build it with __graft_entry__.build() "
            "(hipcc --offload-arch=gfx950); there is no fallback path")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class LBMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


def _check(rc: int, ctx=None):
    if rc != LBM_OK:
        msg = load().lbm_last_error(ctx)
        raise LBMError(rc, msg.decode() if msg else "")


def _dptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


# ------------------------------------------------------------------ C names
def lbm_config_default() -> lbm_config:
    cfg = lbm_config()
    load().lbm_config_default(ctypes.byref(cfg))
    return cfg


def lbm_omega_table(cfg: lbm_config) -> np.ndarray:
    out = np.zeros(Q)
    _check(load().lbm_omega_table(ctypes.byref(cfg), _dptr(out)))
    return out


def lbm_create(cfg: lbm_config) -> int:
    h = _ctx()
    _check(load().lbm_create(ctypes.byref(cfg), ctypes.byref(h)))
    return h.value


def lbm_init(ctx, rho=None, u=None):
    _check(load().lbm_init(ctx, _dptr(rho), _dptr(u)), ctx)


def lbm_step(ctx, n: int):
    _check(load().lbm_step(ctx, int(n)), ctx)


def lbm_synchronize(ctx):
    _check(load().lbm_synchronize(ctx), ctx)


def lbm_moments(ctx, rho: np.ndarray, u: np.ndarray):
    _check(load().lbm_moments(ctx, _dptr(rho), _dptr(u)), ctx)


def lbm_moments_device(ctx, rho_ptr: int, u_ptr: int, f64: bool):
    _check(load().lbm_moments_device(ctx, rho_ptr, u_ptr, int(bool(f64))), ctx)


def lbm_diagnostics(ctx, check: bool = True) -> lbm_diag:
    d = lbm_diag()
    rc = load().lbm_diagnostics(ctx, ctypes.byref(d))
    if check or rc not in (LBM_OK, LBM_EUNSTABLE):
        _check(rc, ctx)
    return d


def lbm_get_f(ctx, f: np.ndarray):
    _check(load().lbm_get_f(ctx, _dptr(f)), ctx)


def lbm_get_f_nodes(ctx, nodes, f: np.ndarray):
    n = np.ascontiguousarray(nodes, dtype=np.int64)
    _check(load().lbm_get_f_nodes(ctx, n.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), int(n.size), _dptr(f)), ctx)


def lbm_get_f_nodes_noalloc(ctx, nodes, f: np.ndarray):
    n = np.ascontiguousarray(nodes, dtype=np.int64)
    _check(load().lbm_get_f_nodes_noalloc(ctx, n.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), int(n.size), _dptr(f)),
           ctx)


def lbm_set_f(ctx, f: np.ndarray):
    _check(load().lbm_set_f(ctx, _dptr(f)), ctx)


def lbm_state_bytes(ctx) -> int:
    return int(load().lbm_state_bytes(ctx))


def lbm_get_raw(ctx, buf: np.ndarray):
    _check(load().lbm_get_raw(ctx, buf.ctypes.data, buf.nbytes), ctx)


def lbm_set_raw(ctx, buf: np.ndarray):
    _check(load().lbm_set_raw(ctx, buf.ctypes.data, buf.nbytes), ctx)


def lbm_stream(ctx) -> int:
    return load().lbm_stream(ctx)


def lbm_step_count(ctx) -> int:
    return int(load().lbm_step_count(ctx))


def lbm_set_step_count(ctx, n: int):
    _check(load().lbm_set_step_count(ctx, int(n)), ctx)


def lbm_destroy(ctx):
    load().lbm_destroy(ctx)


def lbm_last_error(ctx=None) -> str:
    m = load().lbm_last_error(ctx)
    return m.decode() if m else ""


# ------------------------------------------------------------------ wrapper
@dataclass
class Config:
    nx: int
    ny: int
    nz: int
    storage: str = "f32"
    walls_y: bool = False
    nu: float = 1.0 / 6.0
    omega_bulk: float = 1.0
    omega_higher: float = 1.0
    omega_mode: str = "paper"
    omega: Optional[Sequence[float]] = None
    force: Sequence[float] = (0.0, 0.0, 0.0)
    hip_stream: Optional[int] = None
    attractor: str = "fpc"
    walls_x: bool = False
    walls_z: bool = False
    lid_velocity: Sequence[float] = (0.0, 0.0, 0.0)
    sym_top: bool = False
    les_cs: float = 0.0
    les_wall_units: float = 0.0
    les_aplus: float = 26.0

    def to_c(self) -> lbm_config:
        c = lbm_config_default()
        c.nx, c.ny, c.nz = int(self.nx), int(self.ny), int(self.nz)
        c.storage = STORAGE[self.storage]
        c.walls_y = int(bool(self.walls_y))
        c.omega_mode = OMEGA_MODE[self.omega_mode]
        c.nu = float(self.nu)
        c.omega_bulk = float(self.omega_bulk)
        c.omega_higher = float(self.omega_higher)
        if self.omega is not None:
            for j, w in enumerate(self.omega):
                c.omega[j] = float(w)
        for d in range(3):
            c.force[d] = float(self.force[d])
        c.hip_stream = self.hip_stream
        c.attractor = ATTRACTOR[self.attractor]
        c.walls_x = int(bool(self.walls_x))
        c.walls_z = int(bool(self.walls_z))
        for d in range(3):
            c.lid_velocity[d] = float(self.lid_velocity[d])
        c.sym_top = int(bool(self.sym_top))
        c.les_cs = float(self.les_cs)
        c.les_wall_units = float(self.les_wall_units)
        c.les_aplus = float(self.les_aplus)
        return c


class Lattice:
    """One library context (device state + stream)."""

    def __init__(self, cfg: Config):
        self.cfg = cfg
        self.n = cfg.nx * cfg.ny * cfg.nz
        self.shape = (cfg.nz, cfg.ny, cfg.nx)
        self._c = cfg.to_c()
        self.ctx = lbm_create(self._c)

    def close(self):
        if self.ctx:
            lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def omega(self) -> np.ndarray:
        return lbm_omega_table(self._c)

    def init(self, rho: Optional[np.ndarray] = None, u: Optional[np.ndarray] = None):
        r = None if rho is None else np.ascontiguousarray(rho, dtype=np.float64).reshape(self.n)
        v = None if u is None else np.ascontiguousarray(u, dtype=np.float64).reshape(3 * self.n)
        lbm_init(self.ctx, r, v)

    def step(self, n: int = 1):
        lbm_step(self.ctx, n)

    def synchronize(self):
        lbm_synchronize(self.ctx)

    def moments(self):
        rho = np.zeros(self.n)
        u = np.zeros(3 * self.n)
        lbm_moments(self.ctx, rho, u)
        return rho.reshape(self.shape), u.reshape((3,) + self.shape)

    def diagnostics(self, check: bool = True) -> dict:
        return lbm_diagnostics(self.ctx, check).as_dict()

    def get_f(self) -> np.ndarray:
        f = np.zeros(Q * self.n)
        lbm_get_f(self.ctx, f)
        return f.reshape((Q,) + self.shape)

    def get_f_nodes(self, nodes) -> np.ndarray:
        """Populations of the listed flat node indices, [27, len(nodes)]."""
        nodes = np.ascontiguousarray(nodes, dtype=np.int64)
        f = np.zeros(Q * max(nodes.size, 1))
        lbm_get_f_nodes(self.ctx, nodes, f)
        return f[: Q * nodes.size].reshape(Q, nodes.size)

    def set_f(self, f: np.ndarray):
        lbm_set_f(self.ctx, np.ascontiguousarray(f, dtype=np.float64).reshape(Q * self.n))

    def get_raw(self) -> np.ndarray:
        buf = np.zeros(lbm_state_bytes(self.ctx), dtype=np.uint8)
        lbm_get_raw(self.ctx, buf)
        return buf

    def set_raw(self, buf: np.ndarray):
        lbm_set_raw(self.ctx, np.ascontiguousarray(buf, dtype=np.uint8))

    @property
    def stream(self) -> int:
        return lbm_stream(self.ctx)

    @property
    def steps(self) -> int:
        return lbm_step_count(self.ctx)

    @steps.setter
    def steps(self, n: int):
        lbm_set_step_count(self.ctx, n)


# ------------------------------------------------------------------ closure
def _f32(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float32 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_fp)


def _check_mlp(rc: int, m=None):
    if rc != LBM_OK:
        msg = load().lbm_mlp_last_error(m)
        raise LBMError(rc, msg.decode() if msg else "")


def lbm_set_closure(ctx, params: Optional[np.ndarray]):
    p = None if params is None else np.ascontiguousarray(params, dtype=np.float32)
    if p is not None:
        assert p.shape == (CLOSURE_NPARAM,)
    _check(load().lbm_set_closure(ctx, _f32(p)), ctx)


def lbm_closure_features(ctx, x_ptr: int):
    _check(load().lbm_closure_features(ctx, x_ptr), ctx)


def lbm_closure_eval(params: np.ndarray, x_ptr: int, nu_ptr: int, n: int, stream: Optional[int] = None):
    p = np.ascontiguousarray(params, dtype=np.float32)
    assert p.shape == (CLOSURE_NPARAM,)
    _check_mlp(load().lbm_closure_eval(_f32(p), x_ptr, nu_ptr, int(n), stream))


def lbm_coarsen(ctx, rho_ptr: int, u_ptr: int, tau_ptr: int, sbar_ptr: Optional[int] = None):
    _check(load().lbm_coarsen(ctx, rho_ptr, u_ptr, tau_ptr, sbar_ptr), ctx)


def lbm_init_device(ctx, rho_ptr: int, u_ptr: int):
    _check(load().lbm_init_device(ctx, rho_ptr, u_ptr), ctx)


def lbm_closure_targets(ctx, rho_ptr: int, u_ptr: int, tau_ptr: int, sbar_ptr: int, eps_rel: float, y_ptr: int):
    _check(load().lbm_closure_targets(ctx, rho_ptr, u_ptr, tau_ptr, sbar_ptr, float(eps_rel), y_ptr), ctx)


class MLP:
    """The closure network's training state on the GPU (lbm_mlp)."""

    def __init__(self, seed: int = 0, stream: Optional[int] = None):
        h = _mlp()
        _check_mlp(load().lbm_mlp_create(int(seed), stream, ctypes.byref(h)))
        self.m = h.value

    def close(self):
        if self.m:
            load().lbm_mlp_destroy(self.m)
            self.m = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, p: np.ndarray):
        p = np.ascontiguousarray(p, dtype=np.float32)
        _check_mlp(load().lbm_mlp_set_params(self.m, _f32(p)), self.m)

    def get_params(self) -> np.ndarray:
        p = np.zeros(CLOSURE_NPARAM, dtype=np.float32)
        _check_mlp(load().lbm_mlp_get_params(self.m, _f32(p)), self.m)
        return p

    def set_normalisation(self, mu, sigma, s_y: float):
        mu = np.ascontiguousarray(mu, dtype=np.float32)
        sg = np.ascontiguousarray(sigma, dtype=np.float32)
        _check_mlp(load().lbm_mlp_set_normalisation(self.m, _f32(mu), _f32(sg), float(s_y)), self.m)

    def get_normalisation(self):
        mu = np.zeros(27, dtype=np.float32)
        sg = np.zeros(27, dtype=np.float32)
        sy = ctypes.c_float()
        _check_mlp(load().lbm_mlp_get_normalisation(self.m, _f32(mu), _f32(sg), ctypes.byref(sy)), self.m)
        return mu, sg, sy.value

    def fit_normalisation(self, x_ptr: int, y_ptr: int, n: int):
        _check_mlp(load().lbm_mlp_fit_normalisation(self.m, x_ptr, y_ptr, int(n)), self.m)

    def loss_grad(self, x_ptr: int, y_ptr: int, n: int):
        loss = ctypes.c_double()
        g = np.zeros(CLOSURE_NPARAM, dtype=np.float32)
        _check_mlp(load().lbm_mlp_loss_grad(self.m, x_ptr, y_ptr, int(n), ctypes.byref(loss), _f32(g)), self.m)
        return loss.value, g

    def train(self, x_ptr: int, y_ptr: int, n: int, batch: int, steps: int, lr: float, seed: int = 0) -> np.ndarray:
        hist = np.zeros(max(int(steps), 1))
        _check_mlp(load().lbm_mlp_train(self.m, x_ptr, y_ptr, int(n), int(batch), int(steps), float(lr), int(seed),
                                        _dptr(hist)), self.m)
        return hist[:steps]

    def export(self) -> np.ndarray:
        p = np.zeros(CLOSURE_NPARAM, dtype=np.float32)
        _check_mlp(load().lbm_mlp_export(self.m, _f32(p)), self.m)
        return p
