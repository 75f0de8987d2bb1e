"""FP64 CPU oracle of the learned second-order closure -- TEST INFRASTRUCTURE.

Only tests/, the smoke check and the benchmark's cpu_baseline leg may import
this module; it never imports the product path.  The paper has no learned
closure: every function here states the reading the library implements, in
plain numpy, one definition at a time.

Network (per node): x in R^27 -> h1 = relu(W1 x + b1) (64) -> h2 = relu(W2 h1 + b2)
(64) -> o = W3 h2 + b3 (6).  Parameters are one flat vector in the order
W1[64][27], b1[64], W2[64][64], b2[64], W3[6][64], b3[6] (6342 values).

Features (27): from the pre-collision central moments kappa_abc (Appendix D
Step 2) and rho: x_000 = rho - 1; x_100 = x_010 = x_001 = 0 (about the velocity
of Step 7, which carries F/2, the first-order central moments are -F/2 whatever
the node's state: they hold no information, and computed in FP32 from 27
populations they are pure rounding noise that standardisation would blow up);
otherwise (kappa_abc - rho E_abc) / rho with E_abc = C1[a] C1[b] C1[c],
C1 = (1, 0, c_s^2), times 3^{(a+b+c)/2} (= 1/c_s^order), in the paper's moment
order.  For training the inputs are standardised,
(x - mu) / sigma, and the outputs scaled, o = nu_t / s_y; both are folded into
W1, b1, W3, b3 for inference.

Outputs (6): eddy viscosities nu_t,j for the second-order groups
j = 110, 101, 011, 2s1, 2d1, 2d2 (relaxed with omega_4, omega_5, omega_6,
omega_7, omega_8, omega_9), applied as 1/omega_j,eff = 1/omega_j + 3 max(nu_t,j, 0)
through Eq. (transportcoeff3DFPCLBM) (nu = c_s^2 (1/omega - 1/2)).

Targets: from a fine run box-filtered 2x2x2 (Favre: u~ = avg(rho u) / avg(rho)),
the sub-filter stress tau_ij = avg(rho u_i u_j) - avg(rho) u~_i u~_j, the coarse
strain S_ij of u~ (centred differences on the coarse grid, periodic x/z,
antisymmetric ghost across half-link walls in y) and the filtered fine strain
Sbar_ij = 2 avg(rho S^f_ij) / avg(rho) (S^f: the same stencil on the fine grid;
the factor 2 turns fine into coarse lattice units).  The coarse node should
carry, beyond the resolved flux rho~ u~ u~, the filtered fine flux
tau - 2 rho~ nu Sbar; with an eddy viscosity it carries -2 rho~ (nu + nu_t) S.
Matching the two per group in the least-squares sense gives
nu*_j = max(0, S_j (nu_j (Sbar_j - S_j) - tau_j / (2 rho~)) / (S_j^2 + eps^2))
for the off-diagonal groups 110, 101, 011 (xy, xz, yz), with nu_j = c_s^2
(1/omega_j - 1/2) the group's coarse viscosity and eps = eps_rel * rms(S), and
nu* = 0 for 2s1 (the trace goes to pressure) and for the normal-stress
differences 2d1, 2d2 (their sub-filter anisotropy is not a dissipation aligned
with the strain; an eddy viscosity fitted there damps the resolved turbulence).
"""
from __future__ import annotations

import numpy as np

NIN, NH, NOUT = 27, 64, 6
NPARAM = NH * NIN + NH + NH * NH + NH + NOUT * NH + NOUT  # 6342
ORDER = ["000", "100", "010", "001", "110", "101", "011", "200", "020", "002", "120", "102",
         "210", "012", "201", "021", "111", "220", "202", "022", "211", "121", "112", "122",
         "212", "221", "222"]
C1 = np.array([1.0, 0.0, 1.0 / 3.0])
MNP = np.array([[int(c) for c in k] for k in ORDER])
E_REST = C1[MNP].prod(1)
NORM = 3.0 ** (MNP.sum(1) / 2.0)


# ------------------------------------------------------------------ parameters
def unpack(p: np.ndarray):
    p = np.asarray(p, dtype=np.float64)
    assert p.shape == (NPARAM,)
    i = 0
    out = []
    for shape in [(NH, NIN), (NH,), (NH, NH), (NH,), (NOUT, NH), (NOUT,)]:
        n = int(np.prod(shape))
        out.append(p[i:i + n].reshape(shape))
        i += n
    return out  # W1, b1, W2, b2, W3, b3


def pack(W1, b1, W2, b2, W3, b3) -> np.ndarray:
    return np.concatenate([np.ravel(a) for a in (W1, b1, W2, b2, W3, b3)]).astype(np.float64)


def init_params(seed: int = 0) -> np.ndarray:
    """He-uniform initialisation (ReLU layers), zero biases."""
    rng = np.random.default_rng(seed)
    W1 = rng.uniform(-1, 1, (NH, NIN)) * np.sqrt(6.0 / NIN)
    W2 = rng.uniform(-1, 1, (NH, NH)) * np.sqrt(6.0 / NH)
    W3 = rng.uniform(-1, 1, (NOUT, NH)) * np.sqrt(6.0 / NH)
    return pack(W1, np.zeros(NH), W2, np.zeros(NH), W3, np.zeros(NOUT))


# ------------------------------------------------------------------ network
def forward(p, X):
    """X [B, 27] -> (O [B, 6], cache)."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    Z1 = X @ W1.T + b1
    H1 = np.maximum(Z1, 0.0)
    Z2 = H1 @ W2.T + b2
    H2 = np.maximum(Z2, 0.0)
    O = H2 @ W3.T + b3
    return O, (X, Z1, H1, Z2, H2)


def loss(p, X, Y) -> float:
    """Mean squared error over all B * 6 outputs."""
    O, _ = forward(p, X)
    return float(np.mean((O - np.asarray(Y, dtype=np.float64)) ** 2))


def loss_and_grad(p, X, Y):
    """Loss and its gradient with respect to the flat parameter vector (chain rule by hand)."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    O, (X, Z1, H1, Z2, H2) = forward(p, X)
    B = X.shape[0]
    dO = 2.0 * (O - Y) / (B * NOUT)
    dW3 = dO.T @ H2
    db3 = dO.sum(0)
    dH2 = dO @ W3
    dZ2 = dH2 * (Z2 > 0)
    dW2 = dZ2.T @ H1
    db2 = dZ2.sum(0)
    dH1 = dZ2 @ W2
    dZ1 = dH1 * (Z1 > 0)
    dW1 = dZ1.T @ X
    db1 = dZ1.sum(0)
    return float(np.mean((O - Y) ** 2)), pack(dW1, db1, dW2, db2, dW3, db3)


def adam_step(p, g, m, v, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam update (Kingma & Ba); t counts from 1.  Returns (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def fold_normalisation(p, mu, sigma, s_y) -> np.ndarray:
    """Parameters acting on raw features and returning raw nu_t: with x_std =
    (x - mu)/sigma (features with sigma == 0 are dropped) and nu_t = s_y o."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    inv = np.where(sigma > 0, 1.0 / np.where(sigma > 0, sigma, 1.0), 0.0)
    W1f = W1 * inv[None, :]
    b1f = b1 - W1f @ mu
    return pack(W1f, b1f, W2, b2, W3 * s_y, b3 * s_y)


# ------------------------------------------------------------------ features
def features(kappa: np.ndarray, rho: np.ndarray) -> np.ndarray:
    """kappa [27, ...] central moments (paper order), rho [...] -> x [..., 27]."""
    kappa = np.asarray(kappa, dtype=np.float64)
    rho = np.asarray(rho, dtype=np.float64)
    shape = (27,) + (1,) * rho.ndim
    x = (kappa - rho[None] * E_REST.reshape(shape)) / rho[None] * NORM.reshape(shape)
    x[0] = rho - 1.0
    x[1:4] = 0.0
    return np.moveaxis(x, 0, -1)


def central_moments(f: np.ndarray, u: np.ndarray, e: np.ndarray) -> np.ndarray:
    """kappa_abc = sum_alpha f_alpha (e - u)^(a,b,c); f [27, ...], u [3, ...]."""
    out = np.zeros((27,) + f.shape[1:])
    for k, (a, b, c) in enumerate(MNP):
        cx = (e[:, 0].reshape((27,) + (1,) * (f.ndim - 1)) - u[0][None]) ** a
        cy = (e[:, 1].reshape((27,) + (1,) * (f.ndim - 1)) - u[1][None]) ** b
        cz = (e[:, 2].reshape((27,) + (1,) * (f.ndim - 1)) - u[2][None]) ** c
        out[k] = np.sum(f * cx * cy * cz, axis=0)
    return out


# ------------------------------------------------------------------ box filter and targets
def box_filter(rho: np.ndarray, u: np.ndarray, factor: int = 2):
    """2x2x2 (factor^3) box filter of fine fields rho [nz,ny,nx], u [3,nz,ny,nx].
    Returns rho~ [nz/f, ny/f, nx/f], Favre u~ [3, ...], tau [6, ...] in the order
    xx, yy, zz, xy, xz, yz."""
    nz, ny, nx = rho.shape
    f = factor

    def avg(a):
        return a.reshape(nz // f, f, ny // f, f, nx // f, f).mean(axis=(1, 3, 5))

    rb = avg(rho)
    mom = np.stack([avg(rho * u[d]) for d in range(3)])
    ut = mom / rb[None]
    pairs = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
    tau = np.stack([avg(rho * u[i] * u[j]) - rb * ut[i] * ut[j] for i, j in pairs])
    return rb, ut, tau


def filtered_strain(rho: np.ndarray, u: np.ndarray, walls_y: bool, factor: int = 2) -> np.ndarray:
    """Favre box filter of the fine strain rate in coarse lattice units:
    Sbar = factor * avg(rho S^f) / avg(rho), S^f = strain(u, walls_y) on the fine
    grid; [6, nz/f, ny/f, nx/f] in the order xx, yy, zz, xy, xz, yz."""
    nz, ny, nx = rho.shape
    f = factor

    def avg(a):
        return a.reshape(nz // f, f, ny // f, f, nx // f, f).mean(axis=(1, 3, 5))

    Sf = strain(u, walls_y)
    rb = avg(rho)
    return np.stack([f * avg(rho * Sf[k]) / rb for k in range(6)])


def strain(u: np.ndarray, walls_y: bool) -> np.ndarray:
    """S_ij = (d_i u_j + d_j u_i)/2 by centred differences; order xx, yy, zz, xy, xz, yz.
    Periodic in x and z; in y periodic or an antisymmetric ghost across the walls."""
    def d(a, axis):
        if axis == 1 and walls_y:
            ap = np.concatenate([a[:, 1:], -a[:, -1:]], axis=1)
            am = np.concatenate([-a[:, :1], a[:, :-1]], axis=1)
            return 0.5 * (ap - am)
        return 0.5 * (np.roll(a, -1, axis=axis) - np.roll(a, 1, axis=axis))

    ax = {0: 2, 1: 1, 2: 0}  # velocity component direction -> array axis of [nz, ny, nx]
    g = [[d(u[j], ax[i]) for j in range(3)] for i in range(3)]  # g[i][j] = d_i u_j
    return np.stack([g[0][0], g[1][1], g[2][2], 0.5 * (g[0][1] + g[1][0]), 0.5 * (g[0][2] + g[2][0]),
                     0.5 * (g[1][2] + g[2][1])])


def group(a6: np.ndarray) -> np.ndarray:
    """xx,yy,zz,xy,xz,yz -> the six second-order groups 110, 101, 011, 2s1, 2d1, 2d2."""
    xx, yy, zz, xy, xz, yz = a6
    return np.stack([xy, xz, yz, xx + yy + zz, xx - yy, xx - zz])


def targets(rho_t: np.ndarray, tau: np.ndarray, S: np.ndarray, Sbar: np.ndarray, nu, eps_rel: float = 0.1,
            clip: bool = True) -> np.ndarray:
    """nu*_j per coarse node, [6, ...]; see the module docstring.  nu: the coarse
    viscosities of the groups 110, 101, 011 (three values, or one for all)."""
    nu3 = np.broadcast_to(np.asarray(nu, dtype=np.float64), (3,))
    tg, sg, sb = group(tau), group(S), group(Sbar)
    eps2 = eps_rel ** 2 * np.mean(S[:3] ** 2 + 2 * S[3:] ** 2)
    out = np.zeros_like(sg)
    for j in range(3):
        out[j] = sg[j] * (nu3[j] * (sb[j] - sg[j]) - tg[j] / (2.0 * rho_t)) / (sg[j] * sg[j] + eps2)
    return np.maximum(out, 0.0) if clip else out


# ------------------------------------------------------------------ reduced-precision inference
def round_bf16(x) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64.
    Values are first rounded to float32, as the GPU holds them."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    nan = (u & 0x7FFFFFFF) > 0x7F800000
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    r = np.where(nan, (u | 0x400000) & 0xFFFF0000, r).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def forward_bf16(p, X):
    """The network with inputs, weights, biases of layers 1-2 used as given, and
    the quantisation of the matrix-core path: inputs, weights and the ReLU'd
    hidden activations rounded to bfloat16; biases and sums in full precision."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    Xq = round_bf16(X)
    H1 = round_bf16(np.maximum(Xq @ round_bf16(W1).T + b1.astype(np.float32), 0.0))
    H2 = round_bf16(np.maximum(H1 @ round_bf16(W2).T + b2.astype(np.float32), 0.0))
    return H2 @ round_bf16(W3).T + b3.astype(np.float32)


# ------------------------------------------------------------------ minibatch sampling
_M64 = (1 << 64) - 1


def _mix64(z: int) -> int:
    """SplitMix64 output function (Steele, Lea & Flood 2014)."""
    z &= _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def sample_indices(seed: int, step: int, batch: int, n: int) -> np.ndarray:
    """Indices of minibatch `step` (0-based): slot j draws
    mix64(seed xor mix64(step * 0x9E3779B97F4A7C15 + j)) mod n."""
    return np.array([_mix64(seed ^ _mix64(step * 0x9E3779B97F4A7C15 + j)) % n for j in range(batch)],
                    dtype=np.int64)


def closure_rates(nu: np.ndarray, omega: np.ndarray) -> np.ndarray:
    """Per-node omega_4..omega_9 from the network outputs:
    1/omega_eff = 1/omega + 3 clamp(nu, 0, 1/3)."""
    nt = np.clip(np.nan_to_num(nu, nan=0.0), 0.0, 1.0 / 3.0)
    return 1.0 / (1.0 / np.asarray(omega)[4:10] + 3.0 * nt)
