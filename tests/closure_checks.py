"""Acceptance checks shared by the closure's GPU parity tests, for results that
may differ from the oracle's bf16-quantised network by a bf16 rounding taken
the other way (a value on a rounding boundary, known only to FP32 accuracy).
They are checked against planted cases on the CPU (test_closure_oracle_pins)."""
import numpy as np

from oracle import closure_oracle as C


def bf16_alternatives(X, xtol, max_flips=4):
    """Nodes with features within xtol of a bf16 rounding boundary, and for each
    the feature vectors with every combination of those features rounded to the
    other side (at most 2^max_flips per node)."""
    q = C.round_bf16(X)
    lo, hi = C.round_bf16(X - xtol), C.round_bf16(X + xtol)
    out = {}
    for i in np.flatnonzero(np.any((lo != q) | (hi != q), axis=1)):
        cols = np.flatnonzero((lo[i] != q[i]) | (hi[i] != q[i]))[:max_flips]
        cands = []
        for m in range(1, 1 << len(cols)):
            x = q[i].copy()
            for b, k in enumerate(cols):
                if m >> b & 1:
                    x[k] = lo[i, k] if lo[i, k] != q[i, k] else hi[i, k]
            cands.append(x)
        out[int(i)] = cands
    return out


def explained_by_one_hidden_flip(p, x, got, tol):
    """True if some network that differs from the oracle's bf16 forward only in
    one hidden activation rounded to its other bf16 neighbour gives got (within
    tol).  A unit is a candidate when its pre-activation, known to FP32
    accumulation accuracy, may lie on either side of a bf16 rounding boundary."""
    W1, b1, W2, b2, W3, b3 = C.unpack(p)
    W1q, W2q, W3q = C.round_bf16(W1), C.round_bf16(W2), C.round_bf16(W3)
    b1f, b2f, b3f = (b.astype(np.float32).astype(np.float64) for b in (b1, b2, b3))
    xq = C.round_bf16(x)

    def other(z, mag):
        d = 64 * 2.0 ** -24 * mag  # FP32 accumulation of up to 64 products
        r = lambda v: C.round_bf16(np.maximum(v, 0.0))  # noqa: E731  (ReLU, then bf16)
        lo, hi, q = r(z - d), r(z + d), r(z)
        return np.where(lo != q, lo, np.where(hi != q, hi, np.nan))

    def layer2_on(h1):
        z2 = h1 @ W2q.T + b2f
        return z2, C.round_bf16(np.maximum(z2, 0.0)), np.abs(h1) @ np.abs(W2q).T + np.abs(b2f)

    z1 = xq @ W1q.T + b1f
    h1 = C.round_bf16(np.maximum(z1, 0.0))
    z2, h2, m2 = layer2_on(h1)
    alt1 = other(z1, np.abs(xq) @ np.abs(W1q).T + np.abs(b1f))
    alt2 = other(z2, m2)
    for k in np.flatnonzero(~np.isnan(alt2)):
        h = h2.copy()
        h[k] = alt2[k]
        if np.all(np.abs(h @ W3q.T + b3f - got) <= tol):
            return True
    for k in np.flatnonzero(~np.isnan(alt1)):
        h = h1.copy()
        h[k] = alt1[k]
        _, hh2, _ = layer2_on(h)
        if np.all(np.abs(hh2 @ W3q.T + b3f - got) <= tol):
            return True
    return False
