"""Start-up of the body-force channel 256 x 128 x 128 (walls half a link outside
y = 0 and y = 127, periodic x and z, nu = 0.01, F_x = 8 nu u_max / H^2 with
u_max = 0.05) from rest, in every storage form: the x-z averaged profile u_x(y)
against the analytic start-up series at several times, and against the FP64 run.

    python -m paper_2410_09739_amd.experiments.poiseuille [--steps 20000]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def analytic(ny: int, nu: float, F: float, t: float, nterms: int = 400) -> np.ndarray:
    H = float(ny)
    y = np.arange(ny) + 0.5
    u = F / (2 * nu) * y * (H - y)
    for n in range(1, 2 * nterms, 2):
        u -= 4 * F * H * H / (nu * n ** 3 * np.pi ** 3) * np.sin(n * np.pi * y / H) * np.exp(-n * n * np.pi ** 2 * nu * t / (H * H))
    return u


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--forms", default="f64,f32,f16dev,bf16dev,f16dev_rne,bf16dev_rne")
    ap.add_argument("--shape", default="256,128,128")
    args = ap.parse_args()
    from paper_2410_09739_amd import lbm as L

    nx, ny, nz = map(int, args.shape.split(","))
    nu, umax = 0.01, 0.05
    F = 8 * nu * umax / ny ** 2
    marks = sorted({m for m in (1000, 2000, 5000, 10000, 20000, args.steps) if m <= args.steps})
    out = {"workload": f"channel {nx}x{ny}x{nz}, nu={nu}, F={F:.6e}, from rest", "steps": args.steps, "forms": {}}
    prof = {}
    for st in args.forms.split(","):
        t0 = time.time()
        rec = {}
        with L.Lattice(L.Config(nx, ny, nz, storage=st, walls_y=True, nu=nu, force=(F, 0, 0))) as lat:
            lat.init()
            done = 0
            for m in marks:
                lat.step(m - done)
                done = m
                _, u = lat.moments()
                p = u[0].mean(axis=(0, 2))
                ua = analytic(ny, nu, F, m - 0.5)
                rec[m] = {"rel_l2_vs_analytic": float(np.sqrt(np.sum((p - ua) ** 2) / np.sum(ua ** 2))),
                          "centre_u": float(p[ny // 2]), "centre_u_analytic": float(ua[ny // 2]), "profile": p}
                print(f"# {st} t={m}: rel L2 {rec[m]['rel_l2_vs_analytic']:.3e}", file=sys.stderr, flush=True)
            d = lat.diagnostics()
        prof[st] = rec
        out["forms"][st] = {str(m): {k: v for k, v in r.items() if k != "profile"} for m, r in rec.items()}
        out["forms"][st]["mass_drift"] = d["mass"] / (nx * ny * nz) - 1.0
        out["forms"][st]["wall_s"] = time.time() - t0
    if "f64" in prof:
        for st in prof:
            for m in marks:
                out["forms"][st][str(m)]["max_abs_vs_f64_over_umax"] = float(
                    np.abs(prof[st][m]["profile"] - prof["f64"][m]["profile"]).max() / umax)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
