"""Orthogonal crossing shear waves (Sec. 4): u_y = U cos(k x) cos(k z) in a
periodic L x ny x L box, nu = 1e-7, U = 1e-5.  The exact solution decays as
exp(-2 nu k^2 t), k = 2 pi / L.  Runs the FPC attractors and the Maxwellian
attractors (MCM) side by side and reports the amplitude history, the decay
rate measured after the initial odd-even transient, and the apparent
viscosity rate / (2 k^2) of each, for several L.

    python -m paper_2410_09739_amd.experiments.crossing_shear_waves [--sizes 30,60,120] [--steps 100000]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", default="30,60,120")
    ap.add_argument("--ny", type=int, default=2)
    ap.add_argument("--steps", type=int, default=100000)
    ap.add_argument("--samples", type=int, default=40)
    ap.add_argument("--nu", type=float, default=1e-7)
    ap.add_argument("--amp", type=float, default=1e-5)
    ap.add_argument("--storage", default="f64")
    args = ap.parse_args()
    from paper_2410_09739_amd import lbm as L

    out = {"workload": f"crossing shear waves, nu={args.nu}, U={args.amp}, ny={args.ny}, {args.storage}",
           "steps": args.steps, "cases": {}}
    t_settle = 300
    for n in map(int, args.sizes.split(",")):
        k = 2 * np.pi / n
        Z, _, X = np.meshgrid(np.arange(n), np.arange(args.ny), np.arange(n), indexing="ij")
        mode = np.cos(k * X) * np.cos(k * Z)
        u = np.zeros((3, n, args.ny, n))
        u[1] = args.amp * mode
        rho = np.ones((n, args.ny, n))
        marks = sorted({t_settle, *np.linspace(t_settle, args.steps, args.samples).astype(int).tolist()})
        for att in ("fpc", "maxwell"):
            t0 = time.time()
            with L.Lattice(L.Config(n, args.ny, n, storage=args.storage, nu=args.nu, attractor=att)) as lat:
                lat.init(rho, u)
                done, amps = 0, []
                for m in marks:
                    lat.step(m - done)
                    done = m
                    uu = lat.moments()[1]
                    amps.append(float((uu[1] * mode).sum() / (mode * mode).sum() / args.amp))
            a = np.array(amps)
            t = np.array(marks, dtype=float)
            ok = a > 0
            rate = float(-np.polyfit(t[ok], np.log(a[ok]), 1)[0]) if ok.sum() > 2 else float("nan")
            exact = 2 * k * k * args.nu
            out["cases"][f"L{n}_{att}"] = {"L": n, "attractor": att, "t": marks, "amplitude": [round(v, 7) for v in amps],
                                            "decay_rate": rate, "exact_rate": exact,
                                            "apparent_nu": rate / (2 * k * k), "wall_s": time.time() - t0}
            print(f"# L={n} {att}: amplitude {amps[-1]:.5f} at t={marks[-1]}, rate {rate:.3e} "
                  f"(exact {exact:.3e}), apparent nu {rate / (2 * k * k):.3e}", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
