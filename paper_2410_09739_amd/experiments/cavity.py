"""Lid-driven cubic cavity (Sec. 4): walls on every face, halfway bounce-back,
the lid above y = L - 1 moving along x with U = Ma c_s.

``profiles``: Re = 100, 400, 1000 at L = 150 (and a coarser L for a grid
comparison), Ma = 0.1, run to a steady state; prints the centreline profiles
u_x(y) at x = z = L/2 and u_y(x) at y = z = L/2 (divided by U), the residual
change of the last interval, and the difference between the two grids.

``stability``: at Ma = 0.2 and L = 48, 64, 80, 96, the largest Reynolds number
(bisection on a geometric grid) for which the run stays finite with rho > 0
for a fixed number of lid-travel times, with the FPC attractors and with the
Maxwellian attractors (the MCM-LBM of the paper's comparison).

    python -m paper_2410_09739_amd.experiments.cavity profiles [--sizes 150,100] [--res 100,400,1000]
    python -m paper_2410_09739_amd.experiments.cavity stability [--sizes 48,64,80,96]
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

CS = 1.0 / math.sqrt(3.0)


def log(msg: str) -> None:
    print(f"# {msg}", file=sys.stderr, flush=True)


def cavity_config(L, n, Re, U, storage, attractor="fpc"):
    return L.Config(n, n, n, storage=storage, nu=U * n / Re, walls_x=True, walls_y=True, walls_z=True,
                    lid_velocity=(U, 0.0, 0.0), attractor=attractor)


def centrelines(u, n, U):
    c = n // 2
    if n % 2:
        ux = u[0][c, :, c]
        uy = u[1][c, c, :]
    else:  # average the two central planes of an even grid
        ux = 0.25 * (u[0][c - 1, :, c - 1] + u[0][c, :, c - 1] + u[0][c - 1, :, c] + u[0][c, :, c])
        uy = 0.25 * (u[1][c - 1, c - 1, :] + u[1][c, c - 1, :] + u[1][c - 1, c, :] + u[1][c, c, :])
    return ux / U, uy / U


def profiles(args):
    from paper_2410_09739_amd import lbm as L
    U = args.ma * CS
    out = {"workload": f"lid-driven cubic cavity, Ma={args.ma}, {args.storage}", "cases": {}}
    for Re in map(float, args.res.split(",")):
        curves = {}
        for n in map(int, args.sizes.split(",")):
            T = n / U  # lid-travel time in steps
            total = int(args.travel * T)
            chunk = max(1, int(T))
            t0 = time.time()
            with L.Lattice(cavity_config(L, n, Re, U, args.storage)) as lat:
                lat.init()
                done, prev, change = 0, None, None
                while done < total:
                    k = min(chunk, total - done)
                    lat.step(k)
                    done += k
                    ux, uy = centrelines(lat.moments()[1], n, U)
                    if prev is not None:
                        change = float(max(np.abs(ux - prev[0]).max(), np.abs(uy - prev[1]).max()))
                    prev = (ux, uy)
                    d = lat.diagnostics()
                    log(f"Re {Re:g} L {n} step {done}: change/U over one lid time {change}, "
                        f"max|u|/U {d['max_speed'] / U:.4f}")
            s = np.linspace(0.5 / n, 1 - 0.5 / n, n)  # cell-centre coordinate / L
            curves[n] = (s, prev[0], prev[1])
            out["cases"][f"Re{Re:g}_L{n}"] = {
                "steps": total, "wall_s": time.time() - t0, "last_change_over_U": change,
                "min_ux_over_U": float(prev[0].min()), "y_at_min_ux": float(s[int(np.argmin(prev[0]))]),
                "max_uy_over_U": float(prev[1].max()), "min_uy_over_U": float(prev[1].min()),
                "ux_centreline": [round(float(v), 5) for v in prev[0]],
                "uy_centreline": [round(float(v), 5) for v in prev[1]],
            }
        ns = sorted(curves)
        if len(ns) > 1:  # compare on the coarse grid's points
            sc, uxc, uyc = curves[ns[0]]
            sf, uxf, uyf = curves[ns[-1]]
            dx = np.abs(np.interp(sc, sf, uxf) - uxc).max()
            dy = np.abs(np.interp(sc, sf, uyf) - uyc).max()
            out["cases"][f"Re{Re:g}_grid_difference"] = {"coarse": ns[0], "fine": ns[-1],
                                                         "max_abs_ux_over_U": float(dx), "max_abs_uy_over_U": float(dy)}
            log(f"Re {Re:g}: L {ns[0]} vs {ns[-1]} centreline difference ux {dx:.4f} uy {dy:.4f} (/U)")
    print(json.dumps(out), flush=True)


def stable(L, n, Re, U, attractor, travel, storage):
    T = n / U
    total = int(travel * T)
    chunk = max(1, int(T))
    with L.Lattice(cavity_config(L, n, Re, U, storage, attractor)) as lat:
        lat.init()
        done = 0
        while done < total:
            k = min(chunk, total - done)
            lat.step(k)
            done += k
            d = lat.diagnostics(check=False)
            if d["n_nonfinite"] > 0 or not (d["min_rho"] > 0.0) or d["max_speed"] > 1.0:
                return False, done
    return True, total


def stability(args):
    from paper_2410_09739_amd import lbm as L
    U = args.ma * CS
    out = {"workload": f"lid-driven cubic cavity stability, Ma={args.ma}, {args.travel} lid-travel times, "
                       f"{args.storage}", "max_stable_re": {}}
    grid = [args.re_min * args.factor ** k for k in range(args.levels)]
    for att in args.attractors.split(","):
        for n in map(int, args.sizes.split(",")):
            lo, hi = -1, len(grid)  # grid[lo] stable, grid[hi] unstable
            ok0, _ = stable(L, n, grid[0], U, att, args.travel, args.storage)
            if not ok0:
                out["max_stable_re"][f"{att}_L{n}"] = None
                log(f"{att} L {n}: unstable already at Re {grid[0]:g}")
                continue
            lo = 0
            while hi - lo > 1:
                mid = (lo + hi) // 2
                ok, when = stable(L, n, grid[mid], U, att, args.travel, args.storage)
                log(f"{att} L {n} Re {grid[mid]:.0f}: {'stable' if ok else f'blew up by step {when}'}")
                if ok:
                    lo = mid
                else:
                    hi = mid
            out["max_stable_re"][f"{att}_L{n}"] = {"stable": grid[lo],
                                                  "unstable": grid[hi] if hi < len(grid) else None}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="mode", required=True)
    p = sub.add_parser("profiles")
    p.add_argument("--sizes", default="100,150")
    p.add_argument("--res", default="100,400,1000")
    p.add_argument("--ma", type=float, default=0.1)
    p.add_argument("--travel", type=float, default=40.0)
    p.add_argument("--storage", default="f32")
    s = sub.add_parser("stability")
    s.add_argument("--sizes", default="48,64,80,96")
    s.add_argument("--attractors", default="fpc,maxwell")
    s.add_argument("--ma", type=float, default=0.2)
    s.add_argument("--travel", type=float, default=20.0)
    s.add_argument("--re-min", type=float, default=500.0)
    s.add_argument("--factor", type=float, default=1.25)
    s.add_argument("--levels", type=int, default=30)
    s.add_argument("--storage", default="f64")
    a = ap.parse_args()
    profiles(a) if a.mode == "profiles" else stability(a)


if __name__ == "__main__":
    main()
