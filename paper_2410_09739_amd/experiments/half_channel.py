"""The paper's turbulent channel setup (Sec. 4): a half channel 2 pi H x H x pi H
(x streamwise, y wall-normal, z spanwise) with a wall half a link below y = 0,
a specular symmetry plane above y = H - 1, periodic x and z, driven by
F = rho u_tau^2 / H at Re_tau = u_tau H / nu = 180, with Smagorinsky LES and
van Driest damping.  Reports the mean velocity U+(y+), the rms fluctuations
and the Reynolds shear stress in wall units, averaged over x, z and time, and
the friction velocity measured at the wall.

    python -m paper_2410_09739_amd.experiments.half_channel [--h 100] [--tstar-transient 25] [--tstar-stats 15]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def log(msg: str) -> None:
    print(f"# {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--h", type=int, default=100)
    ap.add_argument("--re-tau", type=float, default=180.0)
    ap.add_argument("--u-tau", type=float, default=0.0075)
    ap.add_argument("--cs", type=float, default=0.1)
    ap.add_argument("--storage", default="f32")
    ap.add_argument("--tstar-transient", type=float, default=25.0)
    ap.add_argument("--tstar-stats", type=float, default=15.0)
    ap.add_argument("--samples-per-tstar", type=int, default=4)
    ap.add_argument("--perturbation", type=float, default=0.3)
    args = ap.parse_args()
    import torch

    from paper_2410_09739_amd import lbm as L
    from paper_2410_09739_amd import workloads as W
    from paper_2410_09739_amd.experiments.closure_channel import ProfileStats, device_moments

    H = args.h
    nx, ny, nz = int(round(2 * np.pi * H)), H, int(round(np.pi * H))
    ut = args.u_tau
    nu = ut * H / args.re_tau
    F = ut * ut / H
    tstar = int(round(H / ut))
    cfg = L.Config(nx, ny, nz, storage=args.storage, walls_y=True, sym_top=True, nu=nu, force=(F, 0, 0),
                   les_cs=args.cs, les_wall_units=ut / nu)
    out = {"workload": f"half channel {nx}x{ny}x{nz} (2 pi H x H x pi H, H={H}), Re_tau={args.re_tau}, "
                       f"u_tau={ut}, nu={nu:.6e}, F={F:.6e}, Smagorinsky C={args.cs} with van Driest A+=26, "
                       f"{args.storage}", "tstar_steps": tstar}
    # start: the lower half of a perturbed laminar full channel of height 2H
    log(f"building the initial field for {nx}x{ny}x{nz}")
    rho_f, u_f = W.channel_turbulent_start(nx, 2 * ny, nz, u_bulk=15.7 * ut, amp=args.perturbation, seed=1234,
                                           kmax=3)
    rho0, u0 = rho_f[:, :ny, :].copy(), u_f[:, :, :ny, :].copy()
    del rho_f, u_f
    every = max(1, tstar // args.samples_per_tstar)
    n_trans, n_stats = int(args.tstar_transient * tstar), int(args.tstar_stats * tstar)
    t0 = time.time()
    with L.Lattice(cfg) as lat:
        lat.init(rho0, u0)
        del rho0, u0
        log(f"initialised; {n_trans} transient + {n_stats} statistics steps")
        stats = ProfileStats(torch, ny)
        done = 0
        t_run = 0.0
        while done < n_trans + n_stats:
            k = min(every, n_trans + n_stats - done)
            t1 = time.perf_counter()
            lat.step(k)
            lat.synchronize()
            t_run += time.perf_counter() - t1
            done += k
            if done > n_trans:
                _, u = device_moments(L, torch, lat)
                stats.add(u)
            d = lat.diagnostics()
            tau_w = d["wall_force"][0] / (nx * nz)
            log(f"step {done} (t* {done / tstar:.2f}): u_bulk/u_tau {d['momentum'][0] / d['mass'] / ut:.3f} "
                f"u_tau(wall)/u_tau {np.sqrt(max(tau_w, 0)) / ut:.4f} max|u| {d['max_speed']:.4f}")
        dfin = lat.diagnostics()
    pr = stats.result()
    yplus = (np.arange(ny) + 0.5) * ut / nu
    tau_w = dfin["wall_force"][0] / (nx * nz)
    out.update({
        "steps": n_trans + n_stats, "stats_steps": n_stats, "samples": pr["samples"],
        "mlups": nx * ny * nz * (n_trans + n_stats) / t_run / 1e6, "wall_s": time.time() - t0,
        "u_tau_wall_over_u_tau": float(np.sqrt(max(tau_w, 0.0)) / ut),
        "u_bulk_over_u_tau": float(dfin["momentum"][0] / dfin["mass"] / ut),
        "y_plus": [round(float(v), 3) for v in yplus],
        "U_plus": [round(float(v) / ut, 4) for v in pr["U"]],
        "u_rms_plus": [round(float(v) / ut, 4) for v in pr["u_rms"]],
        "v_rms_plus": [round(float(v) / ut, 4) for v in pr["v_rms"]],
        "w_rms_plus": [round(float(v) / ut, 4) for v in pr["w_rms"]],
        "uv_plus": [round(float(v) / ut ** 2, 5) for v in pr["uv"]],
    })
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
