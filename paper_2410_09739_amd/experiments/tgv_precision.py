"""3D Taylor-Green vortex at Re = 1600 (u0 = 0.05, L = N / 2 pi, nu = u0 L / Re)
on an N^3 periodic box: kinetic-energy and dissipation histories of each
storage form against the FP64 run on the same GPU.  Dissipation is reported as
eps = nu <|curl u|^2> (from the enstrophy diagnostic) and as -dE/dt from the
kinetic-energy history; time t* = t u0 / L.

    python -m paper_2410_09739_amd.experiments.tgv_precision [--n 512] [--tstar 10]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--tstar", type=float, default=10.0)
    ap.add_argument("--samples", type=int, default=50)
    ap.add_argument("--forms", default="f64,f32,f16dev,bf16dev")
    ap.add_argument("--re", type=float, default=1600.0)
    args = ap.parse_args()
    import torch

    from paper_2410_09739_amd import lbm as L
    from paper_2410_09739_amd import workloads as W

    n, u0 = args.n, 0.05
    Lc = n / (2 * np.pi)
    nu = u0 * Lc / args.re
    steps = int(round(args.tstar * Lc / u0))
    every = max(1, steps // args.samples)
    rho, u = W.taylor_green(n, u0=u0)
    rd = torch.tensor(rho.ravel(), device="cuda")
    ud = torch.tensor(u.reshape(3, -1).ravel(), device="cuda")
    del rho, u
    torch.cuda.synchronize()
    N = n ** 3
    out = {"workload": f"Taylor-Green {n}^3, Re={args.re}, u0={u0}, nu={nu:.6e}", "steps": steps, "every": every,
           "forms": {}}
    hist = {}
    for st in args.forms.split(","):
        t0 = time.time()
        ts, ke, eps = [], [], []
        with L.Lattice(L.Config(n, n, n, storage=st, nu=nu)) as lat:
            L.lbm_init_device(lat.ctx, rd.data_ptr(), ud.data_ptr())
            done = 0
            while True:
                d = lat.diagnostics()
                ts.append(done * u0 / Lc)
                ke.append(d["kinetic_energy"] / N)
                eps.append(2.0 * nu * d["enstrophy"] / N)
                if done >= steps:
                    break
                k = min(every, steps - done)
                lat.step(k)
                done += k
                if len(ts) % 5 == 0:
                    print(f"# {st} t*={ts[-1]:.2f} KE={ke[-1]:.4e} eps={eps[-1]:.4e}", file=sys.stderr, flush=True)
        ke, eps = np.array(ke), np.array(eps)
        dedt = -np.gradient(ke, np.array(ts) * Lc / u0)
        hist[st] = (ke, eps, dedt)
        out["forms"][st] = {"tstar": ts, "ke": ke.tolist(), "eps_enstrophy": eps.tolist(), "eps_dEdt": dedt.tolist(),
                            "wall_s": time.time() - t0, "mlups_incl_diag": N * steps / (time.time() - t0) / 1e6}
    if "f64" in hist:
        k64, e64, d64 = hist["f64"]
        for st, (k, e, dd) in hist.items():
            out["forms"][st]["max_rel_err_ke_vs_f64"] = float(np.max(np.abs(k - k64) / np.abs(k64)))
            out["forms"][st]["max_err_eps_vs_f64_over_peak"] = float(np.max(np.abs(e - e64)) / np.max(e64))
            out["forms"][st]["max_err_dEdt_vs_f64_over_peak"] = float(np.max(np.abs(dd - d64)) / np.max(np.abs(d64)))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
