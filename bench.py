#!/usr/bin/env python3
"""Benchmark of the fused D3Q27 FPC-LBM stream-and-collide step on one MI355X.

Workload: the 3D Taylor-Green vortex at Re = 1600 on a 512^3 periodic box
(u0 = 0.05, L = 512 / 2 pi, nu = u0 L / Re = 2.5465e-3; u = u0 sin x cos y cos z,
v = -u0 cos x sin y cos z, w = 0, rho = 1 + 3 p' with the matching pressure,
populations at equilibrium).  A step is one fused stream + collide launch over
all 134,217,728 nodes.  Inputs are synthetic and already resident in HBM when
the timed region starts.

Every storage form (FP64, FP32, FP16 and BF16 deviations from the lattice
weights) runs the same sequence from the same start: ``--settle`` untimed steps
(the kernels reach their steady clock and the flow leaves the initial field),
``--warmup`` untimed steps, then ``--steps`` steps timed with HIP events on the
library's stream.  At the end of the window each form's kinetic energy,
dissipation nu <|curl u|^2> and velocity field are compared with the FP64 run
on the same GPU: that is the error at which the form's throughput is stated.

Printed (one JSON line): MLUPS of the FP32-storage form as ``value``, the HBM
roofline of its stream-collide kernel (algorithmic bytes per launch over the
measured launch time), every storage form's MLUPS, roofline fraction and error
against FP64, the learned-closure kernel beside the plain step on the coarse
channel 192x96x96 and on the turbulent-channel grid 384x192x192 for context,
and the FP64 CPU oracle timed on a bounded slab of the same field.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
N_TGV = 512
U0 = 0.05
RE = 1600.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_stream_collide_taylor_green_512.md")


def tgv_params(n: int):
    Lc = n / (2 * np.pi)
    return Lc, U0 * Lc / RE


def closure_params():
    """Parameters of the trained closure if the repository holds them, else a
    He-initialised network (throughput does not depend on the weights)."""
    path = os.path.join(ROOT, "paper_2410_09739_amd", "data", "closure_channel_192x96x96.npy")
    if os.path.exists(path):
        return np.load(path).astype(np.float32)
    rng = np.random.default_rng(0)
    sizes = [(64, 27), (64,), (64, 64), (64,), (6, 64), (6,)]
    parts = []
    for shp in sizes:
        fan = shp[1] if len(shp) == 2 else 1
        parts.append((rng.uniform(-1, 1, shp) * np.sqrt(6.0 / fan) * (len(shp) == 2)).ravel())
    return np.concatenate(parts).astype(np.float32) * 1e-3


def run_tgv_form(L, torch, storage, n, nu, rd, ud, settle, warmup, steps):
    """One storage form: init from the device fields, settle + warmup untimed,
    then ``steps`` launches timed with HIP events on the library's stream.
    Returns the time per step, the end diagnostics and the FP64 velocity field
    at the end (a device tensor)."""
    stream = torch.cuda.Stream()
    cfg = L.Config(n, n, n, storage=storage, nu=nu, hip_stream=stream.cuda_stream)
    with L.Lattice(cfg) as lat:
        L.lbm_init_device(lat.ctx, rd.data_ptr(), ud.data_ptr())
        lat.step(settle + warmup)
        lat.synchronize()
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        start.record(stream)
        lat.step(steps)
        end.record(stream)
        end.synchronize()
        ms = start.elapsed_time(end) / steps
        diag = lat.diagnostics()
        u = torch.empty(3 * n ** 3, dtype=torch.float64, device="cuda")
        L.lbm_moments_device(lat.ctx, 0, u.data_ptr(), True)
        lat.synchronize()
    return ms, diag, u


def run_closure_form(L, torch, storage, shape, nu, F, steps, warmup, params):
    """MLUPS of the fused closure kernel (params: raw-feature parameters) or of
    the plain kernel (params None) on the coarse channel."""
    nx, ny, nz = shape
    stream = torch.cuda.Stream()
    cfg = L.Config(nx, ny, nz, storage=storage, walls_y=True, nu=nu, force=(F, 0.0, 0.0),
                   hip_stream=stream.cuda_stream)
    with L.Lattice(cfg) as lat:
        lat.init()
        if params is not None:
            L.lbm_set_closure(lat.ctx, params)
        lat.step(warmup)
        lat.synchronize()
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        start.record(stream)
        lat.step(steps)
        end.record(stream)
        end.synchronize()
        ms = start.elapsed_time(end) / steps
        d = lat.diagnostics()
    n = nx * ny * nz
    return {"mlups": n / (ms * 1e-3) / 1e6, "ms_per_step": ms, "finite": d["n_nonfinite"] == 0}


def closure_cost_at_equal_error(cg: dict, form: str = "f16dev+closure"):
    """Cost of plain FP32 at the closure form's mean-flow error, over the
    closure form's cost, on the coarse channel 192 x 96 x 96.  The errors are
    those the closure study measured on held-out starts (data file, with the
    command that produced them); the rates are this run's.  Plain runs' error
    goes as dx^p between the two coarse grids, so plain FP32 reaches the
    closure's error on a grid r = (e_plain / e_closure)^(1/p) times finer per
    direction; at equal physical time that costs r^4 (nodes r^3, acoustic steps
    r) at the plain FP32 rate, against the closure form at its own rate."""
    import hashlib
    data = os.path.join(ROOT, "paper_2410_09739_amd", "data")
    path = os.path.join(data, "closure_channel_errors.json")
    if not os.path.exists(path) or "f32" not in cg or form not in cg:
        return None
    d = json.load(open(path))
    # the errors hold for the networks they were measured with
    for name, sha in d.get("networks_sha256", {}).items():
        f = os.path.join(data, name)
        if not os.path.exists(f) or hashlib.sha256(open(f, "rb").read()).hexdigest() != sha:
            return None
    g1, g0 = d["grids"]["192x96x96"], d["grids"]["128x64x64"]
    e_plain, e_cl = float(np.mean(g1["plain_f32"])), float(np.mean(g1["closure_f16dev"]))
    p = float(np.log(np.mean(g0["plain_f32"]) / e_plain) / np.log(1.5))
    r = (e_plain / e_cl) ** (1.0 / p)
    return {"grid": "channel_192x96x96", "form": form, "U_error_closure": round(e_cl, 4),
            "U_error_plain_f32": round(e_plain, 4), "plain_error_order": round(p, 3),
            "plain_refinement_for_equal_error": round(r, 3),
            "plain_f32_cost_over_closure_cost": round(r ** 4 * cg[form]["mlups"] / cg["f32"]["mlups"], 2),
            "errors_from": d["command"]}


def copy_calibration(torch, nbytes: int = 1 << 31, reps: int = 5):
    """A plain device copy of known size, to scale the HBM byte counters."""
    x = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": nbytes, "bytes_written": nbytes, "reps": reps}), flush=True)


def copy_bandwidth(torch, nbytes: int = 1 << 31, reps: int = 10) -> float:
    """GB/s of a plain device-to-device copy (torch, nbytes read and nbytes
    written per copy), timed with events after two untimed copies: the rate a
    simple streaming kernel reaches on this GPU, beside the published peak."""
    x = torch.zeros(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(2):
        y.copy_(x)
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        y.copy_(x)
    end.record()
    end.synchronize()
    gbs = 2.0 * nbytes * reps / (start.elapsed_time(end) * 1e-3) / 1e9
    del x, y
    torch.cuda.empty_cache()
    return gbs


def cpu_baseline(n, nu, planes, steps):
    """The FP64 oracle on the first ``planes`` z-planes of the same n^3 field
    (periodic in z over the slab): the work per node is that of the full box."""
    import oracle as O
    from paper_2410_09739_amd import workloads as W
    rho, u = W.taylor_green(n)
    rho, u = np.ascontiguousarray(rho[:planes]), np.ascontiguousarray(u[:, :planes])
    g = O.init(rho, u)
    del rho, u
    om = O.omega_table(nu)
    t0 = time.perf_counter()
    O.run(g, om, steps=steps)
    dt = time.perf_counter() - t0
    return n * n * planes * steps / dt / 1e6, dt, O.num_threads()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--settle", type=int, default=200,
                    help="untimed steps before the warmup (steady clock, developed flow)")
    ap.add_argument("--n", type=int, default=N_TGV, help="edge of the periodic box (512: the headline case)")
    ap.add_argument("--forms", default="f64,f32,f16dev,bf16dev")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-planes", type=int, default=16)
    ap.add_argument("--cpu-steps", type=int, default=8)
    ap.add_argument("--closure-steps", type=int, default=500)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain copy of known size (for scaling rocprofv3 byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU slab decomposition is designed, not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2410_09739_amd import lbm as L
    from paper_2410_09739_amd import profiling as P
    from paper_2410_09739_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        copy_calibration(torch)
        return
    n = args.n
    N = n ** 3
    Lc, nu = tgv_params(n)
    rho, u = W.taylor_green(n, u0=U0)
    rd = torch.from_numpy(rho.ravel()).cuda()
    ud = torch.from_numpy(u.reshape(-1)).cuda()
    del rho, u
    mass0 = float(rd.sum().item())
    torch.cuda.synchronize()

    forms = [s for s in args.forms.split(",") if s]
    if "f32" not in forms:
        forms.insert(0, "f32")
    if "f64" in forms:  # the reference of every error runs first
        forms.remove("f64")
        forms.insert(0, "f64")
    total = args.settle + args.warmup + args.steps
    results, u64, d64 = {}, None, None
    for st in forms:
        ms, diag, uf = run_tgv_form(L, torch, st, n, nu, rd, ud, args.settle, args.warmup, args.steps)
        sb = L.STORAGE_BYTES[L.STORAGE[st]]
        bytes_launch = N * 54 * sb
        gbs = bytes_launch / (ms * 1e-3) / 1e9
        r = {"mlups": N / (ms * 1e-3) / 1e6, "ms_per_step": ms, "bytes_per_node": 54 * sb,
             "achieved_GBs": gbs, "frac_hbm": gbs / HBM_PEAK_GBS,
             "kinetic_energy_per_node": diag["kinetic_energy"] / N,
             "dissipation_per_node": 2.0 * nu * diag["enstrophy"] / N,
             "mass_rel_drift": (diag["mass"] - mass0) / mass0}
        if st == "f64":
            u64, d64 = uf, diag
        elif u64 is not None:
            r["ke_rel_err_vs_f64"] = abs(diag["kinetic_energy"] - d64["kinetic_energy"]) / d64["kinetic_energy"]
            r["dissipation_rel_err_vs_f64"] = abs(diag["enstrophy"] - d64["enstrophy"]) / d64["enstrophy"]
            r["max_abs_u_err_vs_f64_over_u0"] = float((uf - u64).abs().max().item()) / U0
            r["rms_u_err_vs_f64_over_u0"] = float(((uf - u64) ** 2).mean().sqrt().item()) / U0
        del uf
        results[st] = r
        print(f"# {st}: {r['mlups']:.0f} MLUPS, {gbs:.0f} GB/s ({r['frac_hbm']:.3f} of peak)"
              + (f", KE err {r['ke_rel_err_vs_f64']:.2e}, max|du|/u0 {r['max_abs_u_err_vs_f64_over_u0']:.2e}"
                 if "ke_rel_err_vs_f64" in r else ""), file=sys.stderr, flush=True)
    if "f64" in results:
        results["f64"].update({"ke_rel_err_vs_f64": 0.0, "dissipation_rel_err_vs_f64": 0.0,
                               "max_abs_u_err_vs_f64_over_u0": 0.0, "rms_u_err_vs_f64_over_u0": 0.0})
    del u64, rd, ud
    torch.cuda.empty_cache()

    # learned-closure forms (context): the coarse channel 192 x 96 x 96 of the
    # closure workload (nu and force of the fine channel under 2x coarsening,
    # 2 x 191 MB of 16-bit state: held in the 256 MB last-level cache), and the
    # turbulent-channel grid 384 x 192 x 192 at Re_tau = 180 (u_tau = 0.0025,
    # h = 96), whose state does not fit in that cache.  Each form's plain
    # step beside it; "vs_f32_plain" = MLUPS over the plain FP32 step's.
    closure = {}
    if args.closure_steps > 0:
        params = closure_params()
        ut = 0.0025
        grids = [("channel_192x96x96", (192, 96, 96), 0.005, 2 * 8 * 0.01 * 0.05 / 128 ** 2, args.closure_steps),
                 ("channel_384x192x192", (384, 192, 192), ut * 96 / 180, ut * ut / 96,
                  max(1, args.closure_steps // 5))]
        for gname, cshape, cnu, F, csteps in grids:
            cg = {}
            for st, use in [("f32", False), ("f16dev", False), ("bf16dev", False), ("f32", True),
                            ("f16dev", True), ("bf16dev", True)]:
                key = st + ("+closure" if use else "")
                cg[key] = run_closure_form(L, torch, st, cshape, cnu, F, csteps, 200, params if use else None)
                print(f"# {gname} {key}: {cg[key]['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
            for key in cg:
                cg[key]["vs_f32_plain"] = cg[key]["mlups"] / cg["f32"]["mlups"]
                cg[key] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in cg[key].items()}
            cg["steps"] = csteps
            closure[gname] = cg
        cost = closure_cost_at_equal_error(closure["channel_192x96x96"])
        if cost is not None:
            closure["cost_at_equal_error"] = cost
            print(f"# closure cost at equal mean-flow error: plain FP32 / {cost['form']} = "
                  f"{cost['plain_f32_cost_over_closure_cost']}", file=sys.stderr, flush=True)

    main_form = results["f32"]
    roof = {"bound": "hbm", "achieved": round(main_form["achieved_GBs"], 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(main_form["frac_hbm"], 4), "traffic": None}
    tr = P.read_traffic_md(TRAFFIC_FILE)
    if (tr and tr.get("kernel_source_sha") == P.kernel_source_hash() and "f32" in tr.get("forms", {})
            and tr.get("nodes") == N):
        roof["traffic"] = tr["forms"]["f32"]["hbm_bytes_per_launch"]

    line = {
        "metric": "D3Q27 FPC-LBM MLUPS & % HBM peak, FP32 vs FP16-storage at stated error",
        "value": round(main_form["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_form["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"Taylor-Green vortex {n}^3 periodic, Re=1600, u0=0.05, nu={nu:.5e}; "
                               f"FP32 storage of f - w; {args.settle} settle + {args.warmup} warmup steps "
                               f"untimed, {args.steps} timed",
                   "nx": n, "ny": n, "nz": n, "settle_steps": args.settle,
                   "error_at_step": total, "error_at_tstar": round(total * U0 / Lc, 4),
                   "parallelism": "single GPU"},
        "roofline": roof,
        "forms": {k: {kk: (float(f"{vv:.6g}") if isinstance(vv, float) else vv) for kk, vv in v.items()}
                  for k, v in results.items()},
        "closure_forms": closure,
    }
    cgbs = copy_bandwidth(torch)
    line["copy_reference"] = {"copy_GBs": round(cgbs, 1), "f32_achieved_over_copy": round(roof["achieved"] / cgbs, 4),
                              "what": "torch device-to-device copy of 2 GiB (read + write counted), 10 timed copies"}
    print(f"# plain device copy: {cgbs:.0f} GB/s; FP32 step at {roof['achieved'] / cgbs:.3f} of it",
          file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        mlups, dt, cores = cpu_baseline(n, nu, args.cpu_planes, args.cpu_steps)
        line["cpu_baseline"] = {"value": round(mlups, 3), "unit": "MLUPS", "cores": cores, "kind": "oracle",
                                "sample": f"{args.cpu_steps} steps of the first {args.cpu_planes} z-planes "
                                          f"({n}x{n}x{args.cpu_planes} nodes, periodic) of the same {n}^3 "
                                          f"Taylor-Green field, FP64, {dt:.1f} s"}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
