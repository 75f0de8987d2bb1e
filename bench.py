#!/usr/bin/env python3
"""Benchmark of the fused D3Q27 FPC-LBM stream-and-collide step on one MI355X.

Workload (the channel case): 256 x 128 x 128 nodes, walls half a link outside
y = 0 and y = 127 (halfway bounce-back), periodic in x and z, nu = 0.01,
constant body force F_x = 8 nu u_max / H^2 with u_max = 0.05 and H = 128,
starting from rest.  A step is one fused stream + collide launch over all
nodes.  Inputs are synthetic (no dataset) and already resident in HBM when the
timed region starts.

Printed (one JSON line): MLUPS of the FP32-storage form as ``value``, the HBM
roofline of the stream-collide kernel measured with HIP events on the stream
the kernel runs on, every storage form's MLUPS / roofline fraction / error
against the analytic start-up profile and against the FP64 run, and the FP64
CPU oracle timed on a bounded sample of the same workload.
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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_stream_collide_channel_256x128x128.md")


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


def analytic_startup(ny: int, nu: float, F: float, t: float, nterms: int = 400) -> np.ndarray:
    """Start-up of plane Poiseuille flow from rest between walls at y = 0 and H
    (here the half-link wall positions), u(y, t) for the node centres."""
    H = float(ny)
    y = np.arange(ny) + 0.5
    u = F / (2 * nu) * y * (H - y)
    for n in range(1, 2 * nterms, 2):
        u -= 4 * F * H * H / (nu * n ** 3 * np.pi ** 3) * np.sin(n * np.pi * y / H) * np.exp(-n * n * np.pi ** 2 * nu * t / (H * H))
    return u


def run_form(L, torch, storage, shape, nu, F, steps, warmup):
    nx, ny, nz = shape
    stream = torch.cuda.Stream()
    cfg = L.Config(nx, ny, nz, storage=storage, walls_y=True, nu=nu, force=(F, 0.0, 0.0),
                   hip_stream=stream.cuda_stream)
    with L.Lattice(cfg) as lat:
        lat.init()  # rest: rho = 1, u = 0
        lat.step(warmup)
        lat.synchronize()
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record(stream)
        lat.step(steps)
        end.record(stream)
        end.synchronize()
        torch.cuda.synchronize()
        ms = start.elapsed_time(end)
        _, u = lat.moments()
        diag = lat.diagnostics()
    return ms, u, diag


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


def copy_calibration(torch, nbytes: int = 1 << 31, reps: int = 5):
    """A plain device copy of known size, to scale the HBM byte counters."""
    x = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": nbytes, "bytes_written": nbytes, "reps": reps}), flush=True)


def cpu_baseline(shape, nu, F, steps):
    import oracle as O
    nx, ny, nz = shape
    g = O.init(np.ones((nz, ny, nx)), np.zeros((3, nz, ny, nx)))
    om = O.omega_table(nu)
    t0 = time.perf_counter()
    O.run(g, om, (F, 0.0, 0.0), walls_y=True, steps=steps)
    dt = time.perf_counter() - t0
    return nx * ny * nz * steps / dt / 1e6, dt, O.num_threads()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--forms", default="f32,f64,f16dev,bf16dev")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=200)
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

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        copy_calibration(torch)
        return
    shape = (256, 128, 128)
    nx, ny, nz = shape
    N = nx * ny * nz
    nu, umax = 0.01, 0.05
    F = 8 * nu * umax / ny ** 2

    forms = [s for s in args.forms.split(",") if s]
    if "f32" not in forms:
        forms.insert(0, "f32")
    results, profiles = {}, {}
    for st in forms:
        ms, u, diag = run_form(L, torch, st, shape, nu, F, args.steps, args.warmup)
        sb = L.STORAGE_BYTES[L.STORAGE[st]]
        ms_step = ms / args.steps
        bytes_launch = N * 54 * sb
        gbs = bytes_launch / (ms_step * 1e-3) / 1e9
        prof = u[0].mean(axis=(0, 2))  # x-z average of u_x(y)
        t = args.warmup + args.steps - 0.5
        ua = analytic_startup(ny, nu, F, t)
        profiles[st] = (u, prof)
        results[st] = {
            "mlups": N / (ms_step * 1e-3) / 1e6,
            "ms_per_step": ms_step,
            "bytes_per_node": 54 * sb,
            "achieved_GBs": gbs,
            "frac_hbm": gbs / HBM_PEAK_GBS,
            "profile_rel_l2_vs_analytic": float(np.sqrt(np.sum((prof - ua) ** 2) / np.sum(ua ** 2))),
            "mass_drift": diag["mass"] / N - 1.0,
        }
        print(f"# {st}: {results[st]['mlups']:.0f} MLUPS, {gbs:.0f} GB/s, "
              f"profile err {results[st]['profile_rel_l2_vs_analytic']:.2e}", file=sys.stderr, flush=True)
    if "f64" in profiles:
        u64 = profiles["f64"][0]
        for st in results:
            results[st]["max_abs_u_err_vs_f64_over_umax"] = float(np.abs(profiles[st][0] - u64).max() / umax)

    # learned-closure forms on the coarse channel 192 x 96 x 96 (the closure
    # workload: nu and force of the fine channel under acoustic 2x coarsening)
    closure = {}
    if args.closure_steps > 0:
        cshape = (192, 96, 96)
        params = closure_params()
        for st, use in [("f32", False), ("f16dev", False), ("bf16dev", False), ("f32", True), ("f16dev", True),
                        ("bf16dev", True)]:
            key = st + ("+closure" if use else "")
            closure[key] = run_closure_form(L, torch, st, cshape, nu / 2, 2 * F, args.closure_steps, 20,
                                            params if use else None)
            closure[key] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in closure[key].items()}
            print(f"# coarse {key}: {closure[key]['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)

    main_form = results["f32"]
    roof = {"bound": "hbm", "achieved": round(main_form["achieved_GBs"], 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(main_form["frac_hbm"], 4), "traffic": None}
    tr = P.read_traffic_md(TRAFFIC_FILE)
    if tr and tr.get("kernel_source_sha") == P.kernel_source_hash() and "f32" in tr.get("forms", {}):
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
        "config": {"workload": "channel 256x128x128, halfway bounce-back walls in y, body force, nu=0.01, "
                               "u_max=0.05, from rest; FP32 storage of f - w",
                   "nx": nx, "ny": ny, "nz": nz, "parallelism": "single GPU"},
        "roofline": roof,
        "forms": {k: {kk: (round(vv, 6) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                  for k, v in results.items()},
        "closure_forms_192x96x96": closure,
    }
    if not args.no_cpu_baseline:
        cshape = (256, 128, 16)
        mlups, dt, cores = cpu_baseline(cshape, nu, F, args.cpu_steps)
        line["cpu_baseline"] = {"value": round(mlups, 3), "unit": "MLUPS", "cores": cores, "kind": "oracle",
                                "sample": f"{args.cpu_steps} steps of a 256x128x16 slab of the same channel "
                                          f"(periodic z), FP64, {dt:.1f} s"}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
