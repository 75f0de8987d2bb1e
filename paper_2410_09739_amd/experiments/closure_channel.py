"""Learned-closure channel study: a fine turbulent channel at Re_tau = 180
(384 x 192 x 192, half-width h = 96, u_tau = 0.0025, nu_f = u_tau h / 180,
F_f = rho u_tau^2 / h) gives box-filtered snapshots on the 192 x 96 x 96 grid;
the per-node MLP closure is trained on them on the GPU and drives coarse runs
(acoustic scaling: nu_c = nu_f / 2, F_c = 2 F_f).  Reports, over a statistically
steady window, the bulk velocity and the mean and RMS velocity profiles of the
plain coarse run, the closure run and the filtered fine run, the wall friction
velocity of each, the wall time of each, and the trained parameters (.npy).

    python -m paper_2410_09739_amd.experiments.closure_channel [--tstar-transient 6] [--tstar-stats 6]
        [--shape 256,128,128] [--seeds 3] [--gains 1,3] [--coarse-storage f32,f16dev]
        [--refine 1 --calibrate] [--load-params trained.npy --flow-seed 4321]

Time unit T* = h / u_tau (38,400 fine steps).  The fine run gives a snapshot
every T*/2 of its statistics window (the last one held out of training).  The
coarse runs start from the filtered fine state at the end of the fine transient
and run --coarse-run T*; their statistics cover the last --coarse-stats T*, by
when the bulk velocity of the coarse grid has settled.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def log(msg: str) -> None:
    print(f"# {msg}", file=sys.stderr, flush=True)


class ProfileStats:
    """x-z and time averages of u, v, w, their squares and u v, per y row."""

    def __init__(self, torch, ny: int):
        self.torch = torch
        self.sum = torch.zeros((7, ny), dtype=torch.float64, device="cuda")
        self.count = 0

    def add(self, u):  # u: [3, nz, ny, nx] float64 on the device
        t = self.torch
        m = t.stack([u[0], u[1], u[2], u[0] * u[0], u[1] * u[1], u[2] * u[2], u[0] * u[1]])
        self.sum += m.mean(dim=(1, 3))
        self.count += 1

    def result(self) -> dict:
        s = (self.sum / max(self.count, 1)).cpu().numpy()
        U, V, Wm = s[0], s[1], s[2]
        return {"U": U, "u_rms": np.sqrt(np.maximum(s[3] - U * U, 0)), "v_rms": np.sqrt(np.maximum(s[4] - V * V, 0)),
                "w_rms": np.sqrt(np.maximum(s[5] - Wm * Wm, 0)), "uv": s[6] - U * V, "samples": self.count}


def device_moments(L, torch, lat):
    rho = torch.empty(lat.n, dtype=torch.float64, device="cuda")
    u = torch.empty(3 * lat.n, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    L.lbm_moments_device(lat.ctx, rho.data_ptr(), u.data_ptr(), True)
    lat.synchronize()
    return rho.view(lat.shape), u.view((3,) + lat.shape)


def friction_velocity(d: dict, nx: int, nz: int) -> float:
    tau_w = d["wall_force"][0] / (2.0 * nx * nz)  # two walls, unit area per node
    return float(np.sqrt(max(tau_w, 0.0)))


def run_window(L, torch, lat, steps: int, every: int, stats: ProfileStats | None, tag: str, on_sample=None,
               u_bulk: list | None = None):
    done = 0
    t_run = 0.0
    while done < steps:
        k = min(every, steps - done)
        t0 = time.perf_counter()
        lat.step(k)
        lat.synchronize()
        t_run += time.perf_counter() - t0
        done += k
        if stats is not None:
            _, u = device_moments(L, torch, lat)
            stats.add(u)
        if on_sample is not None:
            on_sample(done)
        d = lat.diagnostics()
        if u_bulk is not None:
            u_bulk.append(d["momentum"][0] / d["mass"])
        log(f"{tag} step {lat.steps}: u_bulk {d['momentum'][0] / d['mass']:.5f} "
            f"u_tau {friction_velocity(d, lat.cfg.nx, lat.cfg.nz):.5f} max|u| {d['max_speed']:.4f}")
    return t_run


def coarse_profile_of_fine(p: dict) -> dict:
    """Average pairs of fine rows onto the coarse rows (the y part of the 2x2x2 filter)."""
    return {k: (0.5 * (v[0::2] + v[1::2]) if isinstance(v, np.ndarray) else v) for k, v in p.items()}


def scaled_output(params: np.ndarray, gain: float) -> np.ndarray:
    """Parameters whose network output is gain times the given one: the output
    layer is linear, so W3 and b3 scale (and the kernel's clamp at zero commutes
    with a positive gain)."""
    p = np.array(params, dtype=np.float32, copy=True)
    p[-(6 * 64 + 6):] *= gain
    return p


def balance_eddy_viscosity(prof_c: dict, filt: dict, u_tau: float, nu: float, cap: float) -> np.ndarray:
    """Eddy viscosity per coarse row that makes the coarse run's total shear
    stress carry the filtered fine mean profile: in a statistically steady
    channel (nu + nu_t) dU/dy - <u'v'> = u_tau^2 (1 - y/h) with y from the lower
    wall (halfway bounce-back: row j at y = j + 1/2), so with the coarse run's
    resolved <u'v'> and the filtered fine dU/dy,
    nu_t = (u_tau^2 (1 - y/h) + <u'v'>_c) / dU_f/dy - nu, clipped to [0, cap].
    The two halves are averaged as mirror images."""
    U, uv = filt["U"], prof_c["uv"]
    ny = len(U)
    h = ny / 2.0
    y = np.arange(ny) + 0.5
    dU = np.empty(ny)
    dU[1:-1] = 0.5 * (U[2:] - U[:-2])
    dU[0] = 0.5 * (U[1] + U[0])  # ghost row below the wall: -U[0] (no slip half a link below row 0)
    dU[-1] = -0.5 * (U[-1] + U[-2])
    tau = u_tau * u_tau * (1.0 - y / h)
    nut = np.zeros(ny)
    ok = np.abs(dU) > 1e-3 * np.abs(dU).max()
    nut[ok] = (tau[ok] + uv[ok]) / dU[ok] - nu
    nut = 0.5 * (nut + nut[::-1])
    return np.clip(nut, 0.0, cap)


def output_gain(u_plain: float, u_net: float, u_fine: float, lo: float = 0.1, hi: float = 2.0) -> float:
    """Scale g of the network output that gives the coarse run the fine bulk
    velocity, with the bulk velocity taken linear in g between the plain run
    (g = 0) and the unscaled network (g = 1); clipped to [lo, hi], 1 when the
    network does not move the bulk velocity."""
    if u_plain == u_net:
        return 1.0
    return float(np.clip((u_plain - u_fine) / (u_plain - u_net), lo, hi))


def main(argv=None) -> dict:
    ap = argparse.ArgumentParser()
    ap.add_argument("--shape", default="384,192,192")
    ap.add_argument("--u-tau", type=float, default=0.0025)
    ap.add_argument("--re-tau", type=float, default=180.0)
    ap.add_argument("--storage", default="f32")
    ap.add_argument("--tstar-transient", type=float, default=6.0)
    ap.add_argument("--tstar-stats", type=float, default=6.0)
    ap.add_argument("--coarse-run", type=float, default=16.0)
    ap.add_argument("--coarse-stats", type=float, default=8.0)
    ap.add_argument("--samples-per-tstar", type=int, default=4)
    ap.add_argument("--snapshots-per-tstar", type=int, default=2)
    ap.add_argument("--train-steps", type=int, default=5000)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--eps-rel", type=float, default=0.1)
    ap.add_argument("--perturbation", type=float, default=0.3)
    ap.add_argument("--flow-seed", type=int, default=1234, help="seed of the initial perturbation")
    ap.add_argument("--seeds", type=int, default=1, help="networks trained from different initialisations")
    ap.add_argument("--gains", default="1", help="comma list: multipliers of the network output (a-posteriori scale)")
    ap.add_argument("--save-params", default="closure_params.npy")
    ap.add_argument("--coarse-storage", default="f32",
                    help="comma list of storage forms for the coarse runs (plain and closure in each)")
    ap.add_argument("--refine", type=int, default=0,
                    help="a-posteriori passes: coarse run with the network, targets from the mean momentum "
                         "balance of that run, retraining (first network only)")
    ap.add_argument("--refine-relax", type=float, default=0.5, help="under-relaxation of the refined targets")
    ap.add_argument("--refine-groups", default="110",
                    help="off-diagonal groups that take the refined target, the others 0 (the mean momentum "
                         "balance fixes the x-y shear viscosity only; 110,101,011 gives it to all three)")
    ap.add_argument("--calibrate", action="store_true",
                    help="scale the first network's output (first network only) so that the coarse run on the "
                         "training start has the filtered fine bulk velocity (linear between the plain run and the "
                         "unscaled network)")
    ap.add_argument("--load-params", default=None,
                    help="closure parameters (.npy) to evaluate instead of training: a network from another start")
    args = ap.parse_args(argv)
    import torch

    from paper_2410_09739_amd import lbm as L
    from paper_2410_09739_amd import workloads as W

    nx, ny, nz = map(int, args.shape.split(","))
    h = ny / 2.0
    ut = args.u_tau
    nu_f = ut * h / args.re_tau
    F_f = ut * ut / h
    tstar = int(round(h / ut))
    cshape = (nx // 2, ny // 2, nz // 2)
    nc = cshape[0] * cshape[1] * cshape[2]
    out = {"workload": f"turbulent channel {nx}x{ny}x{nz}, Re_tau={args.re_tau}, u_tau={ut}, nu={nu_f:.6e}, "
                       f"F={F_f:.6e}; closure grid {cshape[0]}x{cshape[1]}x{cshape[2]}",
           "tstar_steps": tstar, "args": vars(args)}

    def dev(*shape, dtype=torch.float64):
        return torch.zeros(shape, dtype=dtype, device="cuda")

    # ---- fine run: transient, then statistics and training snapshots
    u_bulk0 = 15.7 * ut  # bulk velocity of the turbulent state at Re_tau = 180 (u_b / u_tau ~ 15.7)
    rho0, u0 = W.channel_turbulent_start(nx, ny, nz, u_bulk=u_bulk0, amp=args.perturbation, seed=args.flow_seed)
    fcfg = L.Config(nx, ny, nz, storage=args.storage, walls_y=True, nu=nu_f, force=(F_f, 0, 0))
    every = max(1, tstar // args.samples_per_tstar)
    snap_every = max(every, tstar // args.snapshots_per_tstar)
    n_trans, n_stats = int(args.tstar_transient * tstar), int(args.tstar_stats * tstar)
    xs, ys = [], []
    with L.Lattice(fcfg) as fine:
        fine.init(rho0, u0)
        del rho0, u0
        log(f"fine transient {n_trans} steps")
        t_fine = run_window(L, torch, fine, n_trans, every, None, "fine")
        # filtered state at the end of the transient: start of every coarse run
        rc0, uc0, tc0 = dev(nc), dev(3 * nc), dev(6 * nc)
        torch.cuda.synchronize()
        L.lbm_coarsen(fine.ctx, rc0.data_ptr(), uc0.data_ptr(), tc0.data_ptr())
        fine.synchronize()
        ccfg = L.Config(*cshape, storage="f32", walls_y=True, nu=nu_f / 2, force=(2 * F_f, 0, 0))
        feat_lat = L.Lattice(ccfg)

        def snapshot(done):
            if done % snap_every:
                return
            rd, ud, td, sd = dev(nc), dev(3 * nc), dev(6 * nc), dev(6 * nc)
            xd, yd = dev(nc, 27, dtype=torch.float32), dev(nc, 6, dtype=torch.float32)
            torch.cuda.synchronize()
            L.lbm_coarsen(fine.ctx, rd.data_ptr(), ud.data_ptr(), td.data_ptr(), sd.data_ptr())
            fine.synchronize()
            L.lbm_init_device(feat_lat.ctx, rd.data_ptr(), ud.data_ptr())
            L.lbm_closure_features(feat_lat.ctx, xd.data_ptr())
            L.lbm_closure_targets(feat_lat.ctx, rd.data_ptr(), ud.data_ptr(), td.data_ptr(), sd.data_ptr(),
                                  args.eps_rel, yd.data_ptr())
            feat_lat.synchronize()
            xs.append(xd)
            ys.append(yd)
            log(f"snapshot {len(xs)}: mean target nu_t / nu_c {(yd[:, :3].mean(dim=0) / (nu_f / 2)).cpu().numpy()}")

        fstats = ProfileStats(torch, ny)
        f_ub = []
        log(f"fine statistics {n_stats} steps, snapshot every {snap_every}")
        t_fine += run_window(L, torch, fine, n_stats, every, fstats, "fine", snapshot, f_ub)
        dfin = fine.diagnostics()
        feat_lat.close()
    fine_prof = fstats.result()
    out["fine"] = {"wall_s": t_fine, "steps": n_trans + n_stats, "u_tau_end": friction_velocity(dfin, nx, nz),
                   "u_bulk_over_u_tau": float(np.mean(f_ub) / ut), "u_bulk_std_over_u_tau": float(np.std(f_ub) / ut)}
    filt = coarse_profile_of_fine(fine_prof)

    # ---- training on all snapshots but the last; the last is held out
    X = torch.cat(xs[:-1]) if len(xs) > 1 else xs[0]
    Y = torch.cat(ys[:-1]) if len(ys) > 1 else ys[0]
    Xh, Yh = xs[-1], ys[-1]
    torch.cuda.synchronize()
    ntr = X.shape[0]
    gains = [float(g) for g in args.gains.split(",")]
    nets = []
    out["training"] = []
    if args.load_params:
        nets.append(np.load(args.load_params).astype(np.float32))
        log(f"closure parameters from {args.load_params} (no training)")
    for k in range(0 if args.load_params else args.seeds):
        m = L.MLP(seed=11 + k)
        m.fit_normalisation(X.data_ptr(), Y.data_ptr(), ntr)
        l0, _ = m.loss_grad(X.data_ptr(), Y.data_ptr(), ntr)
        lh0, _ = m.loss_grad(Xh.data_ptr(), Yh.data_ptr(), Xh.shape[0])
        t0 = time.perf_counter()
        hist = m.train(X.data_ptr(), Y.data_ptr(), ntr, args.batch, args.train_steps, args.lr, 5 + k)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        l1, _ = m.loss_grad(X.data_ptr(), Y.data_ptr(), ntr)
        lh1, _ = m.loss_grad(Xh.data_ptr(), Yh.data_ptr(), Xh.shape[0])
        nets.append(m.export())
        m.close()
        out["training"].append({"seed": 11 + k, "samples": int(ntr), "held_out": int(Xh.shape[0]),
                                "loss_train_before": l0, "loss_train_after": l1, "loss_heldout_before": lh0,
                                "loss_heldout_after": lh1, "wall_s": t_train, "steps": args.train_steps,
                                "batch": args.batch, "loss_history_every_100": [float(v) for v in hist[::100]]})
        log(f"training {k}: loss {l0:.4e} -> {l1:.4e}, held-out {lh0:.4e} -> {lh1:.4e}, {t_train:.1f} s")
    # ---- coarse runs from the filtered fine state
    cforms = [s for s in args.coarse_storage.split(",") if s]
    ctstar = tstar // 2  # dt_c = 2 dt_f
    cevery = max(1, every // 2)
    c_settle = int((args.coarse_run - args.coarse_stats) * ctstar)
    c_stats = int(args.coarse_stats * ctstar)

    def coarse_run(st, p, tag):
        with L.Lattice(L.Config(*cshape, storage=st, walls_y=True, nu=nu_f / 2, force=(2 * F_f, 0, 0))) as c:
            L.lbm_init_device(c.ctx, rc0.data_ptr(), uc0.data_ptr())
            if p is not None:
                L.lbm_set_closure(c.ctx, p)
            t_c = run_window(L, torch, c, c_settle, cevery, None, tag)
            cs = ProfileStats(torch, cshape[1])
            c_ub = []
            t_c += run_window(L, torch, c, c_stats, cevery, cs, tag, None, c_ub)
            dc = c.diagnostics()
        return cs.result(), c_ub, dc, t_c

    # ---- a-posteriori refinement of the first network: its coarse run's
    # resolved shear stress and the filtered fine profile give, through the
    # mean momentum balance, the eddy viscosity per row that the coarse grid
    # lacks; every training sample of that row takes it as the target of the
    # off-diagonal groups named by --refine-groups (the others 0), and a
    # network is trained on them
    out["refine"] = []
    if args.refine > 0 and not args.load_params:
        cy = cshape[1]
        rows = torch.arange(X.shape[0], device="cuda") % nc // cshape[0] % cy
        nut_prev = None
        for it in range(args.refine):
            prof_c, c_ub, _, _ = coarse_run(cforms[0], nets[0], f"refine {it}")
            nut = balance_eddy_viscosity(prof_c, filt, ut, nu_f / 2, cap=4.0 * nu_f / 2)
            if nut_prev is not None:
                nut = args.refine_relax * nut + (1.0 - args.refine_relax) * nut_prev
            nut_prev = nut
            err = float(np.sqrt(np.sum((prof_c["U"] - filt["U"]) ** 2) / np.sum(filt["U"] ** 2)))
            log(f"refine {it}: U rel L2 of the run {err:.4f}, U_b/u_tau {np.mean(c_ub) / ut:.3f}; "
                f"target nu_t / nu_c by row {np.round(nut[: cy // 2] / (nu_f / 2), 3).tolist()}")
            Yr = torch.zeros_like(Y)
            tn = torch.tensor(nut, dtype=torch.float32, device="cuda")[rows]
            for j, grp in enumerate(("110", "101", "011")):
                if grp in args.refine_groups.split(","):
                    Yr[:, j] = tn
            m = L.MLP(seed=11)
            m.fit_normalisation(X.data_ptr(), Yr.data_ptr(), ntr)
            hist = m.train(X.data_ptr(), Yr.data_ptr(), ntr, args.batch, args.train_steps, args.lr, 5)
            l1, _ = m.loss_grad(X.data_ptr(), Yr.data_ptr(), ntr)
            nets[0] = m.export()
            m.close()
            out["refine"].append({"pass": it, "run_rel_l2_U": err, "run_u_bulk_over_u_tau": float(np.mean(c_ub) / ut),
                                  "target_nu_t_over_nu_c": [round(float(v), 4) for v in nut / (nu_f / 2)],
                                  "loss_after": l1})
    # ---- output gain of the first network: on the training start, the scale g
    # that brings the coarse run's bulk velocity to the filtered fine run's,
    # interpolated linearly between the plain run (g = 0) and the network (g = 1)
    out["calibration"] = None
    if args.calibrate and not args.load_params:
        _, ub0, _, _ = coarse_run(cforms[0], None, "calibrate g=0")
        _, ub1, _, _ = coarse_run(cforms[0], nets[0], "calibrate g=1")
        u0, u1, uf = float(np.mean(ub0)), float(np.mean(ub1)), float(np.mean(f_ub))
        g = output_gain(u0, u1, uf)
        nets[0] = scaled_output(nets[0], g)
        out["calibration"] = {"gain": g, "u_bulk_over_u_tau_plain": u0 / ut, "u_bulk_over_u_tau_g1": u1 / ut,
                              "u_bulk_over_u_tau_fine": uf / ut}
        log(f"calibration: U_b/u_tau plain {u0 / ut:.3f}, network {u1 / ut:.3f}, fine {uf / ut:.3f} -> gain {g:.3f}")
    np.save(args.save_params, scaled_output(nets[0], gains[0]))
    del X, Y, xs, ys
    res = {}
    runs = []
    for st in cforms:
        pre = "" if len(cforms) == 1 else f"{st}_"
        runs += [(pre + "plain", st, None)]
        runs += [(f"{pre}closure_s{k}_g{g:g}", st, scaled_output(p, g)) for g in gains for k, p in enumerate(nets)]
    for name, st, p in runs:
        pr, c_ub, dc, t_c = coarse_run(st, p, f"coarse {name}")
        res[name] = {"wall_s": t_c, "steps": c_settle + c_stats, "stats_steps": c_stats,
                     "u_tau_end": friction_velocity(dc, cshape[0], cshape[2]),
                     "u_bulk_over_u_tau": float(np.mean(c_ub) / ut), "u_bulk_std_over_u_tau": float(np.std(c_ub) / ut),
                     "profile": pr}
    ub_f = out["fine"]["u_bulk_over_u_tau"]
    for name in res:
        pr = res[name].pop("profile")
        res[name]["u_bulk_rel_err_vs_fine"] = abs(res[name]["u_bulk_over_u_tau"] - ub_f) / ub_f
        res[name]["rel_l2_U_vs_filtered_fine"] = float(np.sqrt(np.sum((pr["U"] - filt["U"]) ** 2) /
                                                               np.sum(filt["U"] ** 2)))
        for q in ("u_rms", "v_rms", "w_rms"):
            res[name][f"rel_l2_{q}_vs_filtered_fine"] = float(np.sqrt(np.sum((pr[q] - filt[q]) ** 2) /
                                                                      np.sum(filt[q] ** 2)))
        res[name]["U_over_u_tau"] = [round(float(v) / ut, 4) for v in pr["U"][: cshape[1] // 2]]
        log(f"coarse {name}: U_b/u_tau {res[name]['u_bulk_over_u_tau']:.3f} (fine {ub_f:.3f}), "
            f"U rel L2 {res[name]['rel_l2_U_vs_filtered_fine']:.4f}, "
            f"u_rms {res[name]['rel_l2_u_rms_vs_filtered_fine']:.4f}, v_rms {res[name]['rel_l2_v_rms_vs_filtered_fine']:.4f}")
    summary = {}
    for st in cforms:
        pre = "" if len(cforms) == 1 else f"{st}_"
        for g in gains:
            names = [f"{pre}closure_s{k}_g{g:g}" for k in range(len(nets))]
            key = f"{pre}gain {g:g}"
            summary[key] = {q: [float(np.mean([res[n][q] for n in names])), float(np.std([res[n][q] for n in names]))]
                            for q in ("u_bulk_over_u_tau", "u_bulk_rel_err_vs_fine", "rel_l2_U_vs_filtered_fine",
                                      "rel_l2_u_rms_vs_filtered_fine", "rel_l2_v_rms_vs_filtered_fine",
                                      "rel_l2_w_rms_vs_filtered_fine")}
            log(f"{key} over {len(nets)} networks (mean, std): {summary[key]}")
    out["coarse"] = res
    out["closure_summary"] = summary
    out["coarse_start_after_fine_steps"] = n_trans
    out["filtered_fine_U_over_u_tau"] = [round(float(v) / ut, 4) for v in filt["U"][: cshape[1] // 2]]
    out["filtered_fine_rms_over_u_tau"] = {q: [round(float(v) / ut, 4) for v in filt[q][: cshape[1] // 2]]
                                           for q in ("u_rms", "v_rms", "w_rms")}
    print(json.dumps(out), flush=True)
    return out


if __name__ == "__main__":
    main()
