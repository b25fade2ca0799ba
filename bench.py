#!/usr/bin/env python3
"""Throughput of the spectral-multigrid Poisson path on one MI355X.

One step = one full solve (azimuthal FFT -> multigrid solve 1 -> screening
mass + DGF convolution -> multigrid solve 2 -> inverse FFT) of the workload's
density from a zero initial guess, to relative residual --tol (default 1e-8)
on every mode.  The DGF tables, the launch-shape tuning and the plan setup
are done before the timed region (one-time, as in the paper).  The timed
form is the chosen one (FP32/FP64 iterative refinement, per-mode cycle
schedules replayed as HIP graphs, autotuned launch shapes, smoothing steps
chosen at setup); the plain GPU form (FP64, host reads after every V-cycle,
V(2,2)) is timed next to it.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2] [--form chosen|plain]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# chosen form: coarsening stops at a level of at most this many cells, solved
# exactly by fast diagonalisation (the plain form keeps the 128-cell default)
COARSE_CELLS = 2048


def measured_traffic(workload, kernel_class):
    """HBM bytes per launch of `kernel_class` from the committed PMC
    summary (profiles/hbm_traffic.txt), or None when there is none or the
    kernel's source has changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        w, k, src, h, val = line.split()[:5]
        if w != workload or k != kernel_class:
            continue
        with open(os.path.join(ROOT, src), "rb") as f:
            if hashlib.sha1(f.read()).hexdigest()[:12] != h:
                return None
        return float(val)
    return None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(workload, tol, budget_s):
    """The CPU oracle (plain FP64 numpy/scipy, single-threaded) timed on a
    bounded sample of the same workload: full solves with the per-mode LU
    factors cached after a first solve; the DGF tables are replaced by zeros
    of the same shape (the boundary convolution costs the same; DGF setup is
    excluded like the GPU's)."""
    import numpy as np

    from oracle.geometry import GridSpec, cell_centres
    from oracle.james import GhostSet
    from oracle.solve import OraclePlan
    from workloads import configs

    g = configs.GRIDS[workload]
    spec = GridSpec(**g)
    a, b, p = cell_centres(spec)
    rho = configs.density(workload, a, b, p)
    ng = GhostSet(spec).n
    plan = OraclePlan(spec, dgf=np.zeros((spec.n_modes, ng, ng)))
    t0 = time.perf_counter()
    plan.solve(rho)                       # factorises every mode once
    t_first = time.perf_counter() - t0
    n, t0 = 0, time.perf_counter()
    while True:
        plan.solve(rho)
        n += 1
        el = time.perf_counter() - t0
        if el > budget_s or n >= 50:
            break
    return dict(value=n / el, unit="solves/s", cores=1, kind="oracle",
                sample=f"{n} full oracle solves of {workload} (direct per-mode LU, factors cached; "
                       f"first solve incl. factorisation {t_first:.2f}s; DGF zeros, setup excluded)")


def _plan(smg, g, form, line_solver, max_cycles=60):
    """The chosen form (mixed precision, scheduled graph replay, autotuned
    launch shapes, smoothing steps chosen at setup: V(1,1) when the finest
    level is smoothed by whole-grid launches, else V(2,2)) or the plain GPU
    form (FP64, host reads after every V-cycle, built-in launch shapes, the
    paper's SOR line smoother, V(2,2))."""
    if form == "chosen":
        return smg.Plan(**g, precision="mixed", launch="graph", autotune=True, line_solver=line_solver,
                        max_cycles=max_cycles, coarse_cells=COARSE_CELLS, nu_pre=smg.NU_AUTO, nu_post=smg.NU_AUTO)
    return smg.Plan(**g, precision="fp64", launch="dynamic", autotune=False, line_solver="sor", max_cycles=max_cycles)


def _timed(plan, rho, phi, steps, tol, torch):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.solve_nosync(rho, phi, tol=tol)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def bench_accel(args, smg, configs, torch):
    """The step after the solve: g = -grad Phi on every face of the workload's
    grid (one smg_acceleration call per step, the potential and Theta of one
    chosen-form solve resident in HBM)."""
    wl = "c5" if args.workload == "c5-snapshot" else args.workload
    g = configs.GRIDS[wl]
    log(f"face acceleration on the {args.workload} grid")
    plan = _plan(smg, g, "chosen", args.line_solver).setup("cuda:0")
    a, b, p, _ = plan.geometry()
    rho = torch.from_numpy(configs.density(wl, a, b, p)).to("cuda:0")
    phi, info = plan.solve(rho, tol=args.tol)
    out = plan.acceleration(phi)
    for _ in range(args.warmup):
        plan.acceleration(phi, out=out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        plan.acceleration(phi, out=out)
    e1.record()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    ms = e0.elapsed_time(e1) / args.steps
    na, nb, nph = g["n_a"], g["n_b"], g["n_phi"]
    cells = na * nb * nph
    # read phi once, write the three face arrays once, read the ghost potential
    algo = 8.0 * (cells + (na + 1) * nb * nph + na * (nb + 1) * nph + cells + plan.n_ghost * nph)
    achieved = algo / (ms * 1e-3) / 1e9
    print(json.dumps({
        "metric": "face acceleration fields/s", "value": round(args.steps / dt, 2), "unit": "fields/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * dt / args.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{args.workload}: g = -grad Phi on all faces of the solved potential",
                   "cells": cells, "ghosts": plan.n_ghost},
        "roofline": {"bound": "hbm", "kernel": "face_acceleration (ghost c2r + face kernel)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "avg_launch_us": round(1e3 * ms, 3), "bytes_per_launch": round(algo)},
    }), flush=True)


def bench_batch(args, smg, configs, torch):
    """The 16-problem batch: one batched solve of all problems per step
    (chosen form) against the plain GPU form solving them one by one."""
    grids = configs.c4_grids()
    log(f"workload c4: {configs.DESCRIPTION['c4']}")
    t0 = time.perf_counter()
    plans = [_plan(smg, g, "chosen", args.line_solver, 200).setup("cuda:0") for g in grids]
    batch = smg.Batch(plans).setup("cuda:0")
    torch.cuda.synchronize()
    log(f"setup of {len(plans)} plans + batch {time.perf_counter() - t0:.1f}s; "
        f"{sum(p.n_modes for p in plans)} mode planes")
    rhos, phis = [], []
    for q, (g, p) in enumerate(zip(grids, plans)):
        a, b, ph, _ = p.geometry()
        rhos.append(torch.from_numpy(configs.c4_density(q, g, a, b, ph)).to("cuda:0"))
        phis.append(torch.empty_like(rhos[-1]))
    for _ in range(max(args.warmup, 2)):
        batch.solve(rhos, tol=args.tol, outs=phis, info=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        batch.solve(rhos, tol=args.tol, outs=phis, info=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    n = len(plans)
    value = n * args.steps / dt
    _, infos = batch.solve(rhos, tol=args.tol, outs=phis, timings=True)
    log(f"batched: {value:.2f} solves/s ({1e3 * dt / args.steps:.2f} ms per batch of {n})")
    out = {
        "metric": "Poisson solves/s at rel. residual 1e-8",
        "value": round(value, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * dt / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"c4: {configs.DESCRIPTION['c4']}", "tol": args.tol, "form": "chosen, one batch",
                   "line_solver": args.line_solver,
                   "problems": n, "step": "one batched solve of all problems",
                   "v_cycles_per_step": int(sum(i["total_cycles"] for i in infos)),
                   "converged": all(i["converged"] for i in infos)},
        "roofline": None,
    }
    if not args.no_plain:
        plain = [_plan(smg, g, "plain", args.line_solver, 200).setup("cuda:0") for g in grids]
        for _ in range(max(args.warmup, 2)):
            for p, r, o in zip(plain, rhos, phis):
                p.solve_nosync(r, o, tol=args.tol)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            for p, r, o in zip(plain, rhos, phis):
                p.solve_nosync(r, o, tol=args.tol)
        torch.cuda.synchronize()
        dtp = time.perf_counter() - t0
        out["plain_gpu"] = dict(value=round(n * args.steps / dtp, 3), unit="solves/s",
                                ms_per_step=round(1e3 * dtp / args.steps, 3),
                                form="FP64, problems one after another, host reads after every V-cycle")
        out["speedup_vs_plain"] = round(dtp / dt, 3)
        log(f"plain GPU form: {n * args.steps / dtp:.2f} solves/s")
    print(json.dumps(out), flush=True)


def bench_learned(args, smg, configs, torch):
    """The orbiting-blob trajectory (64 snapshots, 256x128x256 log sphere):
    warm-started solves with the learned guess of modes 0..4 (the network
    trained at setup on 8 method-generated trajectories, seeds 50-57) vs
    the previous step's solution as the guess, and the plain GPU form."""
    import numpy as np

    from paper_2606_17636_amd import learn
    from workloads.densities import keplerian_snapshot_device
    from workloads.netinit import init_params

    g = configs.GRIDS["c5"]
    m_max, n_snap = 4, 64
    log(f"workload c5: {configs.DESCRIPTION['c5']}")
    dt = configs.keplerian_dt()
    t0 = time.perf_counter()
    plan = _plan(smg, g, "chosen", args.line_solver).setup("cuda:0")
    a, b, ph, _ = plan.geometry()
    net = smg.Net()
    net.set_params(init_params(0))
    plan.attach_net(net, m_max)
    log(f"setup (tables + DGF + tuning) {time.perf_counter() - t0:.1f}s")

    def traj(seed, steps):
        blobs = configs.c5_blobs(seed)
        return (keplerian_snapshot_device(a, b, ph, blobs, k * dt) for k in range(steps))

    t0 = time.perf_counter()
    seeds = list(range(50, 50 + args.train_traj))
    cap = len(seeds) * (n_snap - 1) * learn.samples_per_step(m_max)
    buf = learn.sample_buffer(plan, cap)
    n, _ = learn.record_trajectories(plan, [traj(s, n_snap) for s in seeds], args.tol, buf, cap)
    log(f"recorded {n} samples from {len(seeds)} trajectories in {time.perf_counter() - t0:.1f}s")
    t0 = time.perf_counter()
    losses = learn.train(net, buf, n, g["n_a"], g["n_b"], steps=args.train_steps, batch=16, lr=1e-3, seed=1,
                         log_every=max(1, args.train_steps // 5), log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    log(f"trained {args.train_steps} steps in {t_train:.1f}s")
    del buf
    torch.cuda.empty_cache()

    rhos = list(traj(5, n_snap))
    phi = torch.empty_like(rhos[0])

    taken = [0]

    def run(pl, use_net, with_info):
        cyc = []
        torch.cuda.synchronize()
        t = time.perf_counter()
        for k, r in enumerate(rhos):
            if with_info:
                _, info = pl.solve(r, tol=args.tol, warm=k > 0, out=phi, net=use_net)
                cyc.append(learn.low_mode_cycles(info, m_max) if k >= 2 else 0)
                if use_net and k >= 2:
                    taken[0] += int(pl.net_used().sum())
            else:
                pl.solve_nosync(r, phi, tol=args.tol, warm=k > 0, net=use_net)
        torch.cuda.synchronize()
        return time.perf_counter() - t, cyc

    # cycle counts (info pass), then the timed passes
    _, cyc_net = run(plan, True, True)
    _, cyc_prev = run(plan, False, True)
    for _ in range(max(args.warmup, 1)):
        run(plan, True, False)
    dt_net, _ = run(plan, True, False)
    dt_prev, _ = run(plan, False, False)
    zero = []
    for r in rhos[:8]:
        _, info = plan.solve(r, tol=args.tol, out=phi)
        zero.append(learn.low_mode_cycles(info, m_max))
    value = n_snap / dt_net
    out = {
        "metric": "Poisson solves/s at rel. residual 1e-8",
        "value": round(value, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": n_snap,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * dt_net / n_snap, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"c5: {configs.DESCRIPTION['c5']}", "tol": args.tol,
                   "form": "chosen + learned guess of modes 0..4", "step": "one warm-started solve of the 64-snapshot trajectory",
                   "train": {"trajectories": len(seeds), "samples": n, "steps": args.train_steps,
                             "loss_first": float(np.mean(losses[:10])), "loss_last": float(np.mean(losses[-20:])),
                             "seconds": round(t_train, 1)},
                   "low_mode_v_cycles_per_step": {"zero_guess": round(float(np.mean(zero)), 2),
                                                  "previous_step": round(float(np.sum(cyc_prev)) / (n_snap - 2), 2),
                                                  "network": round(float(np.sum(cyc_net)) / (n_snap - 2), 2)},
                   "network_guess_taken": f"{taken[0]} of {2 * (m_max + 1) * (n_snap - 2)} mode solves",
                   "previous_step_guess_solves_per_s": round(n_snap / dt_prev, 3)},
        "roofline": None,
    }
    if not args.no_plain:
        pl = _plan(smg, g, "plain", args.line_solver).setup("cuda:0")
        run(pl, False, False)
        dtp, _ = run(pl, False, False)
        out["plain_gpu"] = dict(value=round(n_snap / dtp, 3), unit="solves/s", ms_per_step=round(1e3 * dtp / n_snap, 3),
                                form="FP64, previous-step warm start, host reads after every V-cycle, no graph, no network")
        out["speedup_vs_plain"] = round(dtp / dt_net, 3)
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--form", default="chosen", choices=["chosen", "plain"])
    ap.add_argument("--line-solver", default="sor", choices=["sor", "exact"])
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-GPU comparison leg")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--train-traj", type=int, default=8, help="c5: training trajectories")
    ap.add_argument("--train-steps", type=int, default=2000, help="c5: Adam steps")
    ap.add_argument("--part", default="solve", choices=["solve", "accel"],
                    help="accel: time the face acceleration of the solved potential instead of the solve")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy 5 times (the HBM-counter calibration kernel)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        src = torch.ones(32 << 20, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 8, "copy_bytes_written": dst.numel() * 8}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (asked for --gpus {args.gpus}); the path would shard "
              "by Fourier mode across GPUs, which is not built here.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2606_17636_amd import smg
    from workloads import configs

    if args.part == "accel":
        return bench_accel(args, smg, configs, torch)
    if args.workload == "c4":
        return bench_batch(args, smg, configs, torch)
    if args.workload == "c5":
        return bench_learned(args, smg, configs, torch)
    # c5-snapshot: one snapshot (t = 0) of the orbiting workload, cold solves
    wl = "c5" if args.workload == "c5-snapshot" else args.workload
    desc = configs.DESCRIPTION[wl] + (", snapshot t=0, zero initial guess" if wl != args.workload else "")
    g = configs.GRIDS[wl]
    log(f"workload {args.workload}: {desc}")
    plan = _plan(smg, g, args.form, args.line_solver)
    t0 = time.perf_counter()
    plan.setup("cuda:0")
    torch.cuda.synchronize()
    log(f"setup (tables + DGF + tuning) {time.perf_counter() - t0:.2f}s, levels {plan.level_shapes}, "
        f"ghosts {plan.n_ghost}")
    if plan.tune_report():
        log("autotune: " + " | ".join(l for l in plan.tune_report().splitlines() if l.startswith("planes <=")))
    a, b, p, _ = plan.geometry()
    rho = torch.from_numpy(configs.density(wl, a, b, p)).to("cuda:0")
    phi = torch.empty_like(rho)
    for _ in range(max(args.warmup, 2)):   # the first solve of a kind runs the host loop and fixes the schedule
        plan.solve_nosync(rho, phi, tol=args.tol)
    torch.cuda.synchronize()
    log(f"warmup {max(args.warmup, 2)} done")

    dt = _timed(plan, rho, phi, args.steps, args.tol, torch)
    value = args.steps / dt
    log(f"timed {args.steps} solves in {dt:.3f}s -> {value:.2f} solves/s ({args.form})")

    # per-kernel launch durations: the same solves again, the scheduled
    # launches of the timed replay enqueued from the host instead of the
    # graph, with HIP events on the solve stream: smoother launches record
    # their own start and stop, the other kernels have an event before and
    # after them
    plan.profile_begin()
    _timed(plan, rho, phi, args.steps, args.tol, torch)
    stats = plan.profile_end()
    _, info = plan.solve(rho, tol=args.tol, timings=True)
    cyc = info["total_cycles"]
    name, st = max(stats.items(), key=lambda kv: kv[1]["total_ms"])
    achieved = st["bytes"] / (st["total_ms"] * 1e-3) / 1e9
    roofline = dict(bound="hbm", kernel=name, achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=measured_traffic(args.workload, name),
                    avg_launch_us=round(1e3 * st["total_ms"] / st["launches"], 3),
                    bytes_per_launch=round(st["bytes"] / st["launches"]))
    kern = {k: dict(launches=v["launches"] // args.steps, ms=round(v["total_ms"] / args.steps, 4),
                    gbs=round(v["bytes"] / max(v["total_ms"], 1e-9) / 1e6, 1)) for k, v in stats.items()}
    out = {
        "metric": "Poisson solves/s at rel. residual 1e-8",
        "value": round(value, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * dt / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if args.form == "chosen" else "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {desc}", "tol": args.tol,
                   "form": args.form, "line_solver": args.line_solver, "initial_guess": "zero",
                   "v_cycles_per_solve": cyc,
                   "v_cycles_m0": [int(info["cycles1"][0]), int(info["cycles2"][0])],
                   "component_ms": {k: round(info[k], 3) for k in ("ms_fft", "ms_mg1", "ms_james", "ms_mg2", "ms_ifft")}},
        "roofline": roofline,
        "kernels_per_step": kern,
    }
    if args.form == "chosen" and not args.no_plain:
        pl = _plan(smg, g, "plain", args.line_solver).setup("cuda:0")
        for _ in range(max(args.warmup, 2)):
            pl.solve_nosync(rho, phi, tol=args.tol)
        dtp = _timed(pl, rho, phi, args.steps, args.tol, torch)
        out["plain_gpu"] = dict(value=round(args.steps / dtp, 3), unit="solves/s",
                                ms_per_step=round(1e3 * dtp / args.steps, 3),
                                form="FP64, host reads after every V-cycle, built-in launch shapes, no graph")
        out["speedup_vs_plain"] = round(dtp / dt, 3)
        log(f"plain GPU form: {args.steps / dtp:.2f} solves/s")
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(wl, args.tol, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
