#!/usr/bin/env python
"""Throughput of the fractional PP-WCNS-IS step on one MI355X.

A step is one SSP-RK3 step of the fractional algorithm: wavespeed and time
step from W^n, three stages of the five-equation hyperbolic operator, each
followed by the infinite-rate thermal relaxation.  Workload: the 2D shock on a
liquid column with a gas bubble (three species, 1024 x 512 cells, FP64).

Prints one JSON line.  Inputs are resident in HBM before the timed region.
`roofline` describes the dominant kernel (the y-direction sweep, which also
applies the stage update and the relaxation), timed live with HIP events on
the stream it runs on.  `cpu_baseline` times the CPU oracle on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

METRIC = ("cell-updates/s per RK3 step (plain FP64 vs FP32 vs learned) at stated L1 error; HBM GB/s")
PEAK_FP64_TFLOPS = 78.6   # MI355X FP64 vector, dense
PEAK_HBM_GBS = 8000.0     # MI355X HBM3E


def node_flops(N, D):
    """Primitive state of one node (hot-path step a1)."""
    return 8 * N + 3 * D + 7


def face_flops(N, D):
    """Algorithmic FP64 operations of one midpoint (add, sub, mul, div, sqrt,
    tanh count one each; comparisons, min/max and |x| count zero; limiter
    branches that fire only on bad faces count zero): two HLLC solves, the
    projection set-up and the characteristic values of six nodes, 2M WENO-IS
    interpolations of 105 each, the back-projection, the always-executed part
    of the interpolation limiter, two face states, the HCS flux and the
    sensor, each counted by hand from the formulas."""
    M = 2 * N + D
    return 253 * M + 141 * N + 56 * D + 251


def cell_flops(N, D, final):
    """Flux difference per direction; stage update and relaxation in the last one."""
    M = 2 * N + D
    f = 2 * M + (M if D > 1 else 0)
    if final:
        f += 4 * M + (12 * N + 2 * D + 25)
    return f


def sweep_flops(N, D, n, direction, final):
    """Algorithmic FP64 operations of one launch of the sweep in `direction`."""
    cells = 1
    for k in n:
        cells *= k
    faces = cells // n[direction] * (n[direction] + 1)
    return faces * face_flops(N, D) + cells * (node_flops(N, D) + cell_flops(N, D, final))


def wavespeed_flops(N, D):
    """|u_d| + c of one cell for the time step (Sec. 4.1.2): its primitive
    state and one addition per direction."""
    return node_flops(N, D) + D


def mean_launch_flops(N, D, n, direction):
    """Algorithmic FP64 operations per launch of the sweep in `direction`,
    averaged over its three launches of an RK3 step: the last direction's
    third launch also takes |u_d| + c of every cell it writes, for the next
    step's time step."""
    cells = 1
    for k in n:
        cells *= k
    f = sweep_flops(N, D, n, direction, final=(direction == D - 1))
    if direction == D - 1:
        f += cells * wavespeed_flops(N, D) / 3.0
    return f


COUNTERS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                        "k_sweep_liquid_column_1024x512_fp64_counters.json")


def kernel_source_hash() -> str:
    """sha256 over the library's kernel sources (name, then contents, sorted)."""
    import glob
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2208_04488_amd", "csrc")
    for f in sorted(glob.glob(os.path.join(csrc, "*.hip")) + glob.glob(os.path.join(csrc, "*.hpp"))):
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by the copy calibration), or
    None if the summary is missing, is for another kernel, or was taken on
    other kernel sources than the ones built here."""
    try:
        with open(COUNTERS) as f:
            c = json.load(f)
    except (OSError, ValueError):
        return None
    if c.get("kernel") != kernel or c.get("source_sha256") != kernel_source_hash():
        return None
    cal = c["calibration"]
    return 1024.0 * (c["fetch_kib_per_dispatch"] * cal["fetch_factor"] +
                     c["write_kib_per_dispatch"] * cal["write_factor"])


def algorithmic_bytes_per_cell_step(M):
    """Stage 1 reads W^n, writes W1; stages 2, 3 read W^(s) and W^n, write the
    next state: 8 M doubles per cell per RK3 step."""
    return 64 * M


def batch_flops_per_step(batch):
    """Algorithmic FP64 operations of one SSP-RK3 step of the whole ensemble:
    per problem of n cells, the wavespeed pass (n nodes) and three stages of
    n + 1 faces, n staged nodes and n final cell updates (1D, transmissive)."""
    import numpy as np
    N = batch.N
    n = np.diff(batch.offsets).astype(np.float64)
    per = n * node_flops(N, 1) + 3 * ((n + 1) * face_flops(N, 1) + n * (node_flops(N, 1) + cell_flops(N, 1, True)))
    return float(per.sum())


def bench_batch(args):
    """Ensemble of 4096 1D two-phase Riemann problems (200-2000 cells): one
    persistent launch per `steps_per_launch` steps, launch shape from the
    autotuner; FP32 face arithmetic (the ensemble's stated precision) and the
    FP64 path over the same number of steps for the speedup and L1 error."""
    import numpy as np
    import torch
    from paper_2208_04488_amd import autotune, hrm
    from paper_2208_04488_amd import inputs as I

    batch = I.config4()
    steps = args.batch_steps
    stream = torch.cuda.current_stream()
    res = {}
    for name, prec in (("fp32", hrm.FP32), ("fp64", hrm.FP64)):
        best = autotune.tune_batch(batch, precision=prec, use_cache=False)
        k = best["steps_per_launch"]
        nsteps = max(steps // k, 1) * k
        s = hrm.BatchSolver(batch, precision=prec)
        s.configure(best["threads"], best["blocks"], k)
        s.run(k)  # captures the graph; these warm-up steps count in the state
        torch.cuda.synchronize()
        s.W.copy_(torch.from_numpy(batch.W))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        s.run(nsteps)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        d = s.diagnostics()
        res[name] = dict(ms=ms, steps=nsteps, W=s.state(), shape=best, relax_bad=d["relax_bad"],
                         launches=nsteps // k)
        s.close()
    N = batch.N
    r32, r64 = res["fp32"]["W"][:N].sum(axis=0), res["fp64"]["W"][:N].sum(axis=0)
    l1 = float(np.abs(r32 - r64).sum() / np.abs(r64).sum())
    flops = batch_flops_per_step(batch)
    out = {"workload": f"{batch.nprob} independent 1D two-phase Riemann problems, {int(np.diff(batch.offsets).min())}"
                       f"-{int(np.diff(batch.offsets).max())} cells ({batch.ncell} in total), transmissive, CFL 0.4",
           "steps": res["fp32"]["steps"]}
    for name in ("fp32", "fp64"):
        r = res[name]
        cups = batch.ncell * r["steps"] / (r["ms"] * 1e-3)
        out[name] = {"value": cups, "unit": "cell-updates/s", "ms_per_step": r["ms"] / r["steps"],
                     "launch_shape": {k: r["shape"][k] for k in ("threads", "blocks", "steps_per_launch")},
                     "ms_per_launch": r["ms"] / r["launches"],
                     "achieved_tflops_algorithmic": flops * r["steps"] / (r["ms"] * 1e-3) / 1e12,
                     "relax_bad": r["relax_bad"]}
    out["fp32"]["speedup_vs_fp64"] = out["fp32"]["value"] / out["fp64"]["value"]
    out["fp32"]["l1_rel_rho_vs_fp64"] = l1
    return out


MLP_FLOPS_PER_STENCIL = 2 * (5 * 32 + 32 * 32 + 32 * 3)  # algorithmic multiply-adds x 2


def bench_learned(args):
    """Learned interpolation weights against the plain method on the planar
    config-1 shock tube at 2048 x 1024 (FP64 state; the network in bfloat16
    on the matrix cores).  The network is trained first, on the GPU, from a
    fine ensemble of Riemann problems (untimed)."""
    import numpy as np
    import torch
    from paper_2208_04488_amd import hrm, learned
    from paper_2208_04488_amd import inputs as I

    t0 = time.perf_counter()
    fine = learned.fine_ensemble(nprob=1024, nmin=100, nmax=1000, seed=4001)
    X, T = learned.training_data(fine, snapshots=(40, 120))
    p0 = learned.init_params(0, last_scale=0.0)
    loss0 = learned.mean_loss(p0, X, T)
    params, _ = learned.train(X, T, steps=3000, count=16384, lr=2e-3, seed=0)
    loss1 = learned.mean_loss(params, X, T)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    npairs = X.shape[0]
    del X, T

    prob = I.config5(args.learned_nx, args.learned_ny)
    N, D, M = prob.N, prob.D, prob.M
    stream = torch.cuda.current_stream()
    res = {}
    for name, mlp in (("plain", None), ("learned", params)):
        s = hrm.Solver(prob, flags=hrm.FUSE_RELAX, mlp=mlp)
        s.advance(args.warmup, cfl=prob.cfl)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        s.advance(args.learned_steps, cfl=prob.cfl)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        hrm.hrm_set_timing(s.ctx, (1 << 0) | (1 << 1))
        hrm.hrm_get_timing(s.ctx)
        s.advance(5, cfl=prob.cfl)
        tm = hrm.hrm_get_timing(s.ctx)
        hrm.hrm_set_timing(s.ctx, 0)
        d = s.diagnostics()
        res[name] = dict(ms=ms, W=s.state(), relax_bad=d["relax_bad"],
                         sweep_ms={k: tm[k][0] / max(tm[k][1], 1) for k in ("sweep_x", "sweep_y")})
        s.close()
    nx, ny = prob.n[0], prob.n[1]
    faces = (nx + 1) * ny + nx * (ny + 1)
    cells = nx * ny
    steps = args.warmup + args.learned_steps
    out = {"workload": f"planar config-1 shock tube (liquid 1e9 Pa | air 1e5 Pa), {nx}x{ny} cells, 2 species, "
                       f"transmissive x / periodic y, CFL 0.4",
           "training": {"pairs": npairs, "adam_steps": 3000, "minibatch": 16384, "seconds": train_s,
                        "loss_classical_weights": loss0, "loss_trained": loss1,
                        "data": "1024 fine Riemann problems (200-2000 cells) after 40 and 120 FP64 steps"}}
    for name in ("plain", "learned"):
        r = res[name]
        out[name] = {"value": cells * args.learned_steps / (r["ms"] * 1e-3), "unit": "cell-updates/s",
                     "ms_per_step": r["ms"] / args.learned_steps, "sweep_ms_per_launch": r["sweep_ms"],
                     "relax_bad": r["relax_bad"]}
    out["learned"]["speedup_vs_plain"] = out["learned"]["value"] / out["plain"]["value"]
    rp, rl = res["plain"]["W"][:N].sum(axis=0), res["learned"]["W"][:N].sum(axis=0)
    out["learned"]["l1_rel_rho_vs_plain"] = float(np.abs(rl - rp).sum() / np.abs(rp).sum())
    out["learned"]["after_steps"] = steps
    # matrix-core work of the network: 2 M stencils per face, faces of both sweeps, 3 stages
    mf = 3 * faces * 2 * M * MLP_FLOPS_PER_STENCIL
    out["learned"]["mfma_tflops_algorithmic"] = mf / (out["learned"]["ms_per_step"] * 1e-3) / 1e12
    out["learned"]["mfma_frac_of_bf16_peak"] = out["learned"]["mfma_tflops_algorithmic"] / 2500.0
    return out


def bench_3d(args):
    """The 3D multimode workload (256^3, three species, periodic in y and z):
    FP64 and FP32 face arithmetic, K steps each from the initial condition."""
    import numpy as np
    import torch
    from paper_2208_04488_amd import hrm
    from paper_2208_04488_amd import inputs as I

    prob = I.config3(args.n3d)
    N, D, M = prob.N, prob.D, prob.M
    stream = torch.cuda.current_stream()
    res = {}
    for name, prec in (("fp64", hrm.FP64), ("fp32", hrm.FP32)):
        s = hrm.Solver(prob, flags=hrm.FUSE_RELAX, precision=prec)
        s.step(cfl=prob.cfl)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        s.advance(args.steps3d, cfl=prob.cfl)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        hrm.hrm_set_timing(s.ctx, 0b111)
        hrm.hrm_get_timing(s.ctx)
        s.advance(1, cfl=prob.cfl)
        tm = hrm.hrm_get_timing(s.ctx)
        hrm.hrm_set_timing(s.ctx, 0)
        d = s.diagnostics()
        rho = s.state()[:N].sum(axis=0)
        res[name] = dict(ms=ms, rho=rho, relax_bad=d["relax_bad"], tm=tm)
        s.close()
        del s
    out = {"workload": f"3D multimode interface, Mach-1.5 shock, 10% liquid droplets, 3 species, "
                       f"{prob.n[0]}^3 cells, periodic y/z, CFL 0.4", "steps": args.steps3d + 2}
    for name in ("fp64", "fp32"):
        r = res[name]
        out[name] = {"value": prob.ncell * args.steps3d / (r["ms"] * 1e-3), "unit": "cell-updates/s",
                     "ms_per_step": r["ms"] / args.steps3d, "relax_bad": r["relax_bad"],
                     "sweep_ms_per_launch": {k: r["tm"][k][0] / max(r["tm"][k][1], 1)
                                             for k in ("sweep_x", "sweep_y", "sweep_z")}}
    kx = max(("sweep_x", "sweep_y", "sweep_z"), key=lambda k: out["fp64"]["sweep_ms_per_launch"][k])
    kd = ("sweep_x", "sweep_y", "sweep_z").index(kx)
    fl = mean_launch_flops(N, D, prob.n, kd)
    out["fp64"]["dominant_kernel"] = f"k_sweep direction {kd}"
    out["fp64"]["achieved_tflops_algorithmic"] = fl / (out["fp64"]["sweep_ms_per_launch"][kx] * 1e-3) / 1e12
    out["fp64"]["hbm_gbs_algorithmic"] = algorithmic_bytes_per_cell_step(M) * out["fp64"]["value"] / 1e9
    out["fp32"]["speedup_vs_fp64"] = out["fp32"]["value"] / out["fp64"]["value"]
    r64, r32 = res["fp64"]["rho"], res["fp32"]["rho"]
    out["fp32"]["l1_rel_rho_vs_fp64"] = float(np.abs(r32 - r64).sum() / np.abs(r64).sum())
    return out


def measured_copy_gbs(nbytes=1 << 30, reps=5):
    """HBM bandwidth of a plain device-to-device copy of nbytes (read and
    written once each, 4x the 256 MB Infinity Cache), best of reps, from HIP
    events on the current stream: the reachable ceiling beside the 8 TB/s
    specification."""
    import torch
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    best = None
    stream = torch.cuda.current_stream()
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        b.copy_(a)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * nbytes / (best * 1e-3) / 1e9


def _oracle_rate(prob, budget_s, max_steps, mlp=None):
    import oracle
    o = oracle.from_problem(prob, mlp=mlp)
    W = prob.W
    t0 = time.perf_counter()
    steps = 0
    while steps < max_steps:
        W, _ = o.step(W, cfl=prob.cfl)
        steps += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    el = time.perf_counter() - t0
    return prob.ncell * steps / el, steps, el


def cpu_baseline(prob, budget_s=15.0, max_steps=200, others=True):
    """The oracle as it stands (C, FP64, OpenMP over grid lines) on the host
    cores: complete SSP-RK3 steps from the initial condition of the full
    benchmark workload, and shorter samples of the other workloads."""
    import oracle
    from paper_2208_04488_amd import inputs as I
    oracle.build(force=False)
    threads = oracle.Oracle.set_threads(0)
    rate, steps, el = _oracle_rate(prob, budget_s, max_steps)
    out = {"value": rate, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
           "sample": f"{steps} SSP-RK3 steps of the full {prob.n[0]}x{prob.n[1]} workload from its initial "
                     f"condition, OpenMP over grid lines, {el:.1f} s"}
    if others:
        more = {}
        for name, p in (("multimode_3d_128^3", I.config3(128)), ("planar_shock_tube_512x256", I.config5(512, 256)),
                        ("riemann_problem_1000_cells", I.config4(lengths=[1000]).problem(0))):
            r, k, e = _oracle_rate(p, 5.0, 50)
            more[name] = {"value": r, "steps": k, "seconds": e}
        out["other_workloads"] = more
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--nx", type=int, default=1024)
    ap.add_argument("--ny", type=int, default=512)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-steps", type=int, default=1000,
                    help="steps of the batched ensemble (0 skips it)")
    ap.add_argument("--learned-steps", type=int, default=100,
                    help="timed steps of the learned-weight comparison (0 skips it)")
    ap.add_argument("--learned-nx", type=int, default=2048)
    ap.add_argument("--steps3d", type=int, default=10, help="timed steps of the 3D workload (0 skips it)")
    ap.add_argument("--n3d", type=int, default=256)
    ap.add_argument("--learned-ny", type=int, default=1024)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 512 MiB device copy (reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (a sharded run would split the "
              "grid into slabs and exchange 3-cell halos every stage). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    if args.calibrate_copy:
        # 2 GiB per buffer: larger than the 256 MB Infinity Cache, so every
        # byte of the copy comes from and goes to HBM
        nbytes = 2 << 30
        a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 1.0, out=b)  # elementwise kernel: reads a, writes b
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "elementwise copy b = 1.0 * a", "bytes_read_per_launch": nbytes,
                          "bytes_written_per_launch": nbytes, "launches": 3}), flush=True)
        return
    from paper_2208_04488_amd import hrm
    from paper_2208_04488_amd import inputs as I

    prob = I.config2(args.nx, args.ny)
    N, D, M = prob.N, prob.D, prob.M
    s = hrm.Solver(prob, flags=hrm.FUSE_RELAX)
    stream = torch.cuda.current_stream()
    s.advance(args.warmup, cfl=prob.cfl)
    torch.cuda.synchronize()

    # timed region: K steps in one hrm_advance call (one pass over W^n for
    # the first time step, then K replays of the captured RK3 step graph)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev0.record(stream)
    s.advance(args.steps, cfl=prob.cfl)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_total = ev0.elapsed_time(ev1)
    ms_step = ms_total / args.steps
    w64_timed = s.state()

    # kernel durations: the same K steps with the library's HIP events around
    # every sweep launch on the same stream (direct launches, no graph)
    hrm.hrm_set_timing(s.ctx, (1 << 0) | (1 << 1) | (1 << 3))
    hrm.hrm_get_timing(s.ctx)  # clear
    s.advance(args.steps, cfl=prob.cfl)
    torch.cuda.synchronize()
    timers = hrm.hrm_get_timing(s.ctx)
    hrm.hrm_set_timing(s.ctx, 0)
    diag = s.diagnostics()

    # dominant kernel: the sweep with the larger total time
    kname = max(("sweep_x", "sweep_y"), key=lambda k: timers[k][0])
    kdir = 0 if kname == "sweep_x" else 1
    ms_launch = timers[kname][0] / max(timers[kname][1], 1)
    flops = mean_launch_flops(N, D, prob.n, kdir)
    achieved = flops / (ms_launch * 1e-3) / 1e12
    cups = prob.ncell * args.steps / (ms_total * 1e-3)
    # algorithmic bytes of that launch: W_s read, plus (last direction) W^n and
    # the RHS read and the stage output written; first direction writes the RHS
    final = kdir == D - 1
    if D == 1:
        narrays = 3       # W_s, W^n read; stage output written
    elif final:
        narrays = 4       # W_s, W^n, RHS read; stage output written
    elif kdir == 0:
        narrays = 2       # W_s read; RHS written
    else:
        narrays = 3       # W_s read; RHS read and written
    sweep_bytes = 8 * M * prob.ncell * narrays
    # both instantiations of that direction's sweep (with and without the
    # wavespeed epilogue), averaged over their launches as ms_launch is
    kname_full = f"k_sweep<{N},{D},{kdir},{16 if kdir else (64 if D > 1 else 256)}," \
                 f"{16 if kdir else (4 if D > 1 else 1)},double,0,*>"
    traffic = measured_traffic(kname_full)
    hbm = algorithmic_bytes_per_cell_step(M) * cups / 1e9

    out = {
        "metric": METRIC, "value": cups, "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"2D Mach-1.47 shock on a liquid column with a gas bubble, 3 species, "
                               f"{prob.n[0]}x{prob.n[1]} cells, FP64 PP-WCNS-IS + thermal relaxation, CFL 0.4",
                   "cells": prob.ncell, "species": N, "dim": D, "components": M},
        "roofline": {"bound": "alu", "kernel": f"k_sweep direction {kdir} (N={N}, D={D})",
                     "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS, "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "traffic_gbs": None if traffic is None else traffic / (ms_launch * 1e-3) / 1e9,
                     "algorithmic_bytes_per_launch": sweep_bytes,
                     "flops_per_launch": flops, "ms_per_launch": ms_launch},
        "hbm_gbs_algorithmic": hbm, "hbm_frac_algorithmic": hbm / PEAK_HBM_GBS,
        "hbm_copy_gbs_measured": measured_copy_gbs(),
        "kernel_ms_per_step": {k: v[0] / args.steps for k, v in timers.items() if v[1]},
        "wall_s_timed": wall,
        "positivity": {"relax_bad": diag["relax_bad"], "interp_hs": diag["interp_hs"],
                       "flux_hs": diag["flux_hs"]},
    }
    w64 = w64_timed
    s.close()

    # FP32 face arithmetic on the same workload: throughput and L1 error of
    # the mixture density after the same warm-up + timed steps
    s32 = hrm.Solver(prob, flags=hrm.FUSE_RELAX, precision=hrm.FP32)
    s32.advance(args.warmup, cfl=prob.cfl)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    s32.advance(args.steps, cfl=prob.cfl)
    e1.record(stream)
    torch.cuda.synchronize()
    ms32 = e0.elapsed_time(e1)
    w32 = s32.state()
    d32 = s32.diagnostics()
    s32.close()
    rho64, rho32 = w64[:N].sum(axis=0), w32[:N].sum(axis=0)
    cups32 = prob.ncell * args.steps / (ms32 * 1e-3)
    out["fp32"] = {"value": cups32, "unit": "cell-updates/s", "speedup_vs_fp64": cups32 / cups,
                   "ms_per_step": ms32 / args.steps,
                   "l1_rel_rho_vs_fp64": float(np.abs(rho32 - rho64).sum() / np.abs(rho64).sum()),
                   "after_steps": args.warmup + args.steps, "relax_bad": d32["relax_bad"]}
    if args.batch_steps > 0:
        out["batched"] = bench_batch(args)
    if args.learned_steps > 0:
        out["learned"] = bench_learned(args)
    if args.steps3d > 0:
        out["multimode_3d"] = bench_3d(args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
