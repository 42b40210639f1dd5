#!/usr/bin/env python
"""Throughput of the fractional PP-WCNS-IS step on one MI355X.

A step is one SSP-RK3 step of the fractional algorithm: wavespeed and time
step from W^n, three stages of the five-equation hyperbolic operator, each
followed by the infinite-rate thermal relaxation.  Headline workload: the 3D
multimode interface (256^3 cells, three species: light and heavy gas with
liquid droplets, Mach-1.5 shock), FP64, the largest workload one GPU runs;
the FP32 form runs beside it, and both go on to the workload's 200 steps for
their L1 difference.

Prints one JSON line.  Inputs are resident in HBM before the timed region.
`roofline` describes the dominant kernel (the z-direction sweep, which also
applies the stage update and the relaxation), timed live with HIP events on
the stream it runs on.  Extra keys: the 2D liquid column (1024 x 512, FP64
and FP32 to its 500 steps), the batched ensemble of 1D Riemann problems, and
the learned interpolation weights against the plain method and against the
network's own prior on the planar shock tube (2048 x 1024 to 240 us, L1
against the exact solution).  `cpu_baseline` times the CPU oracle on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
METRIC = ("cell-updates/s per RK3 step (plain FP64 vs FP32 vs learned) at stated L1 error; HBM GB/s")
PEAK_FP64_TFLOPS = 78.6    # MI355X FP64 vector, dense
PEAK_HBM_GBS = 8000.0      # MI355X HBM3E
PEAK_BF16_TFLOPS = 2500.0  # MI355X dense bfloat16 matrix


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


def sweep_arrays(D, direction):
    """M x ncell double arrays one launch of the sweep in `direction` reads
    or writes: W_s read; the first direction writes the RHS, middle ones read
    and write it, the last reads it (D > 1) and W^n and writes the stage output."""
    if D == 1:
        return 3
    if direction == D - 1:
        return 4
    return 2 if direction == 0 else 3


def counters_path(name):
    return os.path.join(ROOT, "profiles", name)


def kernel_source_hash() -> str:
    """sha256 over the sources of the grid sweeps: csrc/hrm.hip and every
    header it includes, directly or through another header (name, then
    contents, sorted by name).  The ensemble and training kernels are other
    translation units and do not enter it."""
    import hashlib
    import re
    dirs = [os.path.join(ROOT, "paper_2208_04488_amd", "csrc"), os.path.join(ROOT, "include")]
    seen, todo = {}, ["hrm.hip"]
    while todo:
        name = todo.pop()
        if name in seen:
            continue
        path = next(os.path.join(d, name) for d in dirs if os.path.exists(os.path.join(d, name)))
        with open(path, "rb") as fh:
            seen[name] = fh.read()
        todo += re.findall(r'^#include "([^"]+)"', seen[name].decode(), re.M)
    h = hashlib.sha256()
    for name in sorted(seen):
        h.update(name.encode())
        h.update(seen[name])
    return h.hexdigest()


def measured_traffic(counters_file: str, kernel: str):
    """HBM bytes per launch of `kernel` from a committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by the copy calibration), or
    None if the summary is missing, is for another kernel, or was taken on
    other kernel sources than the ones built here."""
    try:
        with open(counters_path(counters_file)) as f:
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


def sweep_kernel_name(N, D, direction):
    """The sweep's template name as the profiler prints it (both
    instantiations, with and without the wavespeed epilogue)."""
    if D == 1:
        bs, ba = 256, 1
    elif direction == 0:
        bs, ba = 64, 4
    else:
        bs, ba = 16, 16
    return f"k_sweep<{N},{D},{direction},{bs},{ba},double,0,*>"


def l1_rel(a, b):
    import numpy as np
    return float(np.abs(a - b).sum() / np.abs(b).sum())


def timed_advance(s, steps, cfl, stream):
    """Milliseconds of `steps` RK3 steps in one hrm_advance call, between
    torch events on the current stream (wall seconds beside)."""
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    e0.record(stream)
    s.advance(steps, cfl=cfl)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1), time.perf_counter() - w0


def sweep_timers(s, steps, cfl):
    """The same steps again with the library's HIP events around every sweep
    and time-step launch, on the stream they run on (direct launches, no
    graph): {name: (total ms, launches)}."""
    from paper_2208_04488_amd import hrm
    hrm.hrm_set_timing(s.ctx, (1 << 0) | (1 << 1) | (1 << 2) | (1 << 3))
    hrm.hrm_get_timing(s.ctx)  # clear
    s.advance(steps, cfl=cfl)
    t = hrm.hrm_get_timing(s.ctx)
    hrm.hrm_set_timing(s.ctx, 0)
    return t


def bench_grid(prob, args, total_steps, counters_file=None):
    """FP64 and FP32 face arithmetic on one grid workload: W warm-up steps,
    K timed steps, K steps with kernel timers, then on to `total_steps` (the
    workload's length) for the L1 difference of the mixture density."""
    import torch
    from paper_2208_04488_amd import hrm
    N, D, M = prob.N, prob.D, prob.M
    stream = torch.cuda.current_stream()
    res = {}
    for name, prec in (("fp64", hrm.FP64), ("fp32", hrm.FP32)):
        s = hrm.Solver(prob, flags=hrm.FUSE_RELAX, precision=prec)
        s.advance(args.warmup, cfl=prob.cfl)
        ms, wall = timed_advance(s, args.steps, prob.cfl, stream)
        timers = sweep_timers(s, args.steps, prob.cfl)
        done = args.warmup + 2 * args.steps
        if total_steps > done:
            s.advance(total_steps - done, cfl=prob.cfl)
            done = total_steps
        torch.cuda.synchronize()
        d = s.diagnostics()
        W = s.state()
        res[name] = dict(ms=ms, wall=wall, timers=timers, diag=d, rho=W[:N].sum(axis=0), steps_run=done,
                         admissible=bool((W[:N] >= 0).all() and (W[N + D + 1:] >= 0).all()
                                         and (W[N + D + 1:].sum(axis=0) <= 1).all()))
        s.close()
        del s, W
        torch.cuda.empty_cache()
    out = {}
    names = ("sweep_x", "sweep_y", "sweep_z")[:D]
    for name in ("fp64", "fp32"):
        r = res[name]
        t = r["timers"]
        out[name] = {"value": prob.ncell * args.steps / (r["ms"] * 1e-3), "unit": "cell-updates/s",
                     "ms_per_step": r["ms"] / args.steps, "wall_s_timed": r["wall"],
                     "sweep_ms_per_launch": {k: t[k][0] / max(t[k][1], 1) for k in names},
                     "kernel_ms_per_step": {k: v[0] / args.steps for k, v in t.items() if v[1]},
                     "positivity": {"relax_bad": r["diag"]["relax_bad"], "interp_hs": r["diag"]["interp_hs"],
                                    "flux_hs": r["diag"]["flux_hs"], "admissible_after_run": r["admissible"],
                                    "steps": r["steps_run"]}}
    f64 = out["fp64"]
    kname = max(names, key=lambda k: res["fp64"]["timers"][k][0])
    kdir = names.index(kname)
    ms_launch = f64["sweep_ms_per_launch"][kname]
    flops = mean_launch_flops(N, D, prob.n, kdir)
    achieved = flops / (ms_launch * 1e-3) / 1e12
    traffic = measured_traffic(counters_file, sweep_kernel_name(N, D, kdir)) if counters_file else None
    f64["roofline"] = {"bound": "alu", "kernel": f"k_sweep direction {kdir} (N={N}, D={D})",
                       "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                       "frac": achieved / PEAK_FP64_TFLOPS, "traffic": traffic,
                       "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                       "traffic_gbs": None if traffic is None else traffic / (ms_launch * 1e-3) / 1e9,
                       "algorithmic_bytes_per_launch": 8 * M * prob.ncell * sweep_arrays(D, kdir),
                       "flops_per_launch": flops, "ms_per_launch": ms_launch}
    # every sweep against the same peak (the roofline object above is the
    # sweep with the largest share of the step)
    f64["sweep_fp64_fraction"] = {}
    for d, nm in enumerate(names):
        fl = mean_launch_flops(N, D, prob.n, d)
        t_ms = f64["sweep_ms_per_launch"][nm]
        f64["sweep_fp64_fraction"][nm] = {"tflops": fl / (t_ms * 1e-3) / 1e12,
                                          "frac": fl / (t_ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS}
    f64["hbm_gbs_algorithmic"] = algorithmic_bytes_per_cell_step(M) * f64["value"] / 1e9
    out["fp32"]["speedup_vs_fp64"] = out["fp32"]["value"] / f64["value"]
    steps = min(res["fp64"]["steps_run"], res["fp32"]["steps_run"])
    assert res["fp64"]["steps_run"] == res["fp32"]["steps_run"]
    out["fp32"]["l1_rel_rho_vs_fp64"] = l1_rel(res["fp32"]["rho"], res["fp64"]["rho"])
    out["fp32"]["l1_after_steps"] = steps
    return out


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
    import numpy as np
    N = batch.N
    r32, r64 = res["fp32"]["W"][:N].sum(axis=0), res["fp64"]["W"][:N].sum(axis=0)
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
    out["fp32"]["l1_rel_rho_vs_fp64"] = l1_rel(r32, r64)
    out["fp32"]["l1_after_steps"] = res["fp32"]["steps"]
    return out


MLP_FLOPS_PER_STENCIL = 2 * (5 * 32 + 32 * 32 + 32 * 3)  # algorithmic multiply-adds x 2


def exact_profile(n):
    """Exact density of the shock tube at 240 us on n cells (stored by
    tests/golden/make_exact_profiles.py)."""
    import numpy as np
    return np.loadtxt(os.path.join(ROOT, "tests", "golden", f"exact_rho_shock_tube_{n}.txt"))


def run_to_end(s, prob, chunk):
    """Steps until the device time reaches the workload's end time (the last
    step is clipped onto it; steps beyond leave the state unchanged)."""
    import torch
    k = 0
    while True:
        s.advance(chunk, cfl=prob.cfl, t_end=prob.t_end)
        k += chunk
        torch.cuda.synchronize()
        if s.slot[4].item() >= prob.t_end:
            return k


def bench_learned(args):
    """Learned interpolation weights on the planar shock tube (2048 x 1024,
    FP64 state; the network in bfloat16 on the matrix cores) against the
    plain method (App. C weights) and against the network's prior alone (a
    zero network: the classical WENO5 weights it rescales).  The network is
    trained first, on the GPU, by the library's own kernels (untimed)."""
    import numpy as np
    import torch
    from paper_2208_04488_amd import hrm, learned
    from paper_2208_04488_amd import inputs as I

    prior = learned.init_params(0, last_scale=0.0)
    sources = {}
    # the same label recipe (injection from a twice finer grid) on two sources:
    # fine 1D Riemann problems of the batched workload's kind, and lines of
    # the 3D multimode workload at 256^3 (every 8th line in each direction)
    for src in ("ensemble_1d", "multimode_3d"):
        t0 = time.perf_counter()
        if src == "ensemble_1d":
            fine = learned.fine_ensemble(nprob=1024, nmin=100, nmax=1000, seed=4001)
            X, T = learned.training_data(fine, snapshots=(40, 120))
            data = "1024 fine 1D two-phase Riemann problems (200-2000 cells) after 40 and 120 FP64 steps"
        else:
            X, T = learned.training_data_grid(I.config3(args.n3d), snapshots=(60, 120), stride=8)
            data = (f"lines of the {args.n3d}^3 multimode workload (every 8th in each transverse direction, all "
                    f"three directions) after 60 and 120 FP64 steps")
        loss0 = learned.mean_loss(prior, X, T)
        params, _ = learned.train(X, T, steps=3000, count=16384, lr=2e-3, seed=0)
        loss1 = learned.mean_loss(params, X, T)
        torch.cuda.synchronize()
        sources[src] = dict(params=params, pairs=int(X.shape[0]), seconds=time.perf_counter() - t0,
                            loss_prior=loss0, loss_trained=loss1, data=data + ", labels by injection")
        del X, T
        torch.cuda.empty_cache()

    stream = torch.cuda.current_stream()
    out = {"workload": f"planar two-phase shock tube (liquid 1e9 Pa | air 1e5 Pa at x = 0.7), "
                       f"{args.learned_nx}x{args.learned_ny} cells, 2 species, transmissive x / periodic y, "
                       f"CFL 0.4, to 240 us",
           "envelope": "learned weights: FP64 face arithmetic, one and two dimensions only",
           "training": {k: {kk: vv for kk, vv in v.items() if kk != "params"} | {"adam_steps": 3000,
                                                                                "minibatch": 16384}
                        for k, v in sources.items()},
           "shipped_weights": "learned = trained on the 1D ensemble; learned_3d = trained on 3D multimode lines"}
    legs = (("plain", None), ("prior", prior), ("learned", sources["ensemble_1d"]["params"]),
            ("learned_3d", sources["multimode_3d"]["params"]))
    # the 1D workload at its own size, to 240 us (cheap; context for the 2D one)
    p1 = I.config1(400)
    ex1 = exact_profile(400)
    for name, mlp in legs:
        if args.learned_no_l1:
            break
        s = hrm.Solver(p1, flags=hrm.FUSE_RELAX, mlp=mlp)
        k = run_to_end(s, p1, 100)
        w = s.state()
        s.close()
        out.setdefault("shock_tube_400", {})[name] = {
            "l1_rho_vs_exact": float(np.abs(w[:2].sum(axis=0)[0, 0] - ex1).sum() * p1.dx[0]), "steps": k}
    prob = I.config5(args.learned_nx, args.learned_ny)
    N, D, M = prob.N, prob.D, prob.M
    ex = exact_profile(prob.n[0]) if prob.n[0] in (400, 2048) else None
    for name, mlp in legs:
        s = hrm.Solver(prob, flags=hrm.FUSE_RELAX, mlp=mlp)
        s.advance(args.warmup, cfl=prob.cfl)
        ms, _ = timed_advance(s, args.learned_steps, prob.cfl, stream)
        tm = sweep_timers(s, 5, prob.cfl)
        steps = args.warmup + args.learned_steps + 5 + (0 if args.learned_no_l1 else run_to_end(s, prob, 200))
        d = s.diagnostics()
        w = s.state()
        s.close()
        rho = w[:N].sum(axis=0).reshape(-1, prob.n[0])  # rows of the planar problem
        leg = {"value": prob.ncell * args.learned_steps / (ms * 1e-3), "unit": "cell-updates/s",
               "ms_per_step": ms / args.learned_steps,
               "sweep_ms_per_launch": {k: tm[k][0] / max(tm[k][1], 1) for k in ("sweep_x", "sweep_y")},
               "relax_bad": d["relax_bad"], "steps_to_end": steps,
               "rows_identical": bool(np.abs(rho - rho[0]).max() <= 1e-9 * rho.max())}
        if ex is not None and not args.learned_no_l1:
            leg["l1_rho_vs_exact"] = float(np.abs(rho[0] - ex).sum() * prob.dx[0])
        out[name] = leg
    for name in ("prior", "learned", "learned_3d"):
        out[name]["speedup_vs_plain"] = out[name]["value"] / out["plain"]["value"]
    faces = (prob.n[0] + 1) * prob.n[1] + prob.n[0] * (prob.n[1] + 1)
    mf = 3 * faces * 2 * M * MLP_FLOPS_PER_STENCIL  # 2M stencils per face, both sweeps, 3 stages
    out["learned"]["mfma_tflops_algorithmic"] = mf / (out["learned"]["ms_per_step"] * 1e-3) / 1e12
    out["learned"]["mfma_frac_of_bf16_peak"] = out["learned"]["mfma_tflops_algorithmic"] / PEAK_BF16_TFLOPS
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


def _oracle_rate(prob, budget_s, max_steps):
    import oracle
    o = oracle.from_problem(prob)
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


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n3d=256):
    """The oracle as it stands (C, FP64, OpenMP over grid lines) on the host
    cores: complete SSP-RK3 steps of the full headline workload from its
    initial condition with every thread (two, unless the first takes 20 s or
    more), the same workload's recipe at 64^3
    on one core, and short samples of the other workloads."""
    import oracle
    from paper_2208_04488_amd import inputs as I
    oracle.build(force=False)
    threads = oracle.Oracle.set_threads(0)
    prob = I.config3(n3d)
    rate, steps, el = _oracle_rate(prob, 20.0, 2)
    del prob
    out = {"value": rate, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
           "sample": f"{steps} SSP-RK3 step(s) of the full {n3d}^3 multimode workload from its initial condition, "
                     f"OpenMP over grid lines on {threads} threads, {el:.1f} s",
           "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
           "cpus_available": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None}
    oracle.Oracle.set_threads(1)
    r1, k1, e1 = _oracle_rate(I.config3(64), 0.0, 1)
    out["one_core"] = {"value": r1, "sample": f"{k1} step of the same recipe at 64^3 on 1 thread, {e1:.1f} s"}
    oracle.Oracle.set_threads(threads)
    more = {}
    for name, p in (("liquid_column_1024x512", I.config2(1024, 512)),
                    ("planar_shock_tube_512x256", I.config5(512, 256)),
                    ("riemann_problem_1000_cells", I.config4(lengths=[1000]).problem(0))):
        r, k, e = _oracle_rate(p, 4.0, 50)
        more[name] = {"value": r, "steps": k, "seconds": e}
    out["other_workloads"] = more
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n3d", type=int, default=256)
    ap.add_argument("--total3d", type=int, default=200, help="steps of the 3D workload (FP64 and FP32 L1)")
    ap.add_argument("--nx", type=int, default=1024)
    ap.add_argument("--ny", type=int, default=512)
    ap.add_argument("--total2d", type=int, default=500, help="steps of the 2D liquid column (0 skips it)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-steps", type=int, default=1000,
                    help="steps of the batched ensemble (0 skips it)")
    ap.add_argument("--learned-steps", type=int, default=50,
                    help="timed steps of the learned-weight comparison (0 skips it)")
    ap.add_argument("--learned-nx", type=int, default=2048)
    ap.add_argument("--learned-ny", type=int, default=1024)
    ap.add_argument("--learned-no-l1", action="store_true",
                    help="time the learned legs only (no runs to 240 us; for profiling)")
    ap.add_argument("--only-2d", action="store_true",
                    help="run the 2D liquid column leg alone (for profiling its kernels)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 2 GiB elementwise copy (reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (a sharded run would split the "
              "grid into slabs and exchange 3-cell halos every stage). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

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
    from paper_2208_04488_amd import inputs as I

    if args.only_2d:
        print(json.dumps({"liquid_column_2d": bench_grid(I.config2(args.nx, args.ny), args, args.total2d)}),
              flush=True)
        return
    prob = I.config3(args.n3d)
    N, D, M = prob.N, prob.D, prob.M
    g = bench_grid(prob, args, args.total3d, counters_file="k_sweep_multimode_256cube_fp64_counters.json")
    del prob
    f64 = g["fp64"]
    out = {
        "metric": METRIC, "value": f64["value"], "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": f64["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"3D multimode interface: light/heavy gas (density ratio 3) perturbed by 32 random "
                               f"modes, 10% liquid droplets, Mach-1.5 shock, 3 species, {args.n3d}^3 cells, "
                               f"periodic y/z, FP64 PP-WCNS-IS + thermal relaxation, CFL 0.4",
                   "cells": args.n3d ** 3, "species": N, "dim": D, "components": M},
        "roofline": f64["roofline"],
        "sweep_fp64_fraction": f64["sweep_fp64_fraction"],
        "hbm_gbs_algorithmic": f64["hbm_gbs_algorithmic"],
        "hbm_frac_algorithmic": f64["hbm_gbs_algorithmic"] / PEAK_HBM_GBS,
        "hbm_copy_gbs_measured": measured_copy_gbs(),
        "kernel_ms_per_step": f64["kernel_ms_per_step"],
        "wall_s_timed": f64["wall_s_timed"],
        "positivity": f64["positivity"],
        "fp32": g["fp32"],
        "tiles": "grid sweeps: x 64x4, or 32x8 where it needs fewer face threads (256^3: 32x8); y and z 16x16; the ensemble's launch shape is autotuned",
    }
    if args.total2d > 0:
        p2 = I.config2(args.nx, args.ny)
        out["liquid_column_2d"] = dict(
            workload=f"2D Mach-1.47 shock on a liquid column with a gas bubble, 3 species, {args.nx}x{args.ny} "
                     f"cells, CFL 0.4", **bench_grid(p2, args, args.total2d,
                                                     counters_file="k_sweep_liquid_column_1024x512_fp64_counters.json"))
    if args.batch_steps > 0:
        out["batched"] = bench_batch(args)
    if args.learned_steps > 0:
        out["learned"] = bench_learned(args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.n3d)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
