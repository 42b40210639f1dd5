"""Launch-shape autotuner of the batched ensemble (hrm_batch_*).

The persistent batch kernel has three free launch parameters: threads per
workgroup (one face per thread; a tile holds threads - 1 cells, so small
workgroups waste fewer faces on short problems but stage more halo nodes),
the number of workgroups (how many problems are in flight at once) and the
SSP-RK3 steps per launch (launch overhead against the length of the tail
in which the last long problems run alone).  ``tune_batch`` times a small
grid of candidates on a private copy of the ensemble and returns the fastest;
results are cached in a JSON file keyed by device, species count, ensemble
size and precision.
"""
from __future__ import annotations

import json
import os
from typing import Optional

from . import hrm

CACHE_ENV = "HRM_TUNE_CACHE"


def _cache_path() -> str:
    return os.environ.get(CACHE_ENV, os.path.join(os.path.expanduser("~"), ".cache", "hrm_batch_tune.json"))


def _key(batch, precision, device_name) -> str:
    return f"{device_name}|N{batch.N}|P{batch.nprob}|T{batch.ncell}|prec{precision}"


def candidates(cus: int):
    """(threads, workgroups, steps per launch): one to three waves per SIMD
    (the kernel's register budget allows three) for 64, 128 and 256 threads."""
    out = []
    for threads in (64, 128, 256):
        per_wave = threads // 64
        for waves_per_simd in (1, 2, 3):
            blocks = cus * 4 * waves_per_simd // per_wave
            for k in (5, 20):
                out.append((threads, blocks, k))
    return out


def time_config(solver, W0, shape, steps: int) -> float:
    """Milliseconds per step of `steps` steps (a multiple of shape[2]) from W0,
    after one untimed launch that also captures the graph."""
    import torch
    threads, blocks, k = shape
    solver.configure(threads, blocks, k)
    solver.W.copy_(W0)
    solver.run(k)
    torch.cuda.synchronize()
    solver.W.copy_(W0)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    solver.run(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def tune_batch(batch, precision=hrm.FP64, steps: int = 20, use_cache: bool = True,
               shapes: Optional[list] = None, verbose: bool = False) -> dict:
    """Fastest (threads, blocks, steps_per_launch) for `batch`; the ensemble's
    own state is not touched (the candidates run on a private handle and copy)."""
    import torch
    props = torch.cuda.get_device_properties(0)
    key = _key(batch, precision, props.name)
    path = _cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            with open(path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
        if key in cache:
            return cache[key]
    shapes = shapes or candidates(props.multi_processor_count)
    s = hrm.BatchSolver(batch, precision=precision)
    W0 = s.W.clone()
    results = []
    try:
        for shape in shapes:
            n = max(steps // shape[2], 1) * shape[2]
            ms = time_config(s, W0, shape, n)
            results.append((ms, shape))
            if verbose:
                print(f"  threads {shape[0]:3d} blocks {shape[1]:5d} steps/launch {shape[2]:3d}: {ms:.4f} ms/step",
                      flush=True)
    finally:
        s.close()
    ms, (threads, blocks, k) = min(results)
    best = {"threads": threads, "blocks": blocks, "steps_per_launch": k, "ms_per_step": ms,
            "tried": [{"threads": sh[0], "blocks": sh[1], "steps_per_launch": sh[2], "ms_per_step": m}
                      for m, sh in results]}
    if use_cache:
        cache[key] = best
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            with open(path, "w") as f:
                json.dump(cache, f, indent=1)
        except OSError:
            pass
    return best
