"""Learned interpolation weights: training data from a fine ensemble and
training on the GPU through the library's own kernels (hrm_mlp_*).

The network (5-32-32-3, ReLU) rescales the classical fifth-order WENO weights
of the three 3-point candidates by at most e either way; it and its use in the
solver are described in include/hrm.h (hrm_set_mlp).  Pairs come from FP64 solutions
of an ensemble of 1D two-phase Riemann problems on a grid twice as fine as
the one the weights are meant for (labels by injection, hrm_mlp_extract).
"""
from __future__ import annotations

import numpy as np

from . import hrm
from . import inputs as I

NPARAM = hrm.MLP_NPARAM


def init_params(seed: int = 0, last_scale: float = 0.1) -> np.ndarray:
    """He-uniform hidden layers, zero biases, a small last layer (the initial
    weights are close to the classical ones)."""
    rng = np.random.default_rng(seed)
    parts = [rng.uniform(-1, 1, 160) * np.sqrt(6.0 / 5.0), np.zeros(32),
             rng.uniform(-1, 1, 1024) * np.sqrt(6.0 / 32.0), np.zeros(32),
             rng.uniform(-1, 1, 96) * np.sqrt(6.0 / 32.0) * last_scale, np.zeros(3)]
    return np.concatenate(parts).astype(np.float32)


def fine_ensemble(nprob: int = 1024, nmin: int = 100, nmax: int = 1000, seed: int = 4001):
    """Riemann problems of the batched workload's kind, on fine grids of even
    length 2 n with n uniform in [nmin, nmax]."""
    rng = np.random.default_rng(seed + 17)
    lengths = 2 * rng.integers(nmin, nmax + 1, size=nprob)
    return I.config4(seed=seed, lengths=lengths)


def training_data(batch, snapshots=(40, 120), cfl: float = 0.4):
    """FP64 solutions of `batch` after each snapshot's step count, turned into
    normalised training pairs on the GPU; returns (X (n, 8), T (n,)) float32
    device tensors."""
    import torch
    e = batch.eos
    eos = hrm.make_eos(e.gamma, e.cv, e.pinf, e.q)
    s = hrm.BatchSolver(batch)
    s.configure(256, 512, 1)
    per = hrm.hrm_mlp_extract(eos, None, batch.offsets)
    X = torch.empty((per * len(snapshots), 8), dtype=torch.float32, device="cuda")
    T = torch.empty(per * len(snapshots), dtype=torch.float32, device="cuda")
    done = 0
    for i, k in enumerate(sorted(snapshots)):
        s.run(k - done, cfl)
        done = k
        got = hrm.hrm_mlp_extract(eos, s.W, batch.offsets, X[i * per:(i + 1) * per], T[i * per:(i + 1) * per])
        assert got == per
    s.close()
    return X, T


def training_data_grid(prob, snapshots=(60, 120), stride: int = 8):
    """Pairs from lines of a grid workload (e.g. the 3D multimode interface
    at 256^3, a grid twice as fine as 128^3): FP64 solutions after each
    snapshot's step count, then the injection recipe along every direction
    on every `stride`-th line (hrm_mlp_extract_grid); returns (X (n, 8), T
    (n,)) float32 device tensors."""
    import torch
    e = prob.eos
    eos = hrm.make_eos(e.gamma, e.cv, e.pinf, e.q)
    grid = hrm.make_grid(prob.D, prob.n, prob.dx, prob.bc)
    per = hrm.hrm_mlp_extract_grid(grid, eos, None, stride)
    X = torch.empty((per * len(snapshots), 8), dtype=torch.float32, device="cuda")
    T = torch.empty(per * len(snapshots), dtype=torch.float32, device="cuda")
    s = hrm.Solver(prob, flags=hrm.FUSE_RELAX)
    done = 0
    for i, k in enumerate(sorted(snapshots)):
        s.advance(k - done, cfl=prob.cfl)
        done = k
        got = hrm.hrm_mlp_extract_grid(grid, eos, s.W, stride, X[i * per:(i + 1) * per], T[i * per:(i + 1) * per])
        assert got == per
    torch.cuda.synchronize()
    s.close()
    return X, T


def train(X, T, steps: int = 2000, count: int = 16384, lr: float = 2e-3, seed: int = 0, params=None,
          log_every: int = 0, lr_final: float = 0.05):
    """Adam on the mean squared normalised residual with a cosine decay of the
    step size from lr to lr * lr_final; minibatch i takes the samples
    (first_i + k stride) mod n, stride = n // count, so each minibatch spans
    the whole data set.  Returns (params float32, losses)."""
    import torch
    n = X.shape[0]
    count = min(count, n)
    dev = torch.device("cuda")
    p = torch.from_numpy(init_params(seed) if params is None else np.asarray(params, np.float32)).to(dev)
    m = torch.zeros(NPARAM, dtype=torch.float32, device=dev)
    v = torch.zeros_like(m)
    g = torch.zeros_like(m)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    work = torch.zeros(hrm.hrm_mlp_grad_workspace(count), dtype=torch.float32, device=dev)
    stride = max(1, n // count)
    losses = []
    for it in range(1, steps + 1):
        first = (it * 7919) % n
        hrm.hrm_mlp_grad(p, X, T, first, stride, count, g, loss, work)
        f = lr_final + (1.0 - lr_final) * 0.5 * (1.0 + np.cos(np.pi * (it - 1) / max(steps - 1, 1)))
        hrm.hrm_mlp_adam(p, g, m, v, it, lr * f)
        if log_every and (it % log_every == 0 or it == 1):
            losses.append((it, float(loss.item())))
    return p.cpu().numpy(), losses


def mean_loss(params, X, T, count: int = 1 << 20) -> float:
    """Loss over (up to) `count` evenly spread samples."""
    import torch
    n = X.shape[0]
    count = min(count, n)
    dev = torch.device("cuda")
    p = torch.from_numpy(np.asarray(params, np.float32)).to(dev)
    g = torch.zeros(NPARAM, dtype=torch.float32, device=dev)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    work = torch.zeros(hrm.hrm_mlp_grad_workspace(count), dtype=torch.float32, device=dev)
    hrm.hrm_mlp_grad(p, X, T, 0, max(1, n // count), count, g, loss, work)
    return float(loss.item())
