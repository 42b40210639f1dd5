"""FP32 face arithmetic (the node primitives, flux limiter, limiter bound
checks, accumulation and relaxation stay double): accuracy against the FP64
path and the oracle, stated as L1 errors, and positivity."""
import numpy as np
import pytest

from paper_2208_04488_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2208_04488_amd import hrm
    return hrm


def l1_rel(a, b):
    """Relative L1 difference of the mixture density."""
    N = a.shape[0]
    return float(np.abs(a - b).sum() / np.abs(b).sum())


def run(H, prob, precision, steps=None, t_end=0.0, flags=None):
    import torch
    s = H.Solver(prob, flags=H.FUSE_RELAX if flags is None else flags, precision=precision)
    s.set_slot(0.0, [0.0] * prob.D)
    k = 0
    while True:
        if steps is not None and k >= steps:
            break
        s.step(cfl=prob.cfl, t_end=t_end)
        k += 1
        if steps is None and k % 50 == 0:
            torch.cuda.synchronize()
            if s.slot[4].item() >= t_end:
                break
    torch.cuda.synchronize()
    out, d = s.state(), s.diagnostics()
    s.close()
    return out, d


def rho(W, N):
    return W[:N].sum(axis=0)


def admissible(W, N, D):
    a = W[N + D + 1:]
    return np.isfinite(W).all() and (W[:N] >= 0).all() and (a >= 0).all() and (1 - a.sum(0) >= 0).all()


@pytest.mark.parametrize("maker,steps,tol", [("config2_small", 20, 2e-6), ("config3_small", 10, 2e-6),
                                             ("shock_tube_extreme", 100, 1e-4)])
def test_fp32_tracks_fp64(H, maker, steps, tol):
    prob = {"config2_small": lambda: I.config2(128, 64), "config3_small": lambda: I.config3(32),
            "shock_tube_extreme": lambda: I.shock_tube(1000, True)}[maker]()
    a64, _ = run(H, prob, H.FP64, steps=1)
    a32, _ = run(H, prob, H.FP32, steps=1)
    e1 = l1_rel(rho(a32, prob.N), rho(a64, prob.N))
    w64, d64 = run(H, prob, H.FP64, steps=steps)
    w32, d32 = run(H, prob, H.FP32, steps=steps)
    err = l1_rel(rho(w32, prob.N), rho(w64, prob.N))
    print(f"{maker}: L1(rho) FP32 vs FP64 after 1 step = {e1:.3e}, after {steps} steps = {err:.3e}")
    assert err <= tol
    assert admissible(w32, prob.N, prob.D) and d32["relax_bad"] == 0


def test_fp32_config1_against_exact_riemann(H):
    """Config-1 shock tube to 240 us: FP32 and FP64 have the same L1 error
    against the exact stiffened-gas solution to three digits."""
    from oracle import exact_riemann as ER
    prob = I.config1(400)
    eos = prob.eos
    L = dict(rho=1000.0, u=0.0, p=1e9, gamma=eos.gamma[0], pinf=eos.pinf[0])
    R = dict(rho=50.0, u=0.0, p=1e5, gamma=eos.gamma[1], pinf=0.0)
    rex, _, _ = ER.solve(prob.centres(0), prob.t_end, 0.7, L, R)
    errs = {}
    for prec in (H.FP64, H.FP32):
        w, d = run(H, prob, prec, t_end=prob.t_end)
        errs[prec] = np.abs(rho(w, 2)[0, 0] - rex).sum() * prob.dx[0]
        assert admissible(w, 2, 1) and d["relax_bad"] == 0
    print(f"config1 L1(rho) vs exact: FP64 {errs[H.FP64]:.6e}  FP32 {errs[H.FP32]:.6e}")
    assert errs[H.FP32] == pytest.approx(errs[H.FP64], rel=1e-3)


@pytest.mark.parametrize("maker", ["config2_96x48", "config3_70"])
def test_fp32_stage_against_oracle(H, maker):
    """One FP32 stage against the FP64 oracle: agreement at FP32 level (in
    3D at 70^3 the x lines take three 32 x 8 tiles, the last with 8 cells)."""
    import torch
    import oracle
    prob = {"config2_96x48": lambda: I.config2(96, 48), "config3_70": lambda: I.config3(70)}[maker]()
    o = oracle.from_problem(prob)
    W0 = prob.W
    dt, lam = o.dt(W0, prob.cfl)
    ref = o.stage(0, W0, W0, dt, lam)
    s = H.Solver(prob, flags=H.FUSE_RELAX, precision=H.FP32)
    s.set_slot(dt, lam)
    got = s.stage(0, s.W, s.W).cpu().numpy()
    M, N, D = prob.M, prob.N, prob.D
    scale = np.abs(ref.reshape(M, -1)).max(axis=1)
    scale[N:N + D] = max(scale[N:N + D].max(), rho(ref, N).max() * o.max_wavespeed(W0).max())
    scale[N + D + 1:] = 1.0
    err = (np.abs(got - ref).reshape(M, -1).max(axis=1) / scale).max()
    print(f"FP32 stage vs oracle: {err:.3e}")
    assert err <= 1e-6
    s.close()
