"""Learned interpolation weights on the GPU: the bfloat16 matrix-core network
against the oracle's rounded evaluation, the float32 training kernels
(extraction, gradient, Adam) against the NumPy FP64 oracle, the solver with
learned weights against the C oracle, the fallback to App. C, and what the
trained network gains over the plain method on the config-1 shock tube."""
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


@pytest.fixture(scope="module")
def M():
    from oracle import mlp_ref
    return mlp_ref


def rand_params(M, seed, scale):
    return M.init(seed, last_scale=scale).astype(np.float32)


def stencils(rng, n):
    """Smooth, kinked, stepped, constant and near-constant stencils at many scales."""
    U = []
    xs = np.arange(-2.0, 3.0)
    for i in range(n):
        kind = i % 5
        a = 10.0 ** rng.uniform(-6, 6)
        if kind == 0:
            u = np.polynomial.Polynomial(rng.normal(size=4))(xs * rng.uniform(0.01, 1))
        elif kind == 1:
            u = np.where(xs < rng.uniform(-2, 2), rng.normal(), rng.normal())
        elif kind == 2:
            u = np.abs(xs - rng.uniform(-2, 2)) + rng.normal() * 0.1
        elif kind == 3:
            u = np.full(5, rng.normal())
        else:
            u = rng.normal() + 1e-9 * rng.normal(size=5)
        U.append(a * u + rng.normal() * a)
    return np.array(U)


def infer(H, prob_params, U):
    import torch
    prob = I.config1(16)
    s = H.Solver(prob, mlp=prob_params)
    d = torch.from_numpy(np.ascontiguousarray(U)).cuda()
    val = torch.empty(len(U), dtype=torch.float64, device="cuda")
    om = torch.empty((len(U), 3), dtype=torch.float32, device="cuda")
    H.hrm_mlp_infer(s.ctx, d, val, om)
    torch.cuda.synchronize()
    out = val.cpu().numpy(), om.cpu().numpy().astype(np.float64)
    s.close()
    return out


def test_zero_last_layer_gives_classical_weights(H, M):
    """z = 0: the classical fifth-order WENO weights of the normalised stencil
    (float evaluation against the double one on the same float inputs)."""
    p = rand_params(M, 1, 0.0)
    rng = np.random.default_rng(11)
    U = stencils(rng, 500)
    val, om = infer(H, p, U)
    x, _ = M.normalise(U)
    ref = M.forward(p, x.astype(np.float32).astype(np.float64))["w"]
    print("classical weights |diff| max %.2e" % np.abs(om - ref).max())
    assert np.abs(om - ref).max() <= 1e-5


def test_matrix_core_network_matches_oracle(H, M, orc):
    """Weights of a trained-looking network (last layer of order one) on
    stencils of every kind: the matrix-core result against the oracle's
    bfloat16 evaluation in double.  Float accumulation can move a hidden
    activation across a bfloat16 rounding boundary, so a few weights may
    differ by a bfloat16 step; the typical difference is float round-off."""
    p = rand_params(M, 2, 3.0)
    rng = np.random.default_rng(12)
    U = stencils(rng, 4000)
    val, om = infer(H, p, U)
    ref_w = np.zeros_like(om)
    ref_v = np.zeros(len(U))
    for i, u in enumerate(U):
        v, w = orc.mlp_interp(p.astype(np.float64), u)
        ref_v[i], ref_w[i] = v, w
    dw = np.abs(om - ref_w).max(axis=1)
    print("omega |diff|: median %.2e  99.9%% %.2e  max %.2e" % (np.median(dw), np.quantile(dw, 0.999), dw.max()))
    assert np.median(dw) <= 1e-6
    assert np.quantile(dw, 0.99) <= 1e-4
    assert dw.max() <= 3e-2
    spread = np.abs(U - U[:, 2:3]).max(axis=1)
    # relative to the stencil's spread (round-off of the candidates for constant ones)
    dv = np.abs(val - ref_v) / np.maximum(spread, 1e-14 * np.abs(U).max(axis=1))
    print("value |diff| / spread: median %.2e  max %.2e" % (np.median(dv), dv.max()))
    assert np.median(dv) <= 1e-6 and dv.max() <= 3e-2
    # the weights are convex and the value lies between the candidates
    assert (om >= 0).all() and np.abs(om.sum(axis=1) - 1).max() < 1e-6
    S = U @ M.CAND.T
    tol = 1e-6 * spread + 1e-12 * np.abs(U).max(axis=1)   # float weights
    assert (val >= S.min(axis=1) - tol).all() and (val <= S.max(axis=1) + tol).all()


def test_training_gradient_matches_numpy_oracle(H, M):
    import torch
    rng = np.random.default_rng(13)
    X64, _ = M.normalise(stencils(rng, 1000))
    X32 = np.zeros((1000, 8), dtype=np.float32)
    X32[:, :5] = X64
    T32 = rng.uniform(-1.5, 1.5, size=1000).astype(np.float32)
    for seed, scale in ((3, 0.0), (4, 1.0), (5, 3.0)):
        p = rand_params(M, seed, scale)
        p[160:192] = rng.normal(size=32) * 0.1       # nonzero biases
        p[1216:1248] = rng.normal(size=32) * 0.1
        p[1344:] = rng.normal(size=3) * 0.1
        dev = torch.device("cuda")
        tp = torch.from_numpy(p).to(dev)
        tX, tT = torch.from_numpy(X32).to(dev), torch.from_numpy(T32).to(dev)
        g = torch.zeros(M.NPARAM, dtype=torch.float32, device=dev)
        loss = torch.zeros(1, dtype=torch.float32, device=dev)
        work = torch.zeros(H.hrm_mlp_grad_workspace(1000), dtype=torch.float32, device=dev)
        H.hrm_mlp_grad(tp, tX, tT, 0, 1, 1000, g, loss, work)
        torch.cuda.synchronize()
        Xd = X32[:, :5].astype(np.float64)
        Td = T32.astype(np.float64)
        gref = M.grad(p.astype(np.float64), Xd, Td)
        err = np.abs(g.cpu().numpy() - gref).max() / np.abs(gref).max()
        lerr = abs(loss.item() - M.loss(p.astype(np.float64), Xd, Td)) / M.loss(p.astype(np.float64), Xd, Td)
        print(f"seed {seed}: grad rel err {err:.2e}, loss rel err {lerr:.2e}")
        assert err <= 2e-5 and lerr <= 2e-6


def test_minibatch_indexing(H, M):
    """Samples (first + k stride) mod n: the gradient of a strided minibatch
    equals that of the same samples gathered on the host."""
    import torch
    rng = np.random.default_rng(14)
    n = 777
    X64, _ = M.normalise(stencils(rng, n))
    X32 = np.zeros((n, 8), dtype=np.float32)
    X32[:, :5] = X64
    T32 = rng.uniform(-1, 1, size=n).astype(np.float32)
    p = rand_params(M, 6, 1.0)
    dev = torch.device("cuda")
    first, stride, count = 700, 13, 200
    idx = (first + np.arange(count) * stride) % n
    tp = torch.from_numpy(p).to(dev)
    g = torch.zeros(M.NPARAM, dtype=torch.float32, device=dev)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    work = torch.zeros(H.hrm_mlp_grad_workspace(count), dtype=torch.float32, device=dev)
    H.hrm_mlp_grad(tp, torch.from_numpy(X32).to(dev), torch.from_numpy(T32).to(dev), first, stride, count, g, loss,
                   work)
    gref = M.grad(p.astype(np.float64), X32[idx, :5].astype(np.float64), T32[idx].astype(np.float64))
    assert np.abs(g.cpu().numpy() - gref).max() / np.abs(gref).max() <= 2e-5


def test_adam_matches_oracle(H, M):
    import torch
    rng = np.random.default_rng(15)
    p = rng.normal(size=M.NPARAM).astype(np.float32)
    dev = torch.device("cuda")
    tp = torch.from_numpy(p.copy()).to(dev)
    tm = torch.zeros(M.NPARAM, dtype=torch.float32, device=dev)
    tv = torch.zeros_like(tm)
    rp, rm, rv = p.astype(np.float64), np.zeros(M.NPARAM), np.zeros(M.NPARAM)
    for step in range(1, 4):
        g = rng.normal(size=M.NPARAM).astype(np.float32)
        H.hrm_mlp_adam(tp, torch.from_numpy(g).to(dev), tm, tv, step, 1e-2)
        rp, rm, rv = M.adam(rp, g.astype(np.float64), rm, rv, step, 1e-2)
    torch.cuda.synchronize()
    assert np.abs(tp.cpu().numpy() - rp).max() <= 1e-6


def test_extraction_matches_oracle(H, M, orc):
    """Training pairs of a small fine ensemble (odd and too-short problems
    give none) against the oracle's injection recipe, field by field."""
    import torch
    lengths = [10, 12, 40, 7, 8, 64]
    fine = I.config4(seed=4201, lengths=lengths)
    e = fine.eos
    eos = H.make_eos(e.gamma, e.cv, e.pinf, e.q)
    W = torch.from_numpy(fine.W).cuda()
    n = H.hrm_mlp_extract(eos, None, fine.offsets)
    X = torch.zeros((n, 8), dtype=torch.float32, device="cuda")
    T = torch.zeros(n, dtype=torch.float32, device="cuda")
    assert H.hrm_mlp_extract(eos, W, fine.offsets, X, T) == n
    X, T = X.cpu().numpy(), T.cpu().numpy()
    o = orc.from_problem(fine.problem(0))
    Nsp = fine.N
    pos = 0
    for b in range(fine.nprob):
        lo, hi = fine.offsets[b], fine.offsets[b + 1]
        w = fine.W[:, lo:hi]
        prim = [o.prim(w[:, i]) for i in range(hi - lo)]
        fields = [w[k] for k in range(Nsp)] + [np.array([q["u"][0] for q in prim]),
                                               np.array([q["p"] for q in prim])] + [w[Nsp + 2 + k] for k in range(Nsp - 1)]
        for f, fv in enumerate(fields):
            if (hi - lo) % 2:
                continue
            xr, tr = M.samples_from_fine(fv, keep_degenerate=True)
            k = len(tr)
            exact = f < Nsp or f >= Nsp + 2
            tol = 0.0 if exact else 2e-6
            assert np.abs(X[pos:pos + k, :5] - xr.astype(np.float32)).max(initial=0) <= tol, (b, f)
            assert np.abs(T[pos:pos + k] - tr.astype(np.float32)).max(initial=0) <= tol * 10, (b, f)
            assert (X[pos:pos + k, 5:] == 0).all()
            pos += k
    assert pos == n


def test_solver_with_learned_weights_matches_oracle(H, M, orc):
    """Three SSP-RK3 stages of the solver with learned weights against the C
    oracle with the same parameters (1D shock tube and 2D liquid column)."""
    import torch
    p = rand_params(M, 7, 1.0)
    for prob in (I.config1(200), I.config2(64, 40)):
        o = orc.from_problem(prob, mlp=p.astype(np.float64))
        W0 = prob.W
        dt, lam = o.dt(W0, prob.cfl)
        s = H.Solver(prob, mlp=p)
        s.set_slot(dt, lam)
        Wn = s.W.clone()
        Ws, Wo = Wn, W0
        N, D = prob.N, prob.D
        for k in range(3):
            ref = o.stage(k, W0, Wo, dt, lam)
            got = s.stage(k, Wn, Ws)
            torch.cuda.synchronize()
            g = got.cpu().numpy()
            # scales as in the parity tests: momentum against max(rho) max(|u| + c)
            sc = np.abs(ref.reshape(prob.M, -1)).max(axis=1)
            sc[N:N + D] = np.maximum(sc[N:N + D], ref[:N].sum(axis=0).max() * o.max_wavespeed(W0).max())
            sc[N + D + 1:] = 1.0
            err = (np.abs(g - ref).reshape(prob.M, -1).max(axis=1) / np.maximum(sc, 1e-300))
            med = (np.abs(g - ref).reshape(prob.M, -1) / np.maximum(sc, 1e-300)[:, None])
            print(f"{prob.name} stage {k}: max rel {err.max():.2e}, median {np.median(med):.2e}")
            assert np.median(med) <= 1e-12
            assert err.max() <= 1e-4, (prob.name, k, err)
            Wo = ref
            Ws = torch.from_numpy(ref).cuda()
        s.close()


def test_non_finite_weights_fall_back_to_app_c(H, M):
    """A network that yields NaN weights everywhere: every stencil falls back
    to the App. C interpolation, so the step equals the plain one to round-off
    (the two kernels are separate compilations of the same arithmetic; a
    learned interpolation would differ at the percent level)."""
    import torch
    p = rand_params(M, 8, 1.0)
    p[1344] = np.nan
    prob = I.config1(300)
    a = H.Solver(prob, mlp=p)
    b = H.Solver(prob)
    for _ in range(3):
        a.step(cfl=prob.cfl)
        b.step(cfl=prob.cfl)
    torch.cuda.synchronize()
    wa, wb = a.state().reshape(prob.M, -1), b.state().reshape(prob.M, -1)
    err = (np.abs(wa - wb).max(axis=1) / np.maximum(np.abs(wb).max(axis=1), 1e-300))
    err[prob.N] = np.abs(wa[prob.N] - wb[prob.N]).max() / (wb[:prob.N].sum(axis=0).max() * 2000.0)
    print("fallback vs plain: max rel per component", err)
    assert np.isfinite(wa).all() and err.max() <= 1e-12
    a.close()
    b.close()


@pytest.fixture(scope="module")
def trained(H):
    from paper_2208_04488_amd import learned
    fine = learned.fine_ensemble(nprob=256, nmin=100, nmax=400, seed=4301)
    X, T = learned.training_data(fine, snapshots=(30, 90))
    p0 = learned.init_params(0, last_scale=0.0)
    l0 = learned.mean_loss(p0, X, T)
    p, hist = learned.train(X, T, steps=1500, count=16384, lr=2e-3, seed=0, log_every=500)
    l1 = learned.mean_loss(p, X, T)
    held = learned.fine_ensemble(nprob=128, nmin=100, nmax=400, seed=4302)
    Xh, Th = learned.training_data(held, snapshots=(60,))
    return dict(p=p, loss_linear=l0, loss=l1, hist=hist, held_linear=learned.mean_loss(p0, Xh, Th),
                held=learned.mean_loss(p, Xh, Th), n=X.shape[0])


def test_training_lowers_the_interpolation_loss(trained):
    t = trained
    print(f"{t['n']} pairs; loss with the classical weights {t['loss_linear']:.4e} -> trained {t['loss']:.4e}; "
          f"held-out {t['held_linear']:.4e} -> {t['held']:.4e}; history {t['hist']}")
    # the best convex combination of the candidates for every pair is about
    # 40% below the linear weights on such data, the classical weights (the
    # starting point here) a few per cent; the network, which may rescale
    # each classical weight by at most e, gets a few per cent further
    assert t["loss"] < 0.97 * t["loss_linear"]
    assert t["held"] < 0.98 * t["held_linear"]


def test_learned_gain_on_config1(H, trained):
    """The gain test: config-1 shock tube (400 cells, to 240 us) with the
    trained weights against the plain method, L1 of the density against the
    exact solution; positivity must hold with the limiters untouched."""
    import torch
    from oracle import exact_riemann as ER
    prob = I.config1(400)
    eos = prob.eos
    L = dict(rho=1000.0, u=0.0, p=1e9, gamma=eos.gamma[0], pinf=eos.pinf[0])
    R = dict(rho=50.0, u=0.0, p=1e5, gamma=eos.gamma[1], pinf=0.0)
    rex, _, _ = ER.solve(prob.centres(0), prob.t_end, 0.7, L, R)
    res = {}
    for name, mlp in (("plain", None), ("learned", trained["p"])):
        s = H.Solver(prob, mlp=mlp)
        k = 0
        while True:
            s.step(cfl=prob.cfl, t_end=prob.t_end)
            k += 1
            if k % 50 == 0:
                torch.cuda.synchronize()
                if s.slot[4].item() >= prob.t_end:
                    break
        w, d = s.state(), s.diagnostics()
        s.close()
        rho = w[:2].sum(axis=0)[0, 0]
        res[name] = (np.abs(rho - rex).sum() * prob.dx[0], d["relax_bad"], w)
    print(f"config1 L1(rho) vs exact: plain {res['plain'][0]:.6e}, learned {res['learned'][0]:.6e}")
    w = res["learned"][2]
    assert res["learned"][1] == 0 and np.isfinite(w).all() and (w[:2] >= 0).all()
    assert res["learned"][0] <= 1.5 * res["plain"][0]


def test_learned_gain_on_config5_full_size(H, trained):
    """The learned-weight workload at full size: the planar config-1 shock
    tube on 2048 x 1024 cells to 240 us.  Every row must stay the same (the
    problem is planar and y is periodic); L1 of the density of a row against
    the exact solution for both methods."""
    import torch
    from oracle import exact_riemann as ER
    prob = I.config5()
    eos = prob.eos
    L = dict(rho=1000.0, u=0.0, p=1e9, gamma=eos.gamma[0], pinf=eos.pinf[0])
    R = dict(rho=50.0, u=0.0, p=1e5, gamma=eos.gamma[1], pinf=0.0)
    x = (np.arange(prob.n[0]) + 0.5) * prob.dx[0]
    rex, _, _ = ER.solve(x, prob.t_end, 0.7, L, R)
    res = {}
    for name, mlp in (("plain", None), ("learned", trained["p"])):
        s = H.Solver(prob, mlp=mlp)
        k = 0
        while True:
            s.step(cfl=prob.cfl, t_end=prob.t_end)
            k += 1
            if k % 200 == 0:
                torch.cuda.synchronize()
                if s.slot[4].item() >= prob.t_end:
                    break
        w, d = s.state(), s.diagnostics()
        s.close()
        rho = w[:2].sum(axis=0)[0]
        assert d["relax_bad"] == 0 and np.isfinite(w).all() and (w[:2] >= 0).all()
        assert np.abs(rho - rho[0]).max() <= 1e-9 * rho.max(), name   # rows identical
        res[name] = np.abs(rho[0] - rex).sum() * prob.dx[0]
        print(f"config5 {name}: {k} steps, L1(rho) vs exact {res[name]:.6e}")
    # reported, not a win: at 2048 cells the plain method is ahead by about 10%
    # (at 400 cells the learned weights are ahead by about 4%)
    assert res["learned"] <= 1.25 * res["plain"]
