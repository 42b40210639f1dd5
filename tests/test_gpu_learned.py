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
    assert np.abs(om - ref).max() <= 1e-6  # float weights against double: measured 1.3e-7


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
    # measured: median 3.1e-8, 99.9 % 1.5e-7, max 1.9e-7 (no bfloat16 flip in this data)
    assert np.median(dw) <= 3e-7
    assert np.quantile(dw, 0.99) <= 1e-6
    assert dw.max() <= 2e-6
    spread = np.abs(U - U[:, 2:3]).max(axis=1)
    # relative to the stencil's spread (round-off of the candidates for constant ones)
    dv = np.abs(val - ref_v) / np.maximum(spread, 1e-14 * np.abs(U).max(axis=1))
    print("value |diff| / spread: median %.2e  max %.2e" % (np.median(dv), dv.max()))
    # measured: median 3.9e-11; max 2.2e-2 on near-constant stencils (spread
    # 1e-9 of the values), where it is the candidates' round-off, not the weights
    assert np.median(dv) <= 4e-10 and dv.max() <= 5e-2
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
        assert err <= 5e-6 and lerr <= 3e-7  # measured up to 6.8e-7 and 3.2e-8


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
    err = np.abs(g.cpu().numpy() - gref).max() / np.abs(gref).max()
    print(f"strided minibatch: grad rel err {err:.2e}")
    assert err <= 5e-6


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
    err = np.abs(tp.cpu().numpy() - rp).max()
    print(f"Adam: max |diff| {err:.2e}")
    assert err <= 1e-6


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


def _stencil_amplification(f):
    """max |u_j| / spread of each stencil of the injection recipe (the
    left-biased ones, then the mirrored ones, as the pairs are ordered)."""
    c = np.asarray(f, dtype=np.float64)[0::2]
    n = c.size
    U = [c[j - 2:j + 3] for j in range(2, n - 2)] + [c[j - 1:j + 4][::-1] for j in range(1, n - 3)]
    U = np.array(U)
    s = np.abs(U - U[:, 2:3]).max(axis=1)
    return np.abs(U).max(axis=1) / np.maximum(s, 1e-300)


@pytest.mark.parametrize("case", ["config3_24", "config2_30x22"])
def test_grid_extraction_matches_oracle(H, M, orc, case):
    """Training pairs from lines of a fine grid (3D multimode interface at
    24^3 after two steps, every 5th line; a 2D liquid column with an odd
    direction that gives no lines) against the oracle's injection recipe
    applied to each line's primitive fields."""
    import torch
    prob = I.config3(24) if case == "config3_24" else I.config2(30, 23)
    stride = 5 if case == "config3_24" else 3
    o = orc.from_problem(prob)
    W = prob.W
    for _ in range(2):
        W, _ = o.step(W, cfl=prob.cfl)
    e = prob.eos
    eos = H.make_eos(e.gamma, e.cv, e.pinf, e.q)
    grid = H.make_grid(prob.D, prob.n, prob.dx, prob.bc)
    n = H.hrm_mlp_extract_grid(grid, eos, None, stride)
    X = torch.zeros((n, 8), dtype=torch.float32, device="cuda")
    T = torch.zeros(n, dtype=torch.float32, device="cuda")
    assert H.hrm_mlp_extract_grid(grid, eos, torch.from_numpy(W).cuda(), stride, X, T) == n
    torch.cuda.synchronize()
    X, T = X.cpu().numpy(), T.cpu().numpy()
    Nsp, D = prob.N, prob.D
    nn = list(prob.n) + [1] * (3 - D)
    Wg = W.reshape(W.shape[0], nn[2], nn[1], nn[0])  # (M, z, y, x)
    pos = 0
    for d in range(D):
        if nn[d] % 2 or nn[d] // 2 < 5:
            continue
        ta, tb = (1, 2) if d == 0 else ((0, 2) if d == 1 else (0, 1))
        for ib in range(0, nn[tb], stride):
            for ia in range(0, nn[ta], stride):
                idx = [0, 0, 0]
                idx[ta], idx[tb] = ia, ib
                cells = []
                for i in range(nn[d]):
                    idx[d] = i
                    cells.append(Wg[:, idx[2], idx[1], idx[0]])
                line = np.array(cells).T  # (M, cells)
                prim = [o.prim(line[:, i]) for i in range(line.shape[1])]
                fields = [line[k] for k in range(Nsp)] + \
                         [np.array([q["u"][c] for q in prim]) for c in range(D)] + \
                         [np.array([q["p"] for q in prim])] + [line[Nsp + D + 1 + k] for k in range(Nsp - 1)]
                for f, fv in enumerate(fields):
                    xr, tr = M.samples_from_fine(fv, keep_degenerate=True)
                    k = len(tr)
                    xg, tg = X[pos:pos + k, :5], T[pos:pos + k]
                    assert (X[pos:pos + k, 5:] == 0).all()
                    if f < Nsp or f > Nsp + D:
                        # partial densities and volume fractions: stored values, the same bits
                        assert np.array_equal(xg, xr.astype(np.float32)), (d, ia, ib, f)
                        assert np.array_equal(tg, tr.astype(np.float32)), (d, ia, ib, f)
                    else:
                        # u and p are formed from W on each side (device and oracle
                        # round differently, up to ~1e-12 relative for p in a liquid,
                        # where p = (rho e - Pi) / Gamma cancels): normalisation by the
                        # stencil's spread s amplifies that by max|u| / s
                        amp = _stencil_amplification(fv)
                        live = amp < 1e6
                        tol = 2e-6 + 1e-11 * amp[live]
                        assert (np.abs(xg[live] - xr[live]).max(axis=1) <= tol).all(), (d, ia, ib, f)
                        assert (np.abs(tg[live] - tr[live]) <= 10 * tol).all(), (d, ia, ib, f)
                        # near-degenerate stencils: a valid normalised pair or a neutral one
                        assert (np.abs(xg[~live]) <= 1.0 + 1e-6).all() and (np.abs(tg[~live]) <= 4.0).all()
                    pos += k
    assert pos == n and n > 0


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
            off = (med.max(axis=0) > 1e-11).mean()
            print(f"{prob.name} stage {k}: max rel {err.max():.2e}, median {np.median(med):.2e}, "
                  f"cells above 1e-11: {100 * off:.2f} %")
            # The two sides differ only where float accumulation moves a hidden
            # activation across a bfloat16 rounding boundary: one bfloat16 step
            # (2^-8) in one unit changes a weight, and the value by that change
            # times the candidates' spread.  Elsewhere the stage agrees to
            # round-off.  Measured: at most 2.1e-7 (config-1 stage 0), 3 % of
            # the cells of the 200-cell tube (6 cells) above 1e-11.
            assert np.median(med) <= 1e-12
            assert off <= 0.05, (prob.name, k, off)
            assert err.max() <= 1e-6, (prob.name, k, err)
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
    assert np.isfinite(wa).all() and err.max() <= 2e-15  # measured 2.3e-16
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


def _three_way(H, prob, trained, check_every):
    """plain (App. C weights), prior (a zero network: the classical WENO5
    weights the network rescales) and trained, each run to the workload's
    end time: (L1 of the density of a row against the exact solution, steps)."""
    import torch
    from oracle import exact_riemann as ER
    from paper_2208_04488_amd import learned
    eos = prob.eos
    L = dict(rho=1000.0, u=0.0, p=1e9, gamma=eos.gamma[0], pinf=eos.pinf[0])
    R = dict(rho=50.0, u=0.0, p=1e5, gamma=eos.gamma[1], pinf=0.0)
    x = (np.arange(prob.n[0]) + 0.5) * prob.dx[0]
    rex, _, _ = ER.solve(x, prob.t_end, 0.7, L, R)
    res = {}
    for name, mlp in (("plain", None), ("prior", learned.init_params(0, last_scale=0.0)), ("trained", trained["p"])):
        s = H.Solver(prob, mlp=mlp)
        k = 0
        while True:
            s.advance(check_every, cfl=prob.cfl, t_end=prob.t_end)
            k += check_every
            torch.cuda.synchronize()
            if s.slot[4].item() >= prob.t_end:
                break
        w, d = s.state(), s.diagnostics()
        s.close()
        rho = w[:prob.N].sum(axis=0).reshape(-1, prob.n[0])
        assert d["relax_bad"] == 0 and np.isfinite(w).all() and (w[:prob.N] >= 0).all(), name
        assert np.abs(rho - rho[0]).max() <= 1e-9 * rho.max(), name   # planar: rows identical
        res[name] = float(np.abs(rho[0] - rex).sum() * prob.dx[0])
    return res


def test_learned_gain_on_config1(H, trained):
    """What the network gains, on the config-1 shock tube (400 cells, to 240
    us): L1 of the density against the exact solution for the plain method,
    the network's prior alone and the trained network, with the positivity
    limiters untouched (every run admissible)."""
    r = _three_way(H, I.config1(400), trained, 100)
    print(f"config1 (400 cells) L1(rho) vs exact: plain {r['plain']:.6e}, prior {r['prior']:.6e}, "
          f"trained {r['trained']:.6e} (trained vs prior {r['trained'] / r['prior'] - 1:+.2%}, "
          f"vs plain {r['trained'] / r['plain'] - 1:+.2%})")


def test_learned_gain_on_config5_full_size(H, trained):
    """The learned-weight workload at full size: the planar config-1 shock
    tube on 2048 x 1024 cells to 240 us, the same three-way comparison (every
    row must stay the same: the problem is planar and y is periodic)."""
    r = _three_way(H, I.config5(), trained, 400)
    print(f"config5 (2048 x 1024) L1(rho) vs exact: plain {r['plain']:.6e}, prior {r['prior']:.6e}, "
          f"trained {r['trained']:.6e} (trained vs prior {r['trained'] / r['prior'] - 1:+.2%}, "
          f"vs plain {r['trained'] / r['plain'] - 1:+.2%})")
