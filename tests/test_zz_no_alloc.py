"""hrm_mlp_grad_noalloc: the gradient of the learned weights with its
per-workgroup partials in the library's fixed device array instead of a
caller's workspace.  Through the C ABI it must equal hrm_mlp_grad bit for bit
(the same kernels in the same order), call after call on the shared array,
a smaller minibatch after a larger one included, and reject minibatches above
its maximum."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _data(n, seed):
    import torch
    rng = np.random.default_rng(seed)
    X = np.zeros((n, 8), np.float32)
    X[:, :5] = rng.uniform(-1.0, 1.0, (n, 5))
    X[:, 2] = 0.0  # normalised stencils are zero at node i
    T = rng.uniform(-1.5, 1.5, n).astype(np.float32)
    return torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()


def test_noalloc_gradient_equals_workspace_gradient():
    import torch
    from paper_2208_04488_amd import hrm, learned
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    X, T = _data(50000, 11)
    p = torch.from_numpy(learned.init_params(3, last_scale=0.5)).cuda()
    for count, first, stride in ((hrm.MLP_GRAD_NOALLOC_MAX, 5, 1), (20000, 123, 2), (777, 9, 61)):
        g_ref = torch.zeros(hrm.MLP_NPARAM, dtype=torch.float32, device="cuda")
        l_ref = torch.zeros(1, dtype=torch.float32, device="cuda")
        work = torch.zeros(hrm.hrm_mlp_grad_workspace(count), dtype=torch.float32, device="cuda")
        hrm.hrm_mlp_grad(p, X, T, first, stride, count, g_ref, l_ref, work)
        g = torch.full_like(g_ref, float("nan"))
        l = torch.full_like(l_ref, float("nan"))
        hrm.hrm_mlp_grad_noalloc(p, X, T, first, stride, count, g, l)
        torch.cuda.synchronize()
        print(f"count {count}: loss {l.item():.6e}, |grad| {g.norm().item():.6e}")
        assert torch.isfinite(g).all() and torch.isfinite(l).all()
        assert torch.equal(g, g_ref) and torch.equal(l, l_ref), count


def test_noalloc_gradient_rejects_oversize_minibatch():
    import torch
    from paper_2208_04488_amd import hrm, learned
    X, T = _data(1000, 12)
    p = torch.from_numpy(learned.init_params(4)).cuda()
    g = torch.zeros(hrm.MLP_NPARAM, dtype=torch.float32, device="cuda")
    l = torch.zeros(1, dtype=torch.float32, device="cuda")
    with pytest.raises(hrm.HrmError):
        hrm.hrm_mlp_grad_noalloc(p, X, T, 0, 1, hrm.MLP_GRAD_NOALLOC_MAX + 1, g, l)
    with pytest.raises(hrm.HrmError):
        hrm.hrm_mlp_grad_noalloc(p, X, T, 0, 1, 0, g, l)
