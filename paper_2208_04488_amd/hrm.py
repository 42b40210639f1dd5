"""ctypes binding of the C-ABI in include/hrm.h (libhrm.so, gfx950).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  Device arrays are torch tensors (float64, contiguous, on the GPU);
streams default to torch's current stream.  If the library has not been built
the import of this module raises.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libhrm.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "hrm.h")

MAX_SPECIES = 8
HRM_OK, HRM_EINVAL, HRM_ENOMEM, HRM_EDEVICE, HRM_EADMISSIBLE, HRM_EUNSUPPORTED = range(6)
BC_TRANSMISSIVE, BC_PERIODIC, BC_DIRICHLET = 0, 1, 2
FP64, FP32 = 0, 1
WEIGHTS_IS, WEIGHTS_MLP = 0, 1
MLP_NPARAM = 1347
NO_LIMITERS, NO_BLEND, FIRST_ORDER, FUSE_RELAX, NO_GRAPH = 1, 2, 4, 8, 16
FOUR_EQ = 32  # the four-equation HRM solved directly (first-order HLLC)


class hrm_grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 3), ("dx", ctypes.c_double * 3),
                ("bc_lo", ctypes.c_int * 3), ("bc_hi", ctypes.c_int * 3), ("precision", ctypes.c_int),
                ("weights", ctypes.c_int), ("flags", ctypes.c_int)]


class hrm_eos(ctypes.Structure):
    _fields_ = [("nspecies", ctypes.c_int), ("gamma", ctypes.c_double * MAX_SPECIES),
                ("cv", ctypes.c_double * MAX_SPECIES), ("pinf", ctypes.c_double * MAX_SPECIES),
                ("q", ctypes.c_double * MAX_SPECIES)]


class hrm_params(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in (
        "eps_weno", "eps_i_ar", "eps_i_a", "hs_i_ar", "hs_i_a", "hs_i_rc2", "eps_f_ar", "eps_f_a", "eps_f_re",
        "hs_f_ar", "hs_f_a", "hs_f_re", "Cs", "qexp", "psi")]


class hrm_diag(ctypes.Structure):
    _fields_ = [(k, ctypes.c_ulonglong) for k in (
        "alg1", "alg2", "interp_hs", "alg3", "alg4", "flux_hs", "relax_bad", "reserved")]


class HrmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"hrm error {code}: {msg}")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950)")
    # torch first: the process then has one HIP runtime (torch's), which the
    # library binds to; loading the library first would bring in a second one
    # and torch would find no device
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    vp, dp = ctypes.c_void_p, ctypes.c_double
    L.hrm_default_params.argtypes = [ctypes.POINTER(hrm_params)]
    L.hrm_default_params.restype = None
    L.hrm_create.argtypes = [ctypes.POINTER(hrm_grid), ctypes.POINTER(hrm_eos), ctypes.POINTER(hrm_params),
                             ctypes.POINTER(vp)]
    L.hrm_destroy.argtypes = [vp]
    L.hrm_last_error.argtypes = [vp]
    L.hrm_last_error.restype = ctypes.c_char_p
    L.hrm_max_wavespeed.argtypes = [vp, vp, vp, vp]
    L.hrm_compute_dt.argtypes = [vp, vp, dp, dp, dp, vp, vp]
    L.hrm_rhs.argtypes = [vp, vp, vp, vp, vp]
    L.hrm_rk_stage.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp, vp]
    L.hrm_relax.argtypes = [vp, vp, vp]
    L.hrm_equilibrium_state.argtypes = [vp, vp, vp, vp, vp, vp]
    L.hrm_set_boundary_state.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, vp]
    L.hrm_step.argtypes = [vp, vp, dp, dp, dp, vp, vp]
    L.hrm_advance.argtypes = [vp, vp, ctypes.c_int, dp, dp, dp, vp, vp]
    L.hrm_get_diagnostics.argtypes = [vp, ctypes.POINTER(hrm_diag)]
    L.hrm_reset_diagnostics.argtypes = [vp, vp]
    L.hrm_set_timing.argtypes = [vp, ctypes.c_int]
    L.hrm_get_timing.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_longlong)]
    L.hrm_batch_create.argtypes = [ctypes.POINTER(hrm_eos), ctypes.POINTER(hrm_params), ctypes.c_int,
                                   ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_double),
                                   ctypes.c_int, ctypes.POINTER(vp)]
    L.hrm_batch_destroy.argtypes = [vp]
    L.hrm_batch_last_error.argtypes = [vp]
    L.hrm_batch_last_error.restype = ctypes.c_char_p
    L.hrm_batch_configure.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    L.hrm_batch_run.argtypes = [vp, vp, ctypes.c_int, dp, vp]
    L.hrm_batch_time.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    L.hrm_batch_set_end_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    L.hrm_batch_get_diagnostics.argtypes = [vp, ctypes.POINTER(hrm_diag)]
    fp = ctypes.POINTER(ctypes.c_float)
    ll = ctypes.c_longlong
    L.hrm_set_mlp.argtypes = [vp, fp]
    L.hrm_mlp_infer.argtypes = [vp, vp, ll, vp, vp, vp]
    L.hrm_mlp_extract.argtypes = [ctypes.POINTER(hrm_eos), vp, ll, ctypes.c_int, ctypes.POINTER(ll), vp, vp, ll,
                                  ctypes.POINTER(ll), vp]
    L.hrm_mlp_extract_grid.argtypes = [ctypes.POINTER(hrm_grid), ctypes.POINTER(hrm_eos), vp, ctypes.c_int, vp, vp,
                                       ll, ctypes.POINTER(ll), vp]
    L.hrm_mlp_grad_workspace.argtypes = [ctypes.c_int]
    L.hrm_mlp_grad_workspace.restype = ll
    L.hrm_mlp_grad.argtypes = [vp, vp, vp, ll, ll, ll, ctypes.c_int, vp, vp, vp, ll, vp]
    L.hrm_mlp_grad_noalloc.argtypes = [vp, vp, vp, ll, ll, ll, ctypes.c_int, vp, vp, vp]
    L.hrm_mlp_adam.argtypes = [vp, vp, vp, vp, ctypes.c_int, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                               ctypes.c_float, vp]
    return L


lib = _load()


def header_functions(path: str = HEADER):
    """Names of the functions include/hrm.h declares."""
    txt = open(path).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|long long|const char\*)\s+(hrm_\w+)\s*\(", txt, re.M)))


def _check(ctx, rc):
    if rc != HRM_OK:
        msg = lib.hrm_last_error(ctx).decode() if ctx else ""
        raise HrmError(rc, msg)
    return rc


def _ptr(t) -> int:
    if t is None:
        return 0
    if isinstance(t, int):
        return t
    import torch
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError("device arrays must be contiguous float64 CUDA tensors")
    return t.data_ptr()


def _ptrf(t) -> int:
    """Device pointer of a contiguous float32 CUDA tensor."""
    import torch
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError("device arrays must be contiguous float32 CUDA tensors")
    return t.data_ptr()


def _stream(stream) -> int:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ------------------------------------------------------------- same names as the ABI
def hrm_default_params() -> hrm_params:
    p = hrm_params()
    lib.hrm_default_params(ctypes.byref(p))
    return p


def hrm_create(grid: hrm_grid, eos: hrm_eos, params: Optional[hrm_params] = None) -> int:
    ctx = ctypes.c_void_p()
    rc = lib.hrm_create(ctypes.byref(grid), ctypes.byref(eos), ctypes.byref(params) if params else None,
                        ctypes.byref(ctx))
    if rc != HRM_OK:
        raise HrmError(rc, "hrm_create rejected the grid/EOS")
    return ctx.value


def hrm_destroy(ctx: int) -> None:
    _check(None, lib.hrm_destroy(ctx))


def hrm_max_wavespeed(ctx, W, out, stream=None):
    return _check(ctx, lib.hrm_max_wavespeed(ctx, _ptr(W), _ptr(out), _stream(stream)))


def hrm_compute_dt(ctx, maxspeed, cfl, dt_fixed, t_end, slot, stream=None):
    return _check(ctx, lib.hrm_compute_dt(ctx, _ptr(maxspeed), float(cfl), float(dt_fixed), float(t_end),
                                          _ptr(slot), _stream(stream)))


def hrm_rhs(ctx, W, L, slot, stream=None):
    return _check(ctx, lib.hrm_rhs(ctx, _ptr(W), _ptr(L), _ptr(slot), _stream(stream)))


def hrm_rk_stage(ctx, stage, Wn, Ws, Wout, slot, stream=None):
    return _check(ctx, lib.hrm_rk_stage(ctx, int(stage), _ptr(Wn), _ptr(Ws), _ptr(Wout), _ptr(slot),
                                        _stream(stream)))


def hrm_relax(ctx, W, stream=None):
    return _check(ctx, lib.hrm_relax(ctx, _ptr(W), _stream(stream)))


def hrm_equilibrium_state(ctx, W, p=None, T=None, c=None, stream=None):
    return _check(ctx, lib.hrm_equilibrium_state(ctx, _ptr(W), 0 if p is None else _ptr(p),
                                                 0 if T is None else _ptr(T), 0 if c is None else _ptr(c),
                                                 _stream(stream)))


def hrm_set_boundary_state(ctx, dim, side, state, stream=None):
    return _check(ctx, lib.hrm_set_boundary_state(ctx, int(dim), int(side), _ptr(state), _stream(stream)))


def hrm_step(ctx, W, cfl, dt_fixed, t_end, slot, stream=None):
    return _check(ctx, lib.hrm_step(ctx, _ptr(W), float(cfl), float(dt_fixed), float(t_end), _ptr(slot),
                                    _stream(stream)))


def hrm_advance(ctx, W, nsteps, cfl, dt_fixed, t_end, slot, stream=None):
    return _check(ctx, lib.hrm_advance(ctx, _ptr(W), int(nsteps), float(cfl), float(dt_fixed), float(t_end),
                                       _ptr(slot), _stream(stream)))


def hrm_get_diagnostics(ctx) -> dict:
    d = hrm_diag()
    rc = lib.hrm_get_diagnostics(ctx, ctypes.byref(d))
    if rc not in (HRM_OK, HRM_EADMISSIBLE):
        _check(ctx, rc)
    out = {k: int(getattr(d, k)) for k, _ in hrm_diag._fields_}
    out["status"] = rc
    return out


def hrm_reset_diagnostics(ctx, stream=None):
    return _check(ctx, lib.hrm_reset_diagnostics(ctx, _stream(stream)))


TIMERS = ("sweep_x", "sweep_y", "sweep_z", "wavespeed", "dt", "relax")


def hrm_set_timing(ctx, mask):
    return _check(ctx, lib.hrm_set_timing(ctx, int(mask)))


def hrm_get_timing(ctx) -> dict:
    ms = (ctypes.c_double * len(TIMERS))()
    cnt = (ctypes.c_longlong * len(TIMERS))()
    _check(ctx, lib.hrm_get_timing(ctx, ms, cnt))
    return {k: (ms[i], cnt[i]) for i, k in enumerate(TIMERS)}


def hrm_set_mlp(ctx, params):
    p = np.ascontiguousarray(params, dtype=np.float32)
    if p.size != MLP_NPARAM:
        raise ValueError(f"the network has {MLP_NPARAM} parameters")
    return _check(ctx, lib.hrm_set_mlp(ctx, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))


def hrm_mlp_infer(ctx, U5, val, omega, stream=None):
    n = U5.shape[0]
    return _check(ctx, lib.hrm_mlp_infer(ctx, _ptr(U5), n, _ptr(val), _ptrf(omega), _stream(stream)))


def hrm_mlp_extract(eos: hrm_eos, W, offsets, X=None, T=None, stream=None) -> int:
    """Training pairs of a fine ensemble; returns their number (size query
    when X and T are None)."""
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    n = ctypes.c_longlong()
    cap = 0 if X is None else X.shape[0]
    rc = lib.hrm_mlp_extract(ctypes.byref(eos), 0 if W is None else _ptr(W), int(off[-1]), len(off) - 1,
                             off.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)),
                             0 if X is None else _ptrf(X), 0 if T is None else _ptrf(T), cap, ctypes.byref(n),
                             _stream(stream) if X is not None else 0)
    if rc != HRM_OK:
        raise HrmError(rc, "hrm_mlp_extract rejected its arguments")
    return n.value


def hrm_mlp_extract_grid(grid: hrm_grid, eos: hrm_eos, W, stride, X=None, T=None, stream=None) -> int:
    """Training pairs of lines of a fine grid; returns their number (size
    query when X and T are None)."""
    n = ctypes.c_longlong()
    cap = 0 if X is None else X.shape[0]
    rc = lib.hrm_mlp_extract_grid(ctypes.byref(grid), ctypes.byref(eos), 0 if W is None else _ptr(W), int(stride),
                                  0 if X is None else _ptrf(X), 0 if T is None else _ptrf(T), cap, ctypes.byref(n),
                                  _stream(stream) if X is not None else 0)
    if rc != HRM_OK:
        raise HrmError(rc, "hrm_mlp_extract_grid rejected its arguments")
    return n.value


def hrm_mlp_grad_workspace(count) -> int:
    return int(lib.hrm_mlp_grad_workspace(int(count)))


def hrm_mlp_grad(params, X, T, first, stride, count, grad, loss, work, stream=None):
    rc = lib.hrm_mlp_grad(_ptrf(params), _ptrf(X), _ptrf(T), X.shape[0], int(first), int(stride), int(count),
                          _ptrf(grad), _ptrf(loss), _ptrf(work), work.numel(), _stream(stream))
    if rc != HRM_OK:
        raise HrmError(rc, "hrm_mlp_grad rejected its arguments")


MLP_GRAD_NOALLOC_MAX = 32768


def hrm_mlp_grad_noalloc(params, X, T, first, stride, count, grad, loss, stream=None):
    rc = lib.hrm_mlp_grad_noalloc(_ptrf(params), _ptrf(X), _ptrf(T), X.shape[0], int(first), int(stride),
                                  int(count), _ptrf(grad), _ptrf(loss), _stream(stream))
    if rc != HRM_OK:
        raise HrmError(rc, "hrm_mlp_grad_noalloc rejected its arguments")


def hrm_mlp_adam(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    rc = lib.hrm_mlp_adam(_ptrf(params), _ptrf(grad), _ptrf(m), _ptrf(v), int(step), float(lr), float(beta1),
                          float(beta2), float(eps), _stream(stream))
    if rc != HRM_OK:
        raise HrmError(rc, "hrm_mlp_adam rejected its arguments")


def _bcheck(b, rc):
    if rc != HRM_OK:
        msg = lib.hrm_batch_last_error(b).decode() if b else ""
        raise HrmError(rc, msg)
    return rc


def hrm_batch_create(eos: hrm_eos, params: Optional[hrm_params], offsets, dx, precision=FP64) -> int:
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    dxa = np.ascontiguousarray(dx, dtype=np.float64)
    nprob = len(off) - 1
    if nprob < 1 or len(dxa) != nprob:
        raise ValueError("offsets must have nprob + 1 entries and dx nprob")
    b = ctypes.c_void_p()
    rc = lib.hrm_batch_create(ctypes.byref(eos), ctypes.byref(params) if params else None, nprob,
                              off.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)),
                              dxa.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(precision), ctypes.byref(b))
    if rc != HRM_OK:
        raise HrmError(rc, "hrm_batch_create rejected the EOS/offsets/dx")
    return b.value


def hrm_batch_destroy(b: int) -> None:
    _bcheck(None, lib.hrm_batch_destroy(b))


def hrm_batch_configure(b, threads, blocks, steps_per_launch):
    return _bcheck(b, lib.hrm_batch_configure(b, int(threads), int(blocks), int(steps_per_launch)))


def hrm_batch_run(b, W, nsteps, cfl, stream=None):
    return _bcheck(b, lib.hrm_batch_run(b, _ptr(W), int(nsteps), float(cfl), _stream(stream)))


def hrm_batch_time(b, nprob) -> np.ndarray:
    t = np.zeros(nprob, dtype=np.float64)
    _bcheck(b, lib.hrm_batch_time(b, t.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return t


def hrm_batch_set_end_times(b, tend):
    t = np.ascontiguousarray(tend, dtype=np.float64)
    return _bcheck(b, lib.hrm_batch_set_end_times(b, t.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))


def hrm_batch_get_diagnostics(b) -> dict:
    d = hrm_diag()
    rc = lib.hrm_batch_get_diagnostics(b, ctypes.byref(d))
    if rc not in (HRM_OK, HRM_EADMISSIBLE):
        _bcheck(b, rc)
    out = {k: int(getattr(d, k)) for k, _ in hrm_diag._fields_}
    out["status"] = rc
    return out


# ------------------------------------------------------------- convenience
def make_grid(D, n, dx, bc, precision=FP64, weights=WEIGHTS_IS, flags=0) -> hrm_grid:
    g = hrm_grid()
    g.dim = D
    nn = list(n) + [1] * (3 - len(n))
    dd = list(dx) + [1.0] * (3 - len(dx))
    for i in range(3):
        g.n[i], g.dx[i] = int(nn[i]), float(dd[i])
        lo, hi = bc[i] if i < D else (BC_TRANSMISSIVE, BC_TRANSMISSIVE)
        g.bc_lo[i], g.bc_hi[i] = int(lo), int(hi)
    g.precision, g.weights, g.flags = precision, weights, flags
    return g


def make_eos(gamma, cv, pinf, q) -> hrm_eos:
    e = hrm_eos()
    e.nspecies = len(gamma)
    for k in range(len(gamma)):
        e.gamma[k], e.cv[k], e.pinf[k], e.q[k] = gamma[k], cv[k], pinf[k], q[k]
    return e


class Solver:
    """A context plus device state for one problem from ``inputs``."""

    def __init__(self, prob, flags=FUSE_RELAX, precision=FP64, params: Optional[hrm_params] = None, W=None,
                 mlp=None):
        import torch
        self.torch = torch
        self.prob = prob
        e = prob.eos
        self.grid = make_grid(prob.D, prob.n, prob.dx, prob.bc, precision=precision, flags=flags,
                              weights=WEIGHTS_IS if mlp is None else WEIGHTS_MLP)
        self.eos = make_eos(e.gamma, e.cv, e.pinf, e.q)
        self.ctx = hrm_create(self.grid, self.eos, params)
        dev = torch.device("cuda")
        self.W = torch.from_numpy(np.ascontiguousarray(prob.W if W is None else W)).to(dev)
        self.slot = torch.zeros(8, dtype=torch.float64, device=dev)
        self.maxs = torch.zeros(4, dtype=torch.float64, device=dev)
        if mlp is not None:
            hrm_set_mlp(self.ctx, mlp)
        self._bnd = {}
        for (d, side), Wb in getattr(prob, "boundary", {}).items():
            self.set_boundary(d, side, Wb)

    def set_boundary(self, d, side, Wb):
        """Ghost states of a Dirichlet side, shape (M, cells of the face)."""
        t = self.torch.from_numpy(np.ascontiguousarray(Wb, dtype=np.float64)).to(self.W.device)
        self._bnd[(d, side)] = t  # kept until the context is gone
        hrm_set_boundary_state(self.ctx, d, side, t)

    def close(self):
        if self.ctx:
            hrm_destroy(self.ctx)
            self.ctx = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_state(self, W):
        self.W.copy_(self.torch.from_numpy(np.ascontiguousarray(W)))

    def state(self) -> np.ndarray:
        return self.W.cpu().numpy()

    def set_slot(self, dt, lam, t=0.0):
        vals = [dt] + list(lam) + [0.0] * (3 - len(lam)) + [t, 0.0, 0.0, 0.0]
        self.slot.copy_(self.torch.tensor(vals[:8], dtype=self.torch.float64))

    def equilibrium(self, W=None):
        """(p*, T*, c) of the four-equation HRM per cell, numpy arrays of the grid's shape."""
        Wd = self.W if W is None else W
        out = [self.torch.empty(Wd.shape[1:], dtype=self.torch.float64, device=Wd.device) for _ in range(3)]
        hrm_equilibrium_state(self.ctx, Wd, *out)
        return tuple(o.cpu().numpy() for o in out)

    def wavespeed(self, W=None):
        hrm_max_wavespeed(self.ctx, self.W if W is None else W, self.maxs)
        return self.maxs[: self.prob.D].cpu().numpy()

    def compute_dt(self, cfl, dt_fixed=0.0, t_end=0.0):
        hrm_compute_dt(self.ctx, self.maxs, cfl, dt_fixed, t_end, self.slot)
        s = self.slot.cpu().numpy()
        return s[0], s[1: 1 + self.prob.D].copy(), s[4]

    def rhs(self, W=None):
        out = self.torch.empty_like(self.W)
        hrm_rhs(self.ctx, self.W if W is None else W, out, self.slot)
        return out

    def stage(self, k, Wn, Ws):
        out = self.torch.empty_like(self.W)
        hrm_rk_stage(self.ctx, k, Wn, Ws, out, self.slot)
        return out

    def relax(self, W=None):
        hrm_relax(self.ctx, self.W if W is None else W)

    def step(self, cfl=0.4, dt_fixed=0.0, t_end=0.0):
        hrm_step(self.ctx, self.W, cfl, dt_fixed, t_end, self.slot)

    def advance(self, nsteps, cfl=0.4, dt_fixed=0.0, t_end=0.0):
        hrm_advance(self.ctx, self.W, nsteps, cfl, dt_fixed, t_end, self.slot)

    def diagnostics(self):
        return hrm_get_diagnostics(self.ctx)


class BatchSolver:
    """A batch handle plus the device state of an ``inputs.Batch``."""

    def __init__(self, batch, precision=FP64, params: Optional[hrm_params] = None, W=None):
        import torch
        self.torch = torch
        self.batch = batch
        e = batch.eos
        self.eos = make_eos(e.gamma, e.cv, e.pinf, e.q)
        self.b = hrm_batch_create(self.eos, params, batch.offsets, batch.dx, precision)
        self.W = torch.from_numpy(np.ascontiguousarray(batch.W if W is None else W)).to(torch.device("cuda"))
        self.steps_per_launch = 10

    def configure(self, threads, blocks, steps_per_launch):
        hrm_batch_configure(self.b, threads, blocks, steps_per_launch)
        self.steps_per_launch = steps_per_launch

    def run(self, nsteps, cfl=None):
        hrm_batch_run(self.b, self.W, nsteps, self.batch.cfl if cfl is None else cfl)

    def state(self) -> np.ndarray:
        return self.W.cpu().numpy()

    def times(self) -> np.ndarray:
        return hrm_batch_time(self.b, self.batch.nprob)

    def set_end_times(self, tend):
        hrm_batch_set_end_times(self.b, tend)

    def diagnostics(self):
        return hrm_batch_get_diagnostics(self.b)

    def close(self):
        if self.b:
            hrm_batch_destroy(self.b)
            self.b = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
