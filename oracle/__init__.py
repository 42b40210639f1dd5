"""CPU oracle for the hot path: one SSP-RK3 stage of the five-equation model with
PP-WCNS-IS plus the infinite-rate thermal relaxation (arXiv:2208.04488).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the HIP library and imports nothing from it.

The arithmetic lives in ``hrm_oracle.c`` (plain C, double precision, built
with ``-O2 -ffp-contract=off``); this module only marshals numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hrm_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")

MAXN = 8
TRANSMISSIVE, PERIODIC, DIRICHLET = 0, 1, 2
NO_LIMITERS, NO_BLEND, FIRST_ORDER = 1, 2, 4
FOUR_EQ = 32  # the four-equation HRM solved directly with first-order HLLC
COUNTERS = ("alg1", "alg2", "interp_hs", "alg3", "alg4", "flux_hs", "relax_bad", "unused")

# tolerances and constants as the paper fixes them (Sec. 4.3, App. C)
PAPER_PARAMS = dict(
    eps_weno=1e-15,
    eps_i_ar=1e-10, eps_i_a=1e-10,
    hs_i_ar=1e-11, hs_i_a=1e-11, hs_i_rc2=1e-9,
    eps_f_ar=1e-10, eps_f_a=1e-10, eps_f_re=1e-8,
    hs_f_ar=1e-11, hs_f_a=1e-11, hs_f_re=1e-9,
    Cs=1e12, qexp=2.0, psi=256.0 / 175.0,
)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-o", _LIB, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
    return _LIB


class Setup(ctypes.Structure):
    _fields_ = [
        ("N", ctypes.c_int), ("D", ctypes.c_int),
        ("n", ctypes.c_int * 3), ("dx", ctypes.c_double * 3),
        ("bc_lo", ctypes.c_int * 3), ("bc_hi", ctypes.c_int * 3),
        ("gamma", ctypes.c_double * MAXN), ("cv", ctypes.c_double * MAXN),
        ("pinf", ctypes.c_double * MAXN), ("q", ctypes.c_double * MAXN),
        ("eps_weno", ctypes.c_double),
        ("eps_i_ar", ctypes.c_double), ("eps_i_a", ctypes.c_double),
        ("hs_i_ar", ctypes.c_double), ("hs_i_a", ctypes.c_double), ("hs_i_rc2", ctypes.c_double),
        ("eps_f_ar", ctypes.c_double), ("eps_f_a", ctypes.c_double), ("eps_f_re", ctypes.c_double),
        ("hs_f_ar", ctypes.c_double), ("hs_f_a", ctypes.c_double), ("hs_f_re", ctypes.c_double),
        ("Cs", ctypes.c_double), ("qexp", ctypes.c_double), ("psi", ctypes.c_double),
        ("flags", ctypes.c_int),
        ("weights", ctypes.c_int), ("mlp", ctypes.POINTER(ctypes.c_double)),
        ("bnd", (ctypes.POINTER(ctypes.c_double) * 2) * 3),
    ]

W_IS, W_MLP = 0, 1
MLP_NPARAM = 1347


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        sp = ctypes.POINTER(Setup)
        lp = ctypes.POINTER(ctypes.c_longlong)
        L.orc_rhs.argtypes = [sp, dp, dp, dp, lp]
        L.orc_relax.argtypes = [sp, dp, lp]
        L.orc_max_wavespeed.argtypes = [sp, dp, dp]
        L.orc_dt.argtypes = [sp, dp, ctypes.c_double, ctypes.c_double, dp]
        L.orc_combine_ab.argtypes = [sp, ctypes.c_double, ctypes.c_double, dp, dp, dp, ctypes.c_double, dp,
                                     ctypes.c_int, lp]
        L.orc_combine.argtypes = [sp, ctypes.c_int, dp, dp, dp, ctypes.c_double, dp, ctypes.c_int, lp]
        L.orc_stage.argtypes = [sp, ctypes.c_int, dp, dp, dp, ctypes.c_double, dp, ctypes.c_int, lp]
        L.orc_prim.argtypes = [sp, dp, dp]
        L.orc_cons_from_prim.argtypes = [sp, dp, dp]
        L.orc_weno.argtypes = [dp, ctypes.c_double]
        L.orc_weno.restype = ctypes.c_double
        L.orc_mlp_interp.argtypes = [dp, dp, dp, dp]
        L.orc_mlp_interp.restype = ctypes.c_int
        L.orc_bf16.argtypes = [ctypes.c_double]
        L.orc_bf16.restype = ctypes.c_double
        L.orc_sensor.argtypes = [dp]
        L.orc_sensor.restype = ctypes.c_double
        L.orc_hllc.argtypes = [sp, ctypes.c_int, dp, dp, dp]
        L.orc_hllc4.argtypes = [sp, ctypes.c_int, dp, dp, dp]
        L.orc_hllc4.restype = ctypes.c_double
        L.orc_hrm_eos.argtypes = [sp, dp, dp]
        L.orc_hllc.restype = ctypes.c_double
        L.orc_project.argtypes = [sp, ctypes.c_int, dp, dp, dp, dp, dp]
        L.orc_face.argtypes = [sp, ctypes.c_int, dp, ctypes.c_double, dp, dp, lp]
        L.orc_interp_limit.argtypes = [sp, dp, dp, lp]
        L.orc_interp_limit.restype = ctypes.c_int
        L.orc_flux_limit.argtypes = [sp, ctypes.c_int, dp, dp, ctypes.c_double, dp, dp, dp, dp, dp, dp, lp]
        L.orc_relax_cell.argtypes = [sp, dp, dp]
        L.orc_relax_cell.restype = ctypes.c_int
        L.orc_hcs_coeffs.argtypes = [ctypes.c_double, dp]
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_set_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


class Oracle:
    """A grid, an EOS table and the paper's parameters, with the oracle's calls.

    ``gamma, cv, pinf, q`` list the N species; species 0 is the only one with
    ``pinf > 0``.  ``bc`` is a list of D pairs (lo, hi) of TRANSMISSIVE,
    PERIODIC or DIRICHLET; ``boundary`` maps (dim, side) of each Dirichlet
    side to its ghost states, shape (M, n_a * n_b) with a < b the other two
    dimensions and index i_a + n_a i_b.
    State arrays are float64 of shape (M, nz, ny, nx), M = 2N + D.
    """

    def __init__(self, N, D, n, dx, bc, gamma, cv, pinf, q, flags=0, mlp=None, boundary=None, **params):
        s = Setup()
        s.N, s.D = N, D
        nn = list(n) + [1] * (3 - len(n))
        dd = list(dx) + [1.0] * (3 - len(dx))
        for i in range(3):
            s.n[i] = int(nn[i])
            s.dx[i] = float(dd[i])
            lo, hi = (bc[i] if i < D else (TRANSMISSIVE, TRANSMISSIVE))
            s.bc_lo[i], s.bc_hi[i] = int(lo), int(hi)
        for k in range(N):
            s.gamma[k], s.cv[k], s.pinf[k], s.q[k] = gamma[k], cv[k], pinf[k], q[k]
        p = dict(PAPER_PARAMS)
        p.update(params)
        for key, val in p.items():
            setattr(s, key, float(val))
        s.flags = int(flags)
        if mlp is not None:
            # learned weights: the parameters stay referenced by this object
            self._mlp = _f64(mlp).copy()
            assert self._mlp.size == MLP_NPARAM
            s.weights, s.mlp = W_MLP, _dp(self._mlp)
        self._bnd = {}
        for i in range(D):
            for side in range(2):
                if (s.bc_lo[i], s.bc_hi[i])[side] != DIRICHLET:
                    continue
                a, b = (1, 2) if i == 0 else ((0, 2) if i == 1 else (0, 1))
                arr = _f64((boundary or {})[(i, side)]).reshape(2 * N + D, -1).copy()
                assert arr.shape[1] == nn[a] * nn[b]
                self._bnd[(i, side)] = arr  # referenced by the setup below
                s.bnd[i][side] = _dp(arr)
        self.s = s
        self.N, self.D, self.M = N, D, 2 * N + D
        self.shape = (self.M, nn[2], nn[1], nn[0])
        self.counters = np.zeros(8, dtype=np.int64)
        self._L = lib()

    # ---- helpers ----
    def _cnt(self):
        return self.counters.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong))

    def counter_dict(self):
        return dict(zip(COUNTERS, self.counters.tolist()))

    @staticmethod
    def set_threads(n: int) -> int:
        return lib().orc_set_threads(int(n))

    # ---- whole-grid calls ----
    def rhs(self, W, lam):
        W = _f64(W)
        out = np.zeros_like(W)
        lam = _f64(list(lam) + [0.0] * (3 - len(lam)))
        self._L.orc_rhs(ctypes.byref(self.s), _dp(W), _dp(lam), _dp(out), self._cnt())
        return out

    def relax(self, W):
        W = _f64(W).copy()
        self._L.orc_relax(ctypes.byref(self.s), _dp(W), self._cnt())
        return W

    def max_wavespeed(self, W):
        W = _f64(W)
        out = np.zeros(3)
        self._L.orc_max_wavespeed(ctypes.byref(self.s), _dp(W), _dp(out))
        return out[: self.D]

    def dt(self, W, cfl, dt_fixed=0.0):
        ms = _f64(list(self.max_wavespeed(W)) + [0.0] * (3 - self.D))
        out = np.zeros(4)
        self._L.orc_dt(ctypes.byref(self.s), _dp(ms), float(cfl), float(dt_fixed), _dp(out))
        return out[0], out[1 : 1 + self.D].copy()

    def combine(self, k, Wn, Ws, L, dt, relax=True):
        """SSP-RK3 stage k combination with a given right-hand side L."""
        Wn, Ws, L = _f64(Wn), _f64(Ws), _f64(L)
        out = np.empty_like(Ws)
        self._L.orc_combine(ctypes.byref(self.s), int(k), _dp(Wn), _dp(Ws), _dp(L), float(dt), _dp(out),
                            int(relax), self._cnt())
        return out

    def combine_ab(self, a, b, Wn, Ws, L, dt, relax=True):
        """W_out = a W^n + b (W^(s) + dt L), then relaxation."""
        Wn, Ws, L = _f64(Wn), _f64(Ws), _f64(L)
        out = np.empty_like(Ws)
        self._L.orc_combine_ab(ctypes.byref(self.s), float(a), float(b), _dp(Wn), _dp(Ws), _dp(L), float(dt),
                               _dp(out), int(relax), self._cnt())
        return out

    def stage(self, k, Wn, Ws, dt, lam, relax=True):
        Wn, Ws = _f64(Wn), _f64(Ws)
        out = np.empty_like(Ws)
        lam = _f64(list(lam) + [0.0] * (3 - len(lam)))
        self._L.orc_stage(ctypes.byref(self.s), int(k), _dp(Wn), _dp(Ws), _dp(out), float(dt), _dp(lam),
                          int(relax), self._cnt())
        return out

    def step(self, Wn, cfl=0.4, dt_fixed=0.0, relax=True, t=None, t_end=None):
        """One SSP-RK3 step; dt and lambda from W^n only (clipped to t_end)."""
        dt, lam = self.dt(Wn, cfl, dt_fixed)
        if t is not None and t_end is not None and t + dt > t_end:
            scale = (t_end - t) / dt
            dt, lam = t_end - t, lam * scale
        W1 = self.stage(0, Wn, Wn, dt, lam, relax)
        W2 = self.stage(1, Wn, W1, dt, lam, relax)
        return self.stage(2, Wn, W2, dt, lam, relax), dt

    def run(self, W, cfl=0.4, t_end=None, nsteps=None, dt_fixed=0.0, relax=True):
        t, k = 0.0, 0
        while True:
            if nsteps is not None and k >= nsteps:
                break
            if t_end is not None and t >= t_end * (1 - 1e-14):
                break
            W, dt = self.step(W, cfl, dt_fixed, relax, t, t_end)
            t += dt
            k += 1
        return W, t, k

    # ---- unit calls ----
    def prim(self, w):
        w = _f64(w)
        out = np.zeros(5 + self.D)
        self._L.orc_prim(ctypes.byref(self.s), _dp(w), _dp(out))
        return dict(rho=out[0], p=out[1], rhoc2=out[2], c=out[3], rhoe_t=out[4], u=out[5:].copy())

    def cons_from_prim(self, v):
        v = _f64(v)
        out = np.zeros(self.M)
        self._L.orc_cons_from_prim(ctypes.byref(self.s), _dp(v), _dp(out))
        return out

    def relax_cell(self, w):
        w = _f64(w).copy()
        pT = np.zeros(2)
        bad = self._L.orc_relax_cell(ctypes.byref(self.s), _dp(w), _dp(pT))
        return w, pT[0], pT[1], bad

    def hllc(self, n, wl, wr):
        G = np.zeros(self.M)
        ss = self._L.orc_hllc(ctypes.byref(self.s), int(n), _dp(_f64(wl)), _dp(_f64(wr)), _dp(G))
        return G, ss

    def hllc4(self, n, wl, wr):
        """First-order HLLC flux of the four-equation HRM (alpha slots zero)."""
        G = np.zeros(self.M)
        ss = self._L.orc_hllc4(ctypes.byref(self.s), int(n), _dp(_f64(wl)), _dp(_f64(wr)), _dp(G))
        return G, ss

    def hrm_eos(self, w):
        """(p, T, c) of the four-equation HRM for one conservative vector (the
        volume fractions are ignored); NaNs outside the admissible set."""
        out = np.zeros(3)
        self._L.orc_hrm_eos(ctypes.byref(self.s), _dp(_f64(w)), _dp(out))
        return out[0], out[1], out[2]

    def project(self, n, wa, wb, v):
        U, Vb = np.zeros(self.M), np.zeros(self.M)
        self._L.orc_project(ctypes.byref(self.s), int(n), _dp(_f64(wa)), _dp(_f64(wb)), _dp(_f64(v)), _dp(U),
                            _dp(Vb))
        return U, Vb

    def face(self, n, W6, lam):
        W6 = _f64(W6)
        Gm, Gp = np.zeros(self.M), np.zeros(self.M)
        self._L.orc_face(ctypes.byref(self.s), int(n), _dp(W6), float(lam), _dp(Gm), _dp(Gp), self._cnt())
        return Gm, Gp

    def interp_limit(self, vt, wnode):
        vt = _f64(vt).copy()
        hs = self._L.orc_interp_limit(ctypes.byref(self.s), _dp(vt), _dp(_f64(wnode)), self._cnt())
        return vt, hs

    def flux_limit(self, n, wl, wr, lam, gm_ho, gp_ho, gm_lo, gp_lo):
        Gm, Gp = np.zeros(self.M), np.zeros(self.M)
        self._L.orc_flux_limit(ctypes.byref(self.s), int(n), _dp(_f64(wl)), _dp(_f64(wr)), float(lam),
                               _dp(_f64(gm_ho)), _dp(_f64(gp_ho)), _dp(_f64(gm_lo)), _dp(_f64(gp_lo)), _dp(Gm),
                               _dp(Gp), self._cnt())
        return Gm, Gp


def weno(u5, eps=1e-15) -> float:
    return lib().orc_weno(_dp(_f64(u5)), float(eps))


def mlp_interp(params, u5):
    """Learned interpolation of one stencil (u_{i-2}..u_{i+2}): (value, omega),
    value None if a weight is not finite (the caller then uses App. C)."""
    out = np.zeros(1)
    om = np.zeros(3)
    ok = lib().orc_mlp_interp(_dp(_f64(params)), _dp(_f64(u5)), _dp(out), _dp(om))
    return (float(out[0]) if ok else None), om


def bf16(x) -> float:
    """x rounded to float, then to bfloat16 (ties to even)."""
    return lib().orc_bf16(float(x))


def sensor(u6) -> float:
    return lib().orc_sensor(_dp(_f64(u6)))


def hcs_coeffs(psi=256.0 / 175.0):
    out = np.zeros(3)
    lib().orc_hcs_coeffs(float(psi), _dp(out))
    return out


def from_problem(prob, flags=0, mlp=None, **params) -> Oracle:
    """An Oracle for a problem description from the input module (plain numbers only)."""
    e = prob.eos
    return Oracle(prob.N, prob.D, prob.n, prob.dx, prob.bc, e.gamma, e.cv, e.pinf, e.q, flags=flags, mlp=mlp,
                  boundary=getattr(prob, "boundary", None), **params)
