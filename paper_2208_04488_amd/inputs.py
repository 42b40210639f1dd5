"""Seeded synthetic inputs: species tables, grids and initial conditions.

This module is problem set-up only.  It maps the initial data the paper's
tests are stated in (species densities from pressure and temperature,
velocity, pressure, volume fractions) to the conservative state, and draws the
random parts of the larger workloads from fixed seeds.  It performs none of
the steps of the hyperbolic stage or the relaxation, and serves both the HIP
library's callers and the CPU oracle's tests.

State arrays are float64 of shape (M, nz, ny, nx), M = 2N + D, with the
component order of the paper's conservative vector (Sec. 2):
  alpha_k rho_k (k = 0..N-1), rho u_d (d = 0..D-1), E, alpha_k (k = 0..N-2).
Species 0 is the liquid (stiffened gas); the others are ideal gases.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

TRANSMISSIVE, PERIODIC, DIRICHLET = 0, 1, 2
TRACE = 1e-8  # volume fraction of an absent species (Sec. 5 initial data)


@dataclass
class EOS:
    """Stiffened-gas parameters per species (eq:species_stiffened_EOS)."""
    gamma: List[float]
    cv: List[float]
    pinf: List[float]
    q: List[float]
    names: List[str] = field(default_factory=list)

    @property
    def N(self) -> int:
        return len(self.gamma)

    @property
    def cp(self) -> List[float]:
        return [g * c for g, c in zip(self.gamma, self.cv)]


def eos_from_cp(gamma, cp, pinf, q, names=()) -> EOS:
    """Species table given (gamma, c_p): c_v = c_p / gamma."""
    return EOS(list(map(float, gamma)), [c / g for c, g in zip(cp, gamma)], list(map(float, pinf)),
               list(map(float, q)), list(names))


# Table 1 of the paper: water, air, SF6 / detonation products
def table1_eos(third: Optional[str] = None) -> EOS:
    g, cp, pi, q, nm = [3.0, 1.4], [4200.0, 1007.0], [8.533e8, 0.0], [-0.1148e7, 0.0], ["water", "air"]
    if third == "SF6":
        g.append(1.1), cp.append(664.0), pi.append(0.0), q.append(0.0), nm.append("SF6")
    elif third == "detonation":
        g.append(1.25), cp.append(1000.0), pi.append(0.0), q.append(0.0), nm.append("detonation products")
    return eos_from_cp(g, cp, pi, q, nm)


# Liquids of the benchmark workloads.  Only gamma and pinf are given for them;
# c_p is taken from Table 1 (liquid 4200, air 1007) and the helium-like gas uses
# c_p = 5193 J/(kg K); q = 0 for these liquids.
LIQ_A = dict(gamma=4.4, cp=4200.0, pinf=6e8)       # two-phase shock tube liquid
LIQ_B = dict(gamma=6.12, cp=4200.0, pinf=3.43e8)   # liquid column / droplets
AIR = dict(gamma=1.4, cp=1007.0, pinf=0.0)
HELIUM = dict(gamma=1.67, cp=5193.0, pinf=0.0)


def eos_of(*species) -> EOS:
    return eos_from_cp([s["gamma"] for s in species], [s["cp"] for s in species],
                       [s["pinf"] for s in species], [0.0] * len(species))


# ----------------------------------------------------------------------------
# species thermal EOS used to build initial states
# ----------------------------------------------------------------------------
def species_density(eos: EOS, k: int, p, T):
    """rho_k(p, T) = (p + pinf_k) / ((gamma_k - 1) c_v,k T)."""
    return (p + eos.pinf[k]) / ((eos.gamma[k] - 1.0) * eos.cv[k] * T)


def species_temperature(eos: EOS, k: int, p, rho):
    """T_k = (p + pinf_k) / ((gamma_k - 1) rho_k c_v,k)."""
    return (p + eos.pinf[k]) / ((eos.gamma[k] - 1.0) * rho * eos.cv[k])


def state_from_fields(eos: EOS, alpha: Sequence[np.ndarray], rho_k: Sequence[np.ndarray],
                      u: Sequence[np.ndarray], p: np.ndarray) -> np.ndarray:
    """Conservative state from all N volume fractions, species densities,
    velocity components and pressure.  The energy is the sum of the species
    energies alpha_k rho_k e_k with rho_k (e_k - q_k) = (p + gamma_k pinf_k)/(gamma_k - 1)."""
    N, D = eos.N, len(u)
    p = np.asarray(p, dtype=np.float64)
    shape = np.broadcast(p, *alpha, *rho_k, *u).shape
    # only alpha_1..alpha_{N-1} are stored; alpha_N is 1 minus their sum, as the
    # state defines it, so the last partial density uses that derived value
    alpha = list(alpha[: N - 1]) + [1.0 - sum(np.asarray(a) for a in alpha[: N - 1])]
    ar = [np.broadcast_to(np.asarray(alpha[k]) * np.asarray(rho_k[k]), shape) for k in range(N)]
    rho = sum(ar)
    W = np.empty((2 * N + D,) + shape)
    for k in range(N):
        W[k] = ar[k]
    for d in range(D):
        W[N + d] = rho * u[d]
    E = 0.5 * rho * sum(np.asarray(ud) ** 2 for ud in u)
    for k in range(N):
        g, pi = eos.gamma[k], eos.pinf[k]
        E = E + np.asarray(alpha[k]) * (p + g * pi) / (g - 1.0) + ar[k] * eos.q[k]
    W[N + D] = E
    for k in range(N - 1):
        W[N + D + 1 + k] = alpha[k]
    return np.ascontiguousarray(W)


def equilibrium_state(eos: EOS, alpha: Sequence[np.ndarray], u: Sequence[np.ndarray], p, T) -> np.ndarray:
    """All species at one (p, T) (mechanical and thermal equilibrium, Sec. 5)."""
    rho_k = [species_density(eos, k, p, T) for k in range(eos.N)]
    return state_from_fields(eos, alpha, rho_k, u, p)


def mix_alpha(N: int, major: int, shape=(), trace=TRACE) -> List[np.ndarray]:
    """Volume fractions with one majority species and trace amounts of the rest."""
    a = [np.full(shape, trace) for _ in range(N)]
    a[major] = np.full(shape, 1.0 - (N - 1) * trace)
    return a


def tanh_step(x, x0, width):
    """0 -> 1 across x0 with the tanh profile of App. A (width = C_s dx)."""
    return 0.5 * (1.0 + np.tanh((x - x0) / width))


# ----------------------------------------------------------------------------
# problem container
# ----------------------------------------------------------------------------
@dataclass
class Problem:
    name: str
    eos: EOS
    D: int
    n: Tuple[int, ...]
    dx: Tuple[float, ...]
    bc: List[Tuple[int, int]]
    W: np.ndarray
    cfl: float = 0.4
    t_end: Optional[float] = None
    nsteps: Optional[int] = None
    dt_fixed: float = 0.0
    x0: Tuple[float, ...] = ()  # lower corner of the domain
    meta: dict = field(default_factory=dict)
    # Dirichlet sides: (dim, side) -> ghost states, shape (M, n_a * n_b), a < b the
    # other two dimensions, index i_a + n_a * i_b
    boundary: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return self.eos.N

    @property
    def M(self) -> int:
        return 2 * self.eos.N + self.D

    @property
    def ncell(self) -> int:
        return int(np.prod(self.n))

    def centres(self, d: int) -> np.ndarray:
        """Node positions x_i = x_a + (i + 1/2) dx (cell centres, Sec. 4.1)."""
        return self.x0[d] + (np.arange(self.n[d]) + 0.5) * self.dx[d]


def _grid(n, lo, hi):
    dx = tuple((h - l) / k for k, l, h in zip(n, lo, hi))
    return dx


def _as4(W: np.ndarray, D: int) -> np.ndarray:
    """(M, *spatial) in x-fastest (M, nz, ny, nx) order."""
    M = W.shape[0]
    if D == 1:
        return np.ascontiguousarray(W.reshape(M, 1, 1, -1))
    if D == 2:
        return np.ascontiguousarray(W.reshape(M, 1, W.shape[1], W.shape[2]))
    return np.ascontiguousarray(W)


# ----------------------------------------------------------------------------
# the paper's verification problems (Table 1 EOS)
# ----------------------------------------------------------------------------
P_ATM, T_ATM = 101325.0, 298.0


def advection_1d(n=64):
    """Sec. 5.1 temporal study: [-1, 1) periodic, u = 10, alpha_1 = 0.5 + 0.25 sin(pi x)."""
    eos = table1_eos()
    dx = (2.0 / n,)
    x = -1.0 + (np.arange(n) + 0.5) * dx[0]
    a1 = 0.5 + 0.25 * np.sin(np.pi * x)
    W = equilibrium_state(eos, [a1, 1.0 - a1], [np.full(n, 10.0)], np.full(n, P_ATM), T_ATM)
    return Problem("advection_1d", eos, 1, (n,), dx, [(PERIODIC, PERIODIC)], _as4(W, 1), x0=(-1.0,))


def advection_2d(n=32):
    """Sec. 5.2 spatial study: [-1, 1)^2 periodic, u = v = 10,
    alpha_1 = 0.5 + 0.25 sin(pi (x + y)), dt/dx = 4e-5 s/m, t_end = 0.1 ms."""
    eos = table1_eos()
    dx = (2.0 / n, 2.0 / n)
    c = -1.0 + (np.arange(n) + 0.5) * dx[0]
    Y, X = np.meshgrid(c, c, indexing="ij")
    a1 = 0.5 + 0.25 * np.sin(np.pi * (X + Y))
    W = equilibrium_state(eos, [a1, 1.0 - a1], [np.full_like(X, 10.0), np.full_like(X, 10.0)], P_ATM, T_ATM)
    return Problem("advection_2d", eos, 2, (n, n), dx, [(PERIODIC, PERIODIC)] * 2, _as4(W, 2),
                   t_end=1e-4, dt_fixed=4e-5 * dx[0], x0=(-1.0, -1.0))


def acoustic_1d(n=800, A=0.01, sigma=0.05, x_center=-0.75, c_ref=346.46):
    """Sec. 5.3 acoustic pulse: [-1, 1] m split at -0.5; left air with the
    liquid fraction 1e-8, right a 50/50 mixture, both at 101325 Pa / 298 K
    (Table 1 EOS); a Gaussian density pulse rho' = A exp(-((x - x_c)/sigma)^2)
    with p' = c_ref^2 rho' on the left at fixed mass fractions (T from rho and
    p, then the species densities and volume fractions); u = 0; transmissive.
    The transmitted pulse crosses the mixture at the four-equation (HRM)
    sound speed."""
    eos = table1_eos()
    dx = (2.0 / n,)
    x = -1.0 + (np.arange(n) + 0.5) * dx[0]
    left = x < -0.5
    # background mass fractions of the left region
    a_bg = [np.full(n, TRACE), np.full(n, 1.0 - TRACE)]
    rk_bg = [species_density(eos, k, P_ATM, T_ATM) for k in range(2)]
    rho_bg = a_bg[0] * rk_bg[0] + a_bg[1] * rk_bg[1]
    Y = [a_bg[k] * rk_bg[k] / rho_bg for k in range(2)]
    drho = A * np.exp(-(((x - x_center) / sigma) ** 2))
    rho = rho_bg + drho
    p = P_ATM + c_ref ** 2 * drho
    # 1/rho = sum_k Y_k / rho_k(p, T) with rho_k = (p + pinf_k)/((gamma_k - 1) c_v,k T)
    inv = sum(Y[k] * (eos.gamma[k] - 1.0) * eos.cv[k] / (p + eos.pinf[k]) for k in range(2))
    T = 1.0 / (rho * inv)
    rk = [species_density(eos, k, p, T) for k in range(2)]
    a_left = [Y[k] * rho / rk[k] for k in range(2)]
    rk_mix = [np.full(n, species_density(eos, k, P_ATM, T_ATM)) for k in range(2)]
    alpha = [np.where(left, a_left[k], 0.5) for k in range(2)]
    rho_k = [np.where(left, rk[k], rk_mix[k]) for k in range(2)]
    pp = np.where(left, p, P_ATM)
    W = state_from_fields(eos, alpha, rho_k, [np.zeros(n)], pp)
    return Problem("acoustic_1d", eos, 1, (n,), dx, [(TRANSMISSIVE, TRANSMISSIVE)], _as4(W, 1), cfl=0.4,
                   t_end=50e-3, x0=(-1.0,), meta=dict(x_interface=-0.5, c_ref=c_ref, p_ref=P_ATM))


def interface_advection(n=500, Cs: Optional[float] = None):
    """App. A: [0, 1) periodic, u = 100, water in [0.25, 0.75), air elsewhere,
    uniform 101325 Pa / 298 K; optional tanh smoothing with parameter C_s."""
    eos = table1_eos()
    dx = (1.0 / n,)
    x = (np.arange(n) + 0.5) * dx[0]
    a_mid, a_side = 1.0 - TRACE, TRACE
    if Cs is None:
        f = ((x >= 0.25) & (x < 0.75)).astype(float)
    else:
        w = Cs * dx[0]
        f = 0.5 * (np.tanh((x - 0.25) / w) - np.tanh((x - 0.75) / w))
    a1 = (a_mid - a_side) * f + a_side
    W = equilibrium_state(eos, [a1, 1.0 - a1], [np.full(n, 100.0)], np.full(n, P_ATM), T_ATM)
    return Problem("interface_advection", eos, 1, (n,), dx, [(PERIODIC, PERIODIC)], _as4(W, 1),
                   t_end=0.01, dt_fixed=6.25e-7 * 500 / n, x0=(0.0,))


def _two_state_1d(eos, n, length, x_split, left, right, name, t_end=None, dt_fixed=0.0):
    """Left/right states given as (alpha list, rho_k list, u, p)."""
    dx = (length / n,)
    x = (np.arange(n) + 0.5) * dx[0]
    L = x < x_split
    alpha = [np.where(L, left[0][k], right[0][k]) for k in range(eos.N)]
    rho_k = [np.where(L, left[1][k], right[1][k]) for k in range(eos.N)]
    u = [np.where(L, left[2], right[2])]
    p = np.where(L, left[3], right[3])
    W = state_from_fields(eos, alpha, rho_k, u, p)
    return Problem(name, eos, 1, (n,), dx, [(TRANSMISSIVE, TRANSMISSIVE)], _as4(W, 1), t_end=t_end,
                   dt_fixed=dt_fixed, x0=(0.0,), meta=dict(x_split=x_split, left=left, right=right))


def _side(eos, major, p, rho_major, u=0.0, trace=TRACE):
    """One side of a shock tube: the majority species has density rho_major at
    pressure p; trace species sit at the temperature that gives."""
    T = species_temperature(eos, major, p, rho_major)
    alpha = mix_alpha(eos.N, major, trace=trace)
    rho_k = [species_density(eos, k, p, T) for k in range(eos.N)]
    return [float(a) for a in alpha], rho_k, u, p, T


def shock_tube(n=500, extreme=False):
    """Sec. 5.4 (1e9 | 1e5 Pa) and Sec. 5.5 (1e12 | 1e5 Pa) gas/liquid shock tubes on
    [0, 1.5], split at 0.8; rho_1 = 1000 (left), rho_2 = 20 (right)."""
    eos = table1_eos()
    pl = 1e12 if extreme else 1e9
    left = _side(eos, 0, pl, 1000.0)
    right = _side(eos, 1, 1e5, 20.0)
    t_end = 1e-5 if extreme else 3e-4
    dt = (8e-9 * 1000 / n) if extreme else (5e-7 * 500 / n)
    pr = _two_state_1d(eos, n, 1.5, 0.8, left[:4], right[:4], "shock_tube_extreme" if extreme else "shock_tube",
                       t_end=t_end, dt_fixed=dt)
    pr.meta.update(T_left=left[4], T_right=right[4])
    return pr


def water_jet(nx=1024, ny=512, L=1.0, u_jet=1.5e5, t_end=6e-6):
    """Sec. 5.9 Mach-100 water jet: [0, L] x [-L/4, L/4] of air (liquid
    fraction 1e-8) at 101325 Pa / 298 K, at rest (Table 14).  The left side is
    a Dirichlet inflow (Table 15): water (air fraction 1e-8) at u = 1.5e5 m/s
    for |y| <= 0.05 L, the ambient air at rest elsewhere, both at 101325 Pa /
    298 K; the other sides are transmissive."""
    eos = table1_eos()
    dx = (L / nx, 0.5 * L / ny)
    y = -0.25 * L + (np.arange(ny) + 0.5) * dx[1]
    air = [np.full((ny, nx), TRACE), np.full((ny, nx), 1.0 - TRACE)]
    W = equilibrium_state(eos, air, [np.zeros((ny, nx))] * 2, P_ATM, T_ATM)
    jet = np.abs(y) <= 0.05 * L
    a1 = np.where(jet, 1.0 - TRACE, TRACE)
    Wb = equilibrium_state(eos, [a1, 1.0 - a1], [np.where(jet, u_jet, 0.0), np.zeros(ny)], P_ATM, T_ATM)
    return Problem("water_jet", eos, 2, (nx, ny), dx, [(DIRICHLET, TRANSMISSIVE), (TRANSMISSIVE, TRANSMISSIVE)],
                   _as4(W, 2), cfl=0.4, t_end=t_end, x0=(0.0, -0.25 * L),
                   boundary={(0, 0): Wb.reshape(Wb.shape[0], ny)}, meta=dict(u_jet=u_jet))


# ----------------------------------------------------------------------------
# benchmark workloads
# ----------------------------------------------------------------------------
def config1(n=400):
    """1D two-phase shock tube on [0, 1], split at 0.7: liquid (gamma 4.4,
    pinf 6e8, rho 1000, p 1e9) | air (rho 50, p 1e5); u = 0; trace 1e-8;
    transmissive; SSP-RK3 at CFL 0.4 to t = 240 us."""
    eos = eos_of(LIQ_A, AIR)
    left = _side(eos, 0, 1e9, 1000.0)
    right = _side(eos, 1, 1e5, 50.0)
    pr = _two_state_1d(eos, n, 1.0, 0.7, left[:4], right[:4], "config1_shock_tube", t_end=240e-6)
    pr.meta.update(T_left=left[4], T_right=right[4])
    return pr


def config5(nx=2048, ny=1024):
    """The config-1 shock tube as a planar problem on [0, 1] x [0, 0.5]:
    liquid (p 1e9, rho 1000) for x < 0.7, air (p 1e5, rho 50) beyond, u = v = 0,
    trace 1e-8; transmissive in x, periodic in y; CFL 0.4 to t = 240 us.  The
    workload of the learned interpolation weights against the plain method."""
    eos = eos_of(LIQ_A, AIR)
    left = _side(eos, 0, 1e9, 1000.0)
    right = _side(eos, 1, 1e5, 50.0)
    dx = (1.0 / nx, 0.5 / ny)
    x = (np.arange(nx) + 0.5) * dx[0]
    Lm = np.broadcast_to(x < 0.7, (ny, nx))
    alpha = [np.where(Lm, left[0][k], right[0][k]) for k in range(eos.N)]
    rho_k = [np.where(Lm, left[1][k], right[1][k]) for k in range(eos.N)]
    zero = np.zeros((ny, nx))
    p = np.where(Lm, left[3], right[3])
    W = state_from_fields(eos, alpha, rho_k, [zero, zero], p)
    return Problem("config5_planar_shock_tube", eos, 2, (nx, ny), dx, [(TRANSMISSIVE, TRANSMISSIVE),
                   (PERIODIC, PERIODIC)], _as4(W, 2), t_end=240e-6, x0=(0.0, 0.0),
                   meta=dict(x_split=0.7, left=left[:4], right=right[:4]))


def stiffened_hugoniot(gamma, pinf, rho0, p0, p1):
    """Shock from a stiffened gas at rest (rho0, p0) to the pressure p1: the
    Hugoniot density ratio with p shifted by pinf,
    rho1/rho0 = ((g+1)(p1+pinf) + (g-1)(p0+pinf)) / ((g-1)(p1+pinf) + (g+1)(p0+pinf)),
    then mass and momentum balance: u1 = sqrt((p1 - p0)(1/rho0 - 1/rho1)) and
    the shock speed s = rho1 u1 / (rho1 - rho0).  Returns (rho1, u1, s)."""
    a, b = p1 + pinf, p0 + pinf
    rho1 = rho0 * ((gamma + 1.0) * a + (gamma - 1.0) * b) / ((gamma - 1.0) * a + (gamma + 1.0) * b)
    u1 = math.sqrt((p1 - p0) * (1.0 / rho0 - 1.0 / rho1))
    return rho1, u1, rho1 * u1 / (rho1 - rho0)


def shock_interface(n=1600):
    """Sec. 5.6: 1D extreme shock-interface interaction on [0, 1] m (reading:
    the domain length is not printed).  Water (air and SF6 traces 1e-8 each)
    at 101325 Pa / 298 K, a 1e12 Pa shock at x = 0.15 (post-shock state from
    the stiffened-gas Hugoniot of the water, T from its EOS, traces at that p
    and T), a half air / half SF6 mixture (water trace 1e-8) beyond 0.3;
    transmissive; t = 1.26e-5 s; the paper's step 3e-9 s at 1600 points."""
    eos = table1_eos("SF6")
    x = (np.arange(n) + 0.5) / n
    rho_w0 = species_density(eos, 0, P_ATM, T_ATM)
    rho_w1, u1, _ = stiffened_hugoniot(eos.gamma[0], eos.pinf[0], rho_w0, P_ATM, 1e12)
    T1 = species_temperature(eos, 0, 1e12, rho_w1)
    post, water, gas = x < 0.15, (x >= 0.15) & (x < 0.3), x >= 0.3
    a1 = np.where(gas, TRACE, 1.0 - 2 * TRACE)
    a2 = np.where(gas, 0.5 - 0.5 * TRACE, TRACE)
    alpha = [a1, a2, 1.0 - a1 - a2]
    p = np.where(post, 1e12, P_ATM)
    T = np.where(post, T1, T_ATM)
    W = equilibrium_state(eos, alpha, [np.where(post, u1, 0.0)], p, T)
    return Problem("shock_interface", eos, 1, (n,), (1.0 / n,), [(TRANSMISSIVE, TRANSMISSIVE)], _as4(W, 1),
                   t_end=1.26e-5, dt_fixed=3e-9 * 1600 / n, x0=(0.0,), meta=dict(T_post=T1, u_post=u1))


def bubble_collapse(nx=2048, ny=1280, L=1e-3):
    """Sec. 5.8: a 1.9 GPa shock in water hits an air cylinder.  [0, 24L] x
    [-7.5L, 7.5L], L = 1 mm; the cylinder (radius 3L, centre (12L, 0)) and the
    pre-shock water at 101325 Pa / 298 K (Table 13); the plane shock at
    x = 6.6L with post-shock water from the stiffened-gas Hugoniot (T from the
    EOS, air trace at that p and T); interfaces sharp at the cell centres;
    transmissive.  meta["t0"] is the (negative) time of the initial state so
    that t = 0 when the shock reaches the cylinder."""
    eos = table1_eos()
    dx = (24 * L / nx, 15 * L / ny)
    x = (np.arange(nx) + 0.5) * dx[0]
    y = -7.5 * L + (np.arange(ny) + 0.5) * dx[1]
    X, Y = np.meshgrid(x, y)
    rho_w0 = species_density(eos, 0, P_ATM, T_ATM)
    rho_w1, u1, s = stiffened_hugoniot(eos.gamma[0], eos.pinf[0], rho_w0, P_ATM, 1.9e9)
    T1 = species_temperature(eos, 0, 1.9e9, rho_w1)
    post = X < 6.6 * L
    air = (X - 12 * L) ** 2 + Y ** 2 < (3 * L) ** 2
    a1 = np.where(air, TRACE, 1.0 - TRACE)
    p = np.where(post, 1.9e9, P_ATM)
    T = np.where(post, T1, T_ATM)
    W = equilibrium_state(eos, [a1, 1.0 - a1], [np.where(post, u1, 0.0), np.zeros_like(X)], p, T)
    return Problem("bubble_collapse", eos, 2, (nx, ny), dx, [(TRANSMISSIVE, TRANSMISSIVE)] * 2, _as4(W, 2),
                   cfl=0.4, x0=(0.0, -7.5 * L),
                   meta=dict(t0=-2.4 * L / s, u_post=u1, shock_speed=s, T_post=T1, R_b=3 * L, centre=(12 * L, 0.0)))


def undex(nx=1536, ny=1920, L=1.0):
    """Sec. 5.10: three-species extreme underwater explosion.  Water below
    y = 0, air above, a detonation-product bubble (ideal gas gamma 1.25,
    c_p 1000) of radius 0.3L at (0, -0.5L) at 1e12 Pa and 1250 kg/m^3 (T from
    its EOS); the rest at 101325 Pa / 298 K; traces 1e-8 (Table 16); at rest;
    transmissive; t = 0.25 ms.  Reading: the domain is [-8L, 8L] x [-6L, 14L]
    (16L x 20L with the surface 6L above the bottom, as the figure of the set-up
    shows; the printed y-range [0, 20L] would put the bubble outside it).
    Interfaces sharp at the cell centres."""
    eos = table1_eos("detonation")
    dx = (16 * L / nx, 20 * L / ny)
    x = -8 * L + (np.arange(nx) + 0.5) * dx[0]
    y = -6 * L + (np.arange(ny) + 0.5) * dx[1]
    X, Y = np.meshgrid(x, y)
    gas = X ** 2 + (Y + 0.5 * L) ** 2 < (0.3 * L) ** 2
    water = (Y < 0) & ~gas
    air = (Y >= 0) & ~gas
    a1 = np.where(water, 1.0 - 2 * TRACE, TRACE)
    a2 = np.where(air, 1.0 - 2 * TRACE, TRACE)
    T3 = species_temperature(eos, 2, 1e12, 1250.0)
    p = np.where(gas, 1e12, P_ATM)
    T = np.where(gas, T3, T_ATM)
    W = equilibrium_state(eos, [a1, a2, 1.0 - a1 - a2], [np.zeros_like(X)] * 2, p, T)
    return Problem("undex", eos, 2, (nx, ny), dx, [(TRANSMISSIVE, TRANSMISSIVE)] * 2, _as4(W, 2), cfl=0.4,
                   t_end=0.25e-3, x0=(-8 * L, -6 * L), meta=dict(T_gas=T3))


def rankine_hugoniot_ideal(gamma, R, p0, T0, mach):
    """Post-shock state of a normal shock of Mach number `mach` moving into an
    ideal gas at rest; returns (p1, rho1, u1, T1)."""
    rho0 = p0 / (R * T0)
    c0 = math.sqrt(gamma * p0 / rho0)
    m2 = mach * mach
    p1 = p0 * (1.0 + 2.0 * gamma / (gamma + 1.0) * (m2 - 1.0))
    rho1 = rho0 * (gamma + 1.0) * m2 / ((gamma - 1.0) * m2 + 2.0)
    u1 = mach * c0 * (1.0 - rho0 / rho1)
    return p1, rho1, u1, p1 / (rho1 * R)


def config2(nx=1024, ny=512, L=0.024, Cs=2.0):
    """2D shock on a liquid column with a gas bubble: species liquid (gamma 6.12,
    pinf 3.43e8), air, helium-like gas.  Domain [-L/2, L/2] x [-L/4, L/4]; disk
    r = 0.1 L at the origin containing a bubble r = 0.03 L; ambient 101325 Pa,
    298 K; Mach-1.47 post-shock air for x < -0.15 L; tanh smoothing over C_s
    cells; transmissive; CFL 0.4; 500 steps."""
    eos = eos_of(LIQ_B, AIR, HELIUM)
    dx = (L / nx, 0.5 * L / ny)
    xc = -0.5 * L + (np.arange(nx) + 0.5) * dx[0]
    yc = -0.25 * L + (np.arange(ny) + 0.5) * dx[1]
    Y, X = np.meshgrid(yc, xc, indexing="ij")
    r = np.hypot(X, Y)
    w = Cs * dx[0]
    f_disk = 1.0 - tanh_step(r, 0.1 * L, w)
    f_bub = 1.0 - tanh_step(r, 0.03 * L, w)
    e = TRACE
    a_he = e + (1.0 - 3.0 * e) * f_bub
    a_liq = e + (1.0 - 3.0 * e) * (f_disk - f_bub)
    a_air = 1.0 - a_liq - a_he
    R_air = eos.cp[1] - eos.cv[1]
    p1, rho1, u1, T1 = rankine_hugoniot_ideal(eos.gamma[1], R_air, P_ATM, T_ATM, 1.47)
    post = X < -0.15 * L
    p = np.where(post, p1, P_ATM)
    T = np.where(post, T1, T_ATM)
    u = np.where(post, u1, 0.0)
    W = equilibrium_state(eos, [a_liq, a_air, a_he], [u, np.zeros_like(u)], p, T)
    return Problem("config2_liquid_column", eos, 2, (nx, ny), dx, [(TRANSMISSIVE, TRANSMISSIVE)] * 2,
                   _as4(W, 2), nsteps=500, x0=(-0.5 * L, -0.25 * L),
                   meta=dict(post_shock=(p1, rho1, u1, T1)))


def config3(n=256, L=1.0, seed_modes=3001, seed_drops=3002, Cs=2.0):
    """3D multimode interface: liquid droplets (gamma 6.12), heavy gas (gamma 1.4,
    R = 287.7), light gas (gamma 1.67, R = 3 x 287.7).  Light gas for
    x < 0.5 L + eta(y, z) with 32 random modes (|k| <= 16, uniform phases,
    max |eta| = 0.01 L); droplets r = 0.02 L filling 10% of [0.6 L, L] x [0, L]^2;
    101325 Pa / 298 K; Mach-1.5 shock in the light gas at x = 0.3 L;
    transmissive in x, periodic in y and z; 200 steps at CFL 0.4."""
    R2 = 287.7
    heavy = dict(gamma=1.4, cp=1.4 * R2 / 0.4, pinf=0.0)
    light = dict(gamma=1.67, cp=1.67 * 3.0 * R2 / 0.67, pinf=0.0)
    eos = eos_of(LIQ_B, heavy, light)
    dx = (L / n,) * 3
    c = (np.arange(n) + 0.5) * dx[0]
    rng = np.random.default_rng(seed_modes)
    ks = [(ky, kz) for ky in range(-16, 17) for kz in range(-16, 17) if 1 <= math.hypot(ky, kz) <= 16]
    pick = rng.choice(len(ks), size=32, replace=False)
    phases = rng.uniform(0.0, 2.0 * math.pi, size=32)
    Zc, Yc = np.meshgrid(c, c, indexing="ij")
    eta = np.zeros_like(Yc)
    for (ky, kz), ph in zip([ks[i] for i in pick], phases):
        eta += np.cos(2.0 * math.pi * (ky * Yc + kz * Zc) / L + ph)
    eta *= 0.01 * L / np.abs(eta).max()
    w = Cs * dx[0]
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    f_light = 1.0 - tanh_step(X, 0.5 * L + eta[:, :, None], w)
    rngd = np.random.default_rng(seed_drops)
    rd = 0.02 * L
    vol = 0.4 * L ** 3 * 0.10
    ndrop = int(round(vol / (4.0 / 3.0 * math.pi * rd ** 3)))
    centres = np.column_stack([rngd.uniform(0.6 * L, L, ndrop), rngd.uniform(0, L, ndrop), rngd.uniform(0, L, ndrop)])
    f_liq = np.zeros_like(X)
    for cx, cy, cz in centres:
        i0, i1 = max(0, int((cx - rd - 3 * w) / dx[0])), min(n, int((cx + rd + 3 * w) / dx[0]) + 2)
        sl = slice(i0, i1)
        # periodic distance in y and z
        dyv = (c - cy + 0.5 * L) % L - 0.5 * L
        dzv = (c - cz + 0.5 * L) % L - 0.5 * L
        jy = np.nonzero(np.abs(dyv) < rd + 3 * w)[0]
        jz = np.nonzero(np.abs(dzv) < rd + 3 * w)[0]
        if len(jy) == 0 or len(jz) == 0:
            continue
        ddz, ddy, ddx = np.meshgrid(dzv[jz], dyv[jy], c[sl] - cx, indexing="ij")
        rr = np.sqrt(ddx ** 2 + ddy ** 2 + ddz ** 2)
        f = 1.0 - tanh_step(rr, rd, w)
        sub = f_liq[np.ix_(jz, jy, np.arange(i0, i1))]
        f_liq[np.ix_(jz, jy, np.arange(i0, i1))] = np.maximum(sub, f)
    e = TRACE
    a_liq = e + (1.0 - 3.0 * e) * f_liq
    a_light = e + (1.0 - 3.0 * e) * (1.0 - f_liq) * f_light
    a_heavy = 1.0 - a_liq - a_light
    p1, rho1, u1, T1 = rankine_hugoniot_ideal(light["gamma"], 3.0 * R2, P_ATM, T_ATM, 1.5)
    post = X < 0.3 * L
    p = np.where(post, p1, P_ATM)
    T = np.where(post, T1, T_ATM)
    u = np.where(post, u1, 0.0)
    zero = np.zeros_like(u)
    W = equilibrium_state(eos, [a_liq, a_heavy, a_light], [u, zero, zero], p, T)
    return Problem("config3_multimode", eos, 3, (n, n, n), dx,
                   [(TRANSMISSIVE, TRANSMISSIVE), (PERIODIC, PERIODIC), (PERIODIC, PERIODIC)], _as4(W, 3),
                   nsteps=200, x0=(0.0, 0.0, 0.0), meta=dict(ndrop=ndrop))


def random_admissible(eos: EOS, D: int, count: int, seed: int, p_range=(1e4, 1e9), T_range=(200.0, 2000.0),
                      u_scale=200.0, mixed=True) -> np.ndarray:
    """Random states in the admissible set G at p-T equilibrium: columns of an
    (M, count) array.  Volume fractions are Dirichlet-distributed (or one
    majority species with traces when mixed=False)."""
    rng = np.random.default_rng(seed)
    N = eos.N
    p = np.exp(rng.uniform(math.log(p_range[0]), math.log(p_range[1]), count))
    T = rng.uniform(T_range[0], T_range[1], count)
    if mixed:
        a = rng.dirichlet(np.ones(N), count).T
        a = np.clip(a, TRACE, None)
        a /= a.sum(axis=0)
    else:
        major = rng.integers(0, N, count)
        a = np.full((N, count), TRACE)
        a[major, np.arange(count)] = 1.0 - (N - 1) * TRACE
    u = [rng.normal(0.0, u_scale, count) for _ in range(D)]
    return equilibrium_state(eos, list(a), u, p, T)


@dataclass
class Batch:
    """Ragged ensemble of independent 1D problems stored back to back:
    W is (M, T) with T = offsets[-1]; problem b owns cells offsets[b]..offsets[b+1]-1."""
    name: str
    eos: EOS
    W: np.ndarray
    offsets: np.ndarray
    dx: np.ndarray
    cfl: float = 0.4
    nsteps: int = 1000
    meta: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return self.eos.N

    @property
    def M(self) -> int:
        return 2 * self.eos.N + 1

    @property
    def nprob(self) -> int:
        return len(self.offsets) - 1

    @property
    def ncell(self) -> int:
        return int(self.offsets[-1])

    def problem(self, b: int) -> Problem:
        """Problem b on its own grid (same inputs), for comparisons."""
        lo, hi = int(self.offsets[b]), int(self.offsets[b + 1])
        n = hi - lo
        W = np.ascontiguousarray(self.W[:, lo:hi].reshape(self.M, 1, 1, n))
        return Problem(f"{self.name}[{b}]", self.eos, 1, (n,), (float(self.dx[b]),),
                       [(TRANSMISSIVE, TRANSMISSIVE)], W, cfl=self.cfl, x0=(0.0,))


def config4(nprob=4096, nmin=200, nmax=2000, seed=4001, lengths=None):
    """Batched ensemble of two-phase Riemann problems on [0, 1] with the
    interface at 0.5: lengths uniform in [nmin, nmax]; per side p log-uniform
    in [1e5, 1e9] Pa, majority density log-uniform in [1, 1000] kg/m^3, the
    majority species liquid (gamma 4.4, pinf 6e8) or air with probability 1/2;
    traces 1e-8 at the side's temperature; u = 0; transmissive; CFL 0.4.
    `lengths`, if given, fixes the problem lengths (and their number)."""
    eos = eos_of(LIQ_A, AIR)
    rng = np.random.default_rng(seed)
    if lengths is not None:
        lens = np.asarray(lengths, dtype=np.int64)
        nprob = len(lens)
    else:
        lens = rng.integers(nmin, nmax + 1, size=nprob)
    offsets = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    parts, dxs = [], []
    for b in range(nprob):
        n = int(lens[b])
        sides = []
        for _ in range(2):
            p = float(np.exp(rng.uniform(np.log(1e5), np.log(1e9))))
            rho = float(np.exp(rng.uniform(np.log(1.0), np.log(1000.0))))
            major = int(rng.integers(0, 2))
            sides.append(_side(eos, major, p, rho))
        dx = 1.0 / n
        x = (np.arange(n) + 0.5) * dx
        left = x < 0.5
        L, R = sides
        alpha = [np.where(left, L[0][k], R[0][k]) for k in range(2)]
        rho_k = [np.where(left, L[1][k], R[1][k]) for k in range(2)]
        p = np.where(left, L[3], R[3])
        parts.append(state_from_fields(eos, alpha, rho_k, [np.zeros(n)], p))
        dxs.append(dx)
    W = np.ascontiguousarray(np.concatenate(parts, axis=1))
    return Batch("config4_batched", eos, W, offsets, np.asarray(dxs), meta=dict(seed=seed))
