"""Exact solution of the 1D Riemann problem between two stiffened gases.

TEST INFRASTRUCTURE (an independent pin of the oracle, not a step of the
method).  Textbook two-rarefaction/two-shock construction for the Euler
equations (Toro, Riemann Solvers and Numerical Methods for Fluid Dynamics,
ch. 4) with each side's own gamma and the pressure shifted by that side's
p_inf.  Each side is a single pure material; trace species of the paper's
initial data are ignored.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import brentq


def _side_fun(p, rho, u, pk, g, pi):
    """f_K(p) and the side's wave data."""
    ph, pkh = p + pi, pk + pi
    if ph <= 0.0:
        return -math.inf
    if p > pk:  # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pkh
        return (p - pk) * math.sqrt(A / (ph + B))
    c = math.sqrt(g * pkh / rho)
    return 2.0 * c / (g - 1.0) * ((ph / pkh) ** ((g - 1.0) / (2.0 * g)) - 1.0)


def star_state(L, R):
    """L, R: dicts with rho, u, p, gamma, pinf.  Returns (p*, u*)."""
    def f(p):
        return (_side_fun(p, L["rho"], L["u"], L["p"], L["gamma"], L["pinf"]) +
                _side_fun(p, R["rho"], R["u"], R["p"], R["gamma"], R["pinf"]) + R["u"] - L["u"])
    lo = -min(L["pinf"], R["pinf"]) + 1e-9 * max(1.0, L["p"], R["p"])
    hi = 10.0 * max(L["p"] + L["pinf"], R["p"] + R["pinf"])
    while f(hi) < 0.0:
        hi *= 10.0
    ps = brentq(f, lo, hi, xtol=1e-12 * hi, rtol=1e-15, maxiter=500)
    fl = _side_fun(ps, L["rho"], L["u"], L["p"], L["gamma"], L["pinf"])
    fr = _side_fun(ps, R["rho"], R["u"], R["p"], R["gamma"], R["pinf"])
    us = 0.5 * (L["u"] + R["u"]) + 0.5 * (fr - fl)
    return ps, us


def _sample_side(xi, K, ps, us, sgn):
    """State at x/t = xi on side K (sgn = -1 for left, +1 for right) of the contact."""
    rho, u, p, g, pi = K["rho"], K["u"], K["p"], K["gamma"], K["pinf"]
    c = math.sqrt(g * (p + pi) / rho)
    r = (ps + pi) / (p + pi)
    if ps > p:  # shock
        S = u + sgn * c * math.sqrt((g + 1.0) / (2.0 * g) * r + (g - 1.0) / (2.0 * g))
        if sgn * (xi - S) > 0.0:
            return rho, u, p
        gm = (g - 1.0) / (g + 1.0)
        return rho * (r + gm) / (gm * r + 1.0), us, ps
    # rarefaction
    cs = c * r ** ((g - 1.0) / (2.0 * g))
    head, tail = u + sgn * c, us + sgn * cs
    if sgn * (xi - head) > 0.0:
        return rho, u, p
    if sgn * (xi - tail) < 0.0:
        return rho * r ** (1.0 / g), us, ps
    uf = 2.0 / (g + 1.0) * (-sgn * c + (g - 1.0) / 2.0 * u + xi)
    cf = 2.0 / (g + 1.0) * (c - sgn * (g - 1.0) / 2.0 * (u - xi))
    return rho * (cf / c) ** (2.0 / (g - 1.0)), uf, (p + pi) * (cf / c) ** (2.0 * g / (g - 1.0)) - pi


def solve(x, t, x0, L, R):
    """Density, velocity and pressure at positions x and time t > 0."""
    ps, us = star_state(L, R)
    x = np.asarray(x, dtype=float)
    out = np.empty((3,) + x.shape)
    for idx, xv in np.ndenumerate(x):
        xi = (xv - x0) / t
        if xi < us:
            out[(slice(None),) + idx] = _sample_side(xi, L, ps, us, -1.0)
        else:
            out[(slice(None),) + idx] = _sample_side(xi, R, ps, us, +1.0)
    return out[0], out[1], out[2]
