"""Exact solution of the 1D Riemann problem for two gases with different
equations of state (Toro, "Riemann Solvers and Numerical Methods for Fluid
Dynamics", ch. 4: pressure function, Newton iteration for the star pressure,
sampling of the self-similar solution).  Independent of the scheme: used to
pin the whole Lagrange–Remap step on shock tubes.

A state is (rho, u, p, gamma) for a perfect gas, or (rho, u, p, gamma, pi)
for the stiffened gas p = (gamma-1) rho e - pi written as in §5.2 of the
paper.  The stiffened gas is the perfect gas in the shifted pressure
p + pi/gamma (its sound speed is c^2 = gamma (p + pi/gamma)/rho), so Toro's
formulas hold with every pressure level replaced by the shifted one, and the
differences of pressures unchanged."""
import math

import numpy as np


def _unpack(K):
    rho, u, p, g = K[:4]
    pinf = (K[4] if len(K) > 4 else 0.0) / g  # shift of the pressure
    return rho, u, p, g, pinf


def _f(p, rho, pk, ck, g, pinf):
    """Toro's pressure function and its derivative for one side."""
    P, Pk = p + pinf, pk + pinf
    if p > pk:  # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * Pk
        sq = math.sqrt(A / (P + B))
        return (p - pk) * sq, sq * (1.0 - 0.5 * (p - pk) / (P + B))
    # rarefaction
    r = P / Pk
    return (2.0 * ck / (g - 1.0) * (r ** ((g - 1.0) / (2.0 * g)) - 1.0),
            1.0 / (rho * ck) * r ** (-(g + 1.0) / (2.0 * g)))


def star_state(L, R):
    """(p*, u*) for left/right states (rho, u, p, gamma[, pi])."""
    rl, ul, pl, gl, il = _unpack(L)
    rr, ur, pr, gr, ir = _unpack(R)
    cl, cr = math.sqrt(gl * (pl + il) / rl), math.sqrt(gr * (pr + ir) / rr)
    pmin = max(-il, -ir)  # the shifted pressures stay positive
    p = max(pmin + 1e-8 * (abs(pmin) + 1.0), 0.5 * (pl + pr))
    for _ in range(200):
        fl, dl = _f(p, rl, pl, cl, gl, il)
        fr, dr = _f(p, rr, pr, cr, gr, ir)
        dp = (fl + fr + ur - ul) / (dl + dr)
        pn = max(pmin + 1e-12 * (abs(pmin) + 1.0), p - dp)
        if abs(pn - p) < 1e-15 * (abs(pn) + abs(p)):
            p = pn
            break
        p = pn
    fl, _ = _f(p, rl, pl, cl, gl, il)
    fr, _ = _f(p, rr, pr, cr, gr, ir)
    return p, 0.5 * (ul + ur) + 0.5 * (fr - fl)


def sample(L, R, s, ps=None):
    """(rho, u, p, side) at similarity coordinate s = (x - x0)/t; side 0 is the
    left material, 1 the right."""
    if ps is None:
        ps = star_state(L, R)
    pst, ust = ps
    if s <= ust:
        rho, u, p, g, pinf = _unpack(L)
        side, sgn = 0, 1.0
    else:
        rho, u, p, g, pinf = _unpack(R)
        side, sgn = 1, -1.0
    P, Pst = p + pinf, pst + pinf
    c = math.sqrt(g * P / rho)
    # mirror the right side onto the left-side formulas with u -> -u, s -> -s
    uu, ss, us = sgn * u, sgn * s, sgn * ust
    if pst > p:  # shock
        S = uu - c * math.sqrt((g + 1.0) / (2.0 * g) * Pst / P + (g - 1.0) / (2.0 * g))
        if ss <= S:
            return rho, u, p, side
        gg = (g - 1.0) / (g + 1.0)
        return rho * (Pst / P + gg) / (gg * Pst / P + 1.0), ust, pst, side
    cst = c * (Pst / P) ** ((g - 1.0) / (2.0 * g))
    head, tail = uu - c, us - cst
    if ss <= head:
        return rho, u, p, side
    if ss > tail:
        return rho * (Pst / P) ** (1.0 / g), ust, pst, side
    br = 2.0 / (g + 1.0) + (g - 1.0) / ((g + 1.0) * c) * (uu - ss)
    uf = 2.0 / (g + 1.0) * (c + 0.5 * (g - 1.0) * uu + ss)
    return rho * br ** (2.0 / (g - 1.0)), sgn * uf, P * br ** (2.0 * g / (g - 1.0)) - pinf, side


def cell_averages(L, R, x0, t, edges, sub=32):
    """Exact cell averages of rho and p on cells with the given edges."""
    ps = star_state(L, R)
    n = len(edges) - 1
    rho = np.zeros(n)
    p = np.zeros(n)
    for i in range(n):
        xs = edges[i] + (np.arange(sub) + 0.5) / sub * (edges[i + 1] - edges[i])
        vals = [sample(L, R, (x - x0) / t, ps) for x in xs]
        rho[i] = np.mean([v[0] for v in vals])
        p[i] = np.mean([v[2] for v in vals])
    return rho, p
