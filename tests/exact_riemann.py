"""Exact solution of the 1D Riemann problem for two perfect gases with
different gammas (Toro, "Riemann Solvers and Numerical Methods for Fluid
Dynamics", ch. 4: pressure function, Newton iteration for the star pressure,
sampling of the self-similar solution).  Independent of the scheme: used to
pin the whole Lagrange–Remap step on the Sod tube."""
import math

import numpy as np


def _f(p, rho, pk, ck, g):
    """Toro's pressure function and its derivative for one side."""
    if p > pk:  # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        sq = math.sqrt(A / (p + B))
        return (p - pk) * sq, sq * (1.0 - 0.5 * (p - pk) / (p + B))
    # rarefaction
    r = p / pk
    return (2.0 * ck / (g - 1.0) * (r ** ((g - 1.0) / (2.0 * g)) - 1.0),
            1.0 / (rho * ck) * r ** (-(g + 1.0) / (2.0 * g)))


def star_state(L, R):
    """(p*, u*) for left/right states (rho, u, p, gamma)."""
    rl, ul, pl, gl = L
    rr, ur, pr, gr = R
    cl, cr = math.sqrt(gl * pl / rl), math.sqrt(gr * pr / rr)
    p = max(1e-8, 0.5 * (pl + pr))
    for _ in range(100):
        fl, dl = _f(p, rl, pl, cl, gl)
        fr, dr = _f(p, rr, pr, cr, gr)
        dp = (fl + fr + ur - ul) / (dl + dr)
        pn = max(1e-12, p - dp)
        if abs(pn - p) < 1e-15 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _f(p, rl, pl, cl, gl)
    fr, _ = _f(p, rr, pr, cr, gr)
    return p, 0.5 * (ul + ur) + 0.5 * (fr - fl)


def sample(L, R, s, ps=None):
    """(rho, u, p, side) at similarity coordinate s = (x - x0)/t; side 0 is the
    left material, 1 the right."""
    if ps is None:
        ps = star_state(L, R)
    pst, ust = ps
    if s <= ust:
        rho, u, p, g = L
        side, sgn = 0, 1.0
    else:
        rho, u, p, g = R
        side, sgn = 1, -1.0
    c = math.sqrt(g * p / rho)
    # mirror the right side onto the left-side formulas with u -> -u, s -> -s
    uu, ss, us = sgn * u, sgn * s, sgn * ust
    if pst > p:  # shock
        S = uu - c * math.sqrt((g + 1.0) / (2.0 * g) * pst / p + (g - 1.0) / (2.0 * g))
        if ss <= S:
            return rho, u, p, side
        gg = (g - 1.0) / (g + 1.0)
        return rho * (pst / p + gg) / (gg * pst / p + 1.0), ust, pst, side
    cst = c * (pst / p) ** ((g - 1.0) / (2.0 * g))
    head, tail = uu - c, us - cst
    if ss <= head:
        return rho, u, p, side
    if ss > tail:
        return rho * (pst / p) ** (1.0 / g), ust, pst, side
    br = 2.0 / (g + 1.0) + (g - 1.0) / ((g + 1.0) * c) * (uu - ss)
    uf = 2.0 / (g + 1.0) * (c + 0.5 * (g - 1.0) * uu + ss)
    return rho * br ** (2.0 / (g - 1.0)), sgn * uf, p * br ** (2.0 * g / (g - 1.0)), side


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
