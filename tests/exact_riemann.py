"""Exact solution of the 1D Euler Riemann problem for an ideal gas (test support).

Standard two-wave construction: the star-region pressure solves f_L(p) + f_R(p) + (u_R - u_L) = 0
with shock (Rankine-Hugoniot) or rarefaction (isentropic) branches on each side; the solution
at x/t is then sampled wave by wave.  Used only to check the oracle on Sod's problem.
"""
from __future__ import annotations

import math

import numpy as np


def _f_and_df(p, rho_k, p_k, c_k, g):
    if p > p_k:  # shock
        A = 2.0 / ((g + 1.0) * rho_k)
        B = (g - 1.0) / (g + 1.0) * p_k
        sq = math.sqrt(A / (p + B))
        f = (p - p_k) * sq
        df = sq * (1.0 - 0.5 * (p - p_k) / (B + p))
    else:  # rarefaction
        pr = p / p_k
        f = 2.0 * c_k / (g - 1.0) * (pr ** ((g - 1.0) / (2.0 * g)) - 1.0)
        df = 1.0 / (rho_k * c_k) * pr ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star_state(left, right, g=1.4):
    rl, ul, pl = left
    rr, ur, pr = right
    cl = math.sqrt(g * pl / rl)
    cr = math.sqrt(g * pr / rr)
    p = max(1e-8, 0.5 * (pl + pr))
    for _ in range(100):
        fl, dfl = _f_and_df(p, rl, pl, cl, g)
        fr, dfr = _f_and_df(p, rr, pr, cr, g)
        dp = (fl + fr + ur - ul) / (dfl + dfr)
        pn = max(1e-10, p - dp)
        if abs(pn - p) < 1e-14 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _f_and_df(p, rl, pl, cl, g)
    fr, _ = _f_and_df(p, rr, pr, cr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def sample(s, left, right, g=1.4):
    """Primitive state (rho, u, p) at similarity coordinate s = x / t."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl = math.sqrt(g * pl / rl)
    cr = math.sqrt(g * pr / rr)
    ps, us = star_state(left, right, g)
    if s <= us:  # left of the contact
        if ps > pl:  # left shock
            sl = ul - cl * math.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
            if s <= sl:
                return rl, ul, pl
            r = rl * ((ps / pl + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pl + 1))
            return r, us, ps
        shl = ul - cl
        csl = cl * (ps / pl) ** ((g - 1) / (2 * g))
        stl = us - csl
        if s <= shl:
            return rl, ul, pl
        if s >= stl:
            return rl * (ps / pl) ** (1 / g), us, ps
        u = 2 / (g + 1) * (cl + (g - 1) / 2 * ul + s)
        c = 2 / (g + 1) * (cl + (g - 1) / 2 * (ul - s))
        r = rl * (c / cl) ** (2 / (g - 1))
        return r, u, pl * (c / cl) ** (2 * g / (g - 1))
    if ps > pr:  # right shock
        sr = ur + cr * math.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
        if s >= sr:
            return rr, ur, pr
        r = rr * ((ps / pr + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pr + 1))
        return r, us, ps
    shr = ur + cr
    csr = cr * (ps / pr) ** ((g - 1) / (2 * g))
    str_ = us + csr
    if s >= shr:
        return rr, ur, pr
    if s <= str_:
        return rr * (ps / pr) ** (1 / g), us, ps
    u = 2 / (g + 1) * (-cr + (g - 1) / 2 * ur + s)
    c = 2 / (g + 1) * (cr - (g - 1) / 2 * (ur - s))
    r = rr * (c / cr) ** (2 / (g - 1))
    return r, u, pr * (c / cr) ** (2 * g / (g - 1))


def density_cell_averages(n, t, left, right, g=1.4, x0=-1.0, x1=1.0, xs=0.0, sub=64):
    """Cell averages of the exact density at time t (midpoint rule on `sub` points per cell)."""
    h = (x1 - x0) / n
    out = np.zeros(n)
    for i in range(n):
        xs_ = x0 + i * h + (np.arange(sub) + 0.5) * h / sub
        out[i] = np.mean([sample((x - xs) / t, left, right, g)[0] for x in xs_])
    return out
