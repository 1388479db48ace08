"""Exact solution of the Riemann problem for the ideal-gas Euler equations.

Test-only pin for the oracle.  The method is the textbook one of Toro,
"Riemann Solvers and Numerical Methods for Fluid Dynamics", ch. 4: solve the
pressure function f(p) = f_L(p) + f_R(p) + (u_R - u_L) = 0 for the star
pressure (Newton iteration with bisection safeguard), then sample the wave
pattern (shock or rarefaction on each side) at x/t.  Written from the
mathematics; independent of the oracle's code.
"""
from __future__ import annotations

import math

import numpy as np


def _fk(p, rho, pk, ck, g):
    if p > pk:  # shock
        a = 2.0 / ((g + 1.0) * rho)
        b = (g - 1.0) / (g + 1.0) * pk
        q = math.sqrt(a / (p + b))
        return (p - pk) * q, q * (1.0 - 0.5 * (p - pk) / (p + b))
    # rarefaction
    r = p / pk
    f = 2.0 * ck / (g - 1.0) * (r ** ((g - 1.0) / (2.0 * g)) - 1.0)
    df = 1.0 / (rho * ck) * r ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star_state(rl, ul, pl, rr, ur, pr, g):
    """Star pressure and velocity (p*, u*)."""
    cl = math.sqrt(g * pl / rl)
    cr = math.sqrt(g * pr / rr)
    lo, hi = 1e-14, 10.0 * max(pl, pr) + 10.0
    p = 0.5 * (pl + pr)
    for _ in range(200):
        fl, dl = _fk(p, rl, pl, cl, g)
        fr, dr = _fk(p, rr, pr, cr, g)
        f = fl + fr + (ur - ul)
        if f > 0:
            hi = p
        else:
            lo = p
        pn = p - f / (dl + dr)
        if not (lo < pn < hi):
            pn = 0.5 * (lo + hi)
        if abs(pn - p) <= 1e-15 * p:
            p = pn
            break
        p = pn
    fl, _ = _fk(p, rl, pl, cl, g)
    fr, _ = _fk(p, rr, pr, cr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def star_densities(rl, pl, rr, pr, ps, g):
    def side(r, pk):
        if ps > pk:
            q = ps / pk
            gm = (g - 1.0) / (g + 1.0)
            return r * (q + gm) / (gm * q + 1.0)
        return r * (ps / pk) ** (1.0 / g)
    return side(rl, pl), side(rr, pr)


def sample(rl, ul, pl, rr, ur, pr, g, s):
    """Primitive state (rho, u, p) at similarity coordinates s = x/t (array)."""
    ps, us = star_state(rl, ul, pl, rr, ur, pr, g)
    rsl, rsr = star_densities(rl, pl, rr, pr, ps, g)
    cl = math.sqrt(g * pl / rl)
    cr = math.sqrt(g * pr / rr)
    s = np.asarray(s, dtype=np.float64)
    rho = np.empty_like(s)
    u = np.empty_like(s)
    p = np.empty_like(s)
    for i, x in np.ndenumerate(s):
        if x <= us:  # left of contact
            if ps > pl:
                sl = ul - cl * math.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
                st = (rl, ul, pl) if x <= sl else (rsl, us, ps)
            else:
                csl = cl * (ps / pl) ** ((g - 1) / (2 * g))
                head, tail = ul - cl, us - csl
                if x <= head:
                    st = (rl, ul, pl)
                elif x >= tail:
                    st = (rsl, us, ps)
                else:
                    c = 2 / (g + 1) * (cl + (g - 1) / 2 * (ul - x))
                    uu = 2 / (g + 1) * (cl + (g - 1) / 2 * ul + x)
                    rr_ = rl * (c / cl) ** (2 / (g - 1))
                    st = (rr_, uu, pl * (c / cl) ** (2 * g / (g - 1)))
        else:
            if ps > pr:
                sr = ur + cr * math.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
                st = (rr, ur, pr) if x >= sr else (rsr, us, ps)
            else:
                csr = cr * (ps / pr) ** ((g - 1) / (2 * g))
                head, tail = ur + cr, us + csr
                if x >= head:
                    st = (rr, ur, pr)
                elif x <= tail:
                    st = (rsr, us, ps)
                else:
                    c = 2 / (g + 1) * (cr - (g - 1) / 2 * (ur - x))
                    uu = 2 / (g + 1) * (-cr + (g - 1) / 2 * ur + x)
                    rr_ = rr * (c / cr) ** (2 / (g - 1))
                    st = (rr_, uu, pr * (c / cr) ** (2 * g / (g - 1)))
        rho[i], u[i], p[i] = st
    return rho, u, p
