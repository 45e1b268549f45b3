"""Exact solution of the Riemann problem of the 1D Euler equations (ideal gas).

Test-only helper, written from the textbook construction (Toro, "Riemann Solvers
and Numerical Methods for Fluid Dynamics", 2009, ch. 4): the star pressure is
the root of f_L(p) + f_R(p) + u_R - u_L = 0, where f_K is the shock (Rankine-
Hugoniot) branch for p > p_K and the rarefaction (isentropic) branch otherwise;
the self-similar solution is then sampled at x/t.
"""
from __future__ import annotations

import math

import numpy as np


def _f(p, rho, pk, ck, g):
    if p > pk:
        a = 2.0 / ((g + 1.0) * rho)
        b = (g - 1.0) / (g + 1.0) * pk
        q = math.sqrt(a / (p + b))
        return (p - pk) * q, q * (1.0 - 0.5 * (p - pk) / (b + p))
    r = p / pk
    f = 2.0 * ck / (g - 1.0) * (r ** ((g - 1.0) / (2.0 * g)) - 1.0)
    df = 1.0 / (rho * ck) * r ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star_state(rl, ul, pl, rr, ur, pr, g):
    cl = math.sqrt(g * pl / rl)
    cr = math.sqrt(g * pr / rr)
    p = max(1e-12, 0.5 * (pl + pr) - 0.125 * (ur - ul) * (rl + rr) * (cl + cr))
    for _ in range(100):
        fl, dfl = _f(p, rl, pl, cl, g)
        fr, dfr = _f(p, rr, pr, cr, g)
        pn = p - (fl + fr + ur - ul) / (dfl + dfr)
        pn = max(pn, 1e-14)
        if abs(pn - p) < 1e-15 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _f(p, rl, pl, cl, g)
    fr, _ = _f(p, rr, pr, cr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def sample(s, rl, ul, pl, rr, ur, pr, g):
    """(rho, u, p) of the exact solution at similarity coordinate s = x/t."""
    ps, us = star_state(rl, ul, pl, rr, ur, pr, g)
    gm = (g - 1.0) / (g + 1.0)
    if s <= us:
        rho, u, p, c = rl, ul, pl, math.sqrt(g * pl / rl)
        if ps > p:  # left shock
            sh = u - c * math.sqrt((g + 1) / (2 * g) * ps / p + (g - 1) / (2 * g))
            if s < sh:
                return rho, u, p
            return rho * (ps / p + gm) / (gm * ps / p + 1.0), us, ps
        head = u - c
        cs = c * (ps / p) ** ((g - 1) / (2 * g))
        tail = us - cs
        if s < head:
            return rho, u, p
        if s > tail:
            return rho * (ps / p) ** (1.0 / g), us, ps
        uu = 2.0 / (g + 1) * (c + (g - 1) / 2 * u + s)
        cc = 2.0 / (g + 1) * (c + (g - 1) / 2 * (u - s))
        return rho * (cc / c) ** (2 / (g - 1)), uu, p * (cc / c) ** (2 * g / (g - 1))
    rho, u, p, c = rr, ur, pr, math.sqrt(g * pr / rr)
    if ps > p:  # right shock
        sh = u + c * math.sqrt((g + 1) / (2 * g) * ps / p + (g - 1) / (2 * g))
        if s > sh:
            return rho, u, p
        return rho * (ps / p + gm) / (gm * ps / p + 1.0), us, ps
    head = u + c
    cs = c * (ps / p) ** ((g - 1) / (2 * g))
    tail = us + cs
    if s > head:
        return rho, u, p
    if s < tail:
        return rho * (ps / p) ** (1.0 / g), us, ps
    uu = 2.0 / (g + 1) * (-c + (g - 1) / 2 * u + s)
    cc = 2.0 / (g + 1) * (c - (g - 1) / 2 * (u - s))
    return rho * (cc / c) ** (2 / (g - 1)), uu, p * (cc / c) ** (2 * g / (g - 1))


def density_profile(x, x0, t, left, right, g, mirrored=False):
    """Exact density at positions x for an interface at x0 (left state at x < x0),
    or the mirror image (left state at x > x0)."""
    out = np.empty_like(x)
    for i, xi in enumerate(x):
        s = (x0 - xi) / t if mirrored else (xi - x0) / t
        out[i] = sample(s, *left, *right, g)[0]
    return out
