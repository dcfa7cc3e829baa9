"""Exact solution of the Riemann problem of the 1-D Euler equations for an ideal gas
(Toro, "Riemann Solvers and Numerical Methods for Fluid Dynamics", ch. 4): Newton iteration
for the star pressure, then sampling of the self-similar solution at x/t.

Test reference only: it pins the hydro sweep against the Sod shock tube.
"""

import math

import numpy as np


def _f_side(p, rho_k, p_k, c_k, g):
    """Pressure function f_K(p) and its derivative for one side (shock if p > p_K)."""
    if p > p_k:
        a_k = 2.0 / ((g + 1.0) * rho_k)
        b_k = (g - 1.0) / (g + 1.0) * p_k
        s = math.sqrt(a_k / (p + b_k))
        return (p - p_k) * s, s * (1.0 - 0.5 * (p - p_k) / (p + b_k))
    r = p / p_k
    f = 2.0 * c_k / (g - 1.0) * (r ** ((g - 1.0) / (2.0 * g)) - 1.0)
    df = 1.0 / (rho_k * c_k) * r ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star_state(left, right, g):
    """(p*, u*) for left/right primitive states (rho, u, p)."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl = math.sqrt(g * pl / rl)
    cr = math.sqrt(g * pr / rr)
    p = max(1e-12, 0.5 * (pl + pr) - 0.125 * (ur - ul) * (rl + rr) * (cl + cr))
    for _ in range(100):
        fl, dfl = _f_side(p, rl, pl, cl, g)
        fr, dfr = _f_side(p, rr, pr, cr, g)
        dp = (fl + fr + ur - ul) / (dfl + dfr)
        p_new = max(1e-12, p - dp)
        if abs(p_new - p) < 1e-15 * (p_new + p):
            p = p_new
            break
        p = p_new
    fl, _ = _f_side(p, rl, pl, cl, g)
    fr, _ = _f_side(p, rr, pr, cr, g)
    return p, 0.5 * (ul + ur) + 0.5 * (fr - fl)


def sample(xi, left, right, g):
    """Primitive state (rho, u, p) of the exact solution at xi = x/t."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl = math.sqrt(g * pl / rl)
    cr = math.sqrt(g * pr / rr)
    ps, us = star_state(left, right, g)
    gm = (g - 1.0) / (g + 1.0)
    if xi <= us:
        if ps > pl:
            sl = ul - cl * math.sqrt((g + 1.0) / (2.0 * g) * ps / pl + (g - 1.0) / (2.0 * g))
            if xi <= sl:
                return rl, ul, pl
            return rl * (ps / pl + gm) / (gm * ps / pl + 1.0), us, ps
        shl = ul - cl
        stl = us - cl * (ps / pl) ** ((g - 1.0) / (2.0 * g))
        if xi <= shl:
            return rl, ul, pl
        if xi > stl:
            return rl * (ps / pl) ** (1.0 / g), us, ps
        u = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * ul + xi)
        c = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * (ul - xi))
        return rl * (c / cl) ** (2.0 / (g - 1.0)), u, pl * (c / cl) ** (2.0 * g / (g - 1.0))
    if ps > pr:
        sr = ur + cr * math.sqrt((g + 1.0) / (2.0 * g) * ps / pr + (g - 1.0) / (2.0 * g))
        if xi >= sr:
            return rr, ur, pr
        return rr * (ps / pr + gm) / (gm * ps / pr + 1.0), us, ps
    shr = ur + cr
    sth = us + cr * (ps / pr) ** ((g - 1.0) / (2.0 * g))
    if xi >= shr:
        return rr, ur, pr
    if xi <= sth:
        return rr * (ps / pr) ** (1.0 / g), us, ps
    u = 2.0 / (g + 1.0) * (-cr + 0.5 * (g - 1.0) * ur + xi)
    c = 2.0 / (g + 1.0) * (cr - 0.5 * (g - 1.0) * (ur - xi))
    return rr * (c / cr) ** (2.0 / (g - 1.0)), u, pr * (c / cr) ** (2.0 * g / (g - 1.0))


def profile(xs, t, x0, left, right, g):
    """Arrays rho, u, p at positions xs for a single interface at x0 at time t."""
    out = np.array([sample((x - x0) / t, left, right, g) for x in xs])
    return out[:, 0], out[:, 1], out[:, 2]
