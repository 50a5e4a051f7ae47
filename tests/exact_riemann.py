"""Exact solution of the 1-D Riemann problem for the Euler equations of an
ideal gas: the textbook iterative solver (Toro, "Riemann Solvers and
Numerical Methods for Fluid Dynamics", ch. 4), including the case where the
two rarefactions open a vacuum.  Test infrastructure for the oracle pins."""
import math

import numpy as np


def _fK(p, rho, pK, c, g):
    if p > pK:  # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pK
        s = math.sqrt(A / (p + B))
        return (p - pK) * s, s * (1.0 - 0.5 * (p - pK) / (B + p))
    e = (g - 1.0) / (2.0 * g)
    return 2.0 * c / (g - 1.0) * ((p / pK) ** e - 1.0), (p / pK) ** (-(g + 1.0) / (2.0 * g)) / (rho * c)


def star_state(left, right, g):
    """(p*, u*) or None when a vacuum opens between the rarefactions."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    if 2.0 / (g - 1.0) * (cl + cr) <= ur - ul:
        return None
    # two-rarefaction pressure as the Newton start
    e = (g - 1.0) / (2.0 * g)
    p = ((cl + cr - 0.5 * (g - 1.0) * (ur - ul)) / (cl / pl ** e + cr / pr ** e)) ** (1.0 / e)
    p = max(p, 1e-14 * max(pl, pr))
    for _ in range(200):
        fl, dl = _fK(p, rl, pl, cl, g)
        fr, dr = _fK(p, rr, pr, cr, g)
        f = fl + fr + (ur - ul)
        pn = p - f / (dl + dr)
        if pn <= 0.0:
            pn = 0.5 * p
        if abs(pn - p) <= 1e-15 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _fK(p, rl, pl, cl, g)
    fr, _ = _fK(p, rr, pr, cr, g)
    return p, 0.5 * (ul + ur) + 0.5 * (fr - fl)


def sample(left, right, g, s):
    """Primitive (rho, u, p) at similarity coordinate s = (x - xs)/t."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    st = star_state(left, right, g)
    if st is None:  # vacuum between two rarefactions
        shl, stl = ul - cl, ul + 2.0 * cl / (g - 1.0)
        shr, str_ = ur + cr, ur - 2.0 * cr / (g - 1.0)
        if s <= shl:
            return rl, ul, pl
        if s < stl:
            c = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * (ul - s))
            u = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * ul + s)
            r = rl * (c / cl) ** (2.0 / (g - 1.0))
            return r, u, pl * (c / cl) ** (2.0 * g / (g - 1.0))
        if s <= str_:
            return 0.0, s, 0.0
        if s < shr:
            c = 2.0 / (g + 1.0) * (cr - 0.5 * (g - 1.0) * (ur - s))
            u = 2.0 / (g + 1.0) * (-cr + 0.5 * (g - 1.0) * ur + s)
            r = rr * (c / cr) ** (2.0 / (g - 1.0))
            return r, u, pr * (c / cr) ** (2.0 * g / (g - 1.0))
        return rr, ur, pr
    ps, us = st
    gm = (g - 1.0) / (g + 1.0)
    if s <= us:
        if ps > pl:  # left shock
            sl = ul - cl * math.sqrt((g + 1.0) / (2.0 * g) * ps / pl + (g - 1.0) / (2.0 * g))
            if s <= sl:
                return rl, ul, pl
            return rl * (ps / pl + gm) / (gm * ps / pl + 1.0), us, ps
        shl = ul - cl
        csl = cl * (ps / pl) ** ((g - 1.0) / (2.0 * g))
        if s <= shl:
            return rl, ul, pl
        if s >= us - csl:
            return rl * (ps / pl) ** (1.0 / g), us, ps
        c = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * (ul - s))
        u = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * ul + s)
        return rl * (c / cl) ** (2.0 / (g - 1.0)), u, pl * (c / cl) ** (2.0 * g / (g - 1.0))
    if ps > pr:  # right shock
        sr = ur + cr * math.sqrt((g + 1.0) / (2.0 * g) * ps / pr + (g - 1.0) / (2.0 * g))
        if s >= sr:
            return rr, ur, pr
        return rr * (ps / pr + gm) / (gm * ps / pr + 1.0), us, ps
    shr = ur + cr
    csr = cr * (ps / pr) ** ((g - 1.0) / (2.0 * g))
    if s >= shr:
        return rr, ur, pr
    if s <= us + csr:
        return rr * (ps / pr) ** (1.0 / g), us, ps
    c = 2.0 / (g + 1.0) * (cr - 0.5 * (g - 1.0) * (ur - s))
    u = 2.0 / (g + 1.0) * (-cr + 0.5 * (g - 1.0) * ur + s)
    return rr * (c / cr) ** (2.0 / (g - 1.0)), u, pr * (c / cr) ** (2.0 * g / (g - 1.0))


def cell_averages(left, right, g, xs, t, x0, x1, n, sub=64):
    """Cell averages of (rho, u, p) of the exact solution, by a sub-cell midpoint
    rule (the solution is discontinuous, so averages converge at first order in
    1/sub; sub = 64 is far below the scheme errors tested)."""
    dx = (x1 - x0) / n
    out = np.zeros((3, n))
    for i in range(n):
        acc = np.zeros(3)
        for k in range(sub):
            x = x0 + (i + (k + 0.5) / sub) * dx
            acc += sample(left, right, g, (x - xs) / t)
        out[:, i] = acc / sub
    return out
