"""Exact solution of the Riemann problem for the 1D Euler equations of an
ideal gas (TEST INFRASTRUCTURE ONLY: the reference for the error checks of
the paper's shock-tube experiments, Sec. 5.3; the GPU library never uses it).

The textbook construction: the star-region pressure p* is the root of
    f(p) = f_L(p) + f_R(p) + (u_R - u_L) = 0,
where f_K is the shock (Rankine-Hugoniot) branch for p > p_K and the
rarefaction (isentropic, Riemann-invariant) branch for p <= p_K; then
u* = (u_L + u_R)/2 + (f_R(p*) - f_L(p*))/2, and the solution at x/t is
sampled wave by wave (left wave, contact at u*, right wave).
Vacuum-generating data are rejected.
"""
from __future__ import annotations

import math

import numpy as np


def _sound(g, rho, p):
    return math.sqrt(g * p / rho)


def _fk(g, p, rho, pk, ck):
    """Velocity jump across the K-wave as a function of the star pressure, and its derivative."""
    if p > pk:   # shock
        a = 2.0 / ((g + 1.0) * rho)
        b = (g - 1.0) / (g + 1.0) * pk
        s = math.sqrt(a / (p + b))
        return (p - pk) * s, s * (1.0 - 0.5 * (p - pk) / (p + b))
    # rarefaction
    e = (g - 1.0) / (2.0 * g)
    return 2.0 * ck / (g - 1.0) * ((p / pk) ** e - 1.0), (p / pk) ** (-(g + 1.0) / (2.0 * g)) / (rho * ck)


def star_state(left, right, gamma=1.4, tol=1e-15, maxit=100):
    """(p*, u*) of the Riemann problem with primitive states (rho, u, p)."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = _sound(gamma, rl, pl), _sound(gamma, rr, pr)
    if 2.0 * (cl + cr) / (gamma - 1.0) <= ur - ul:
        raise ValueError("the data generate a vacuum")
    p = max(0.5 * (pl + pr), 1e-12)
    for _ in range(maxit):
        fl, dl = _fk(gamma, p, rl, pl, cl)
        fr, dr = _fk(gamma, p, rr, pr, cr)
        pn = p - (fl + fr + ur - ul) / (dl + dr)
        if pn <= 0.0:
            pn = 0.5 * p
        if abs(pn - p) <= tol * 0.5 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _fk(gamma, p, rl, pl, cl)
    fr, _ = _fk(gamma, p, rr, pr, cr)
    return p, 0.5 * (ul + ur) + 0.5 * (fr - fl)


def sample(left, right, xi, gamma=1.4):
    """Primitive state (rho, u, p) at similarity coordinate xi = (x - x0)/t."""
    g = gamma
    rl, ul, pl = left
    rr, ur, pr = right
    ps, us = star_state(left, right, g)
    if xi <= us:   # left of the contact
        cl = _sound(g, rl, pl)
        if ps > pl:   # left shock
            s = ul - cl * math.sqrt((g + 1.0) / (2.0 * g) * ps / pl + (g - 1.0) / (2.0 * g))
            if xi <= s:
                return rl, ul, pl
            r = rl * (ps / pl + (g - 1.0) / (g + 1.0)) / ((g - 1.0) / (g + 1.0) * ps / pl + 1.0)
            return r, us, ps
        # left rarefaction
        rs = rl * (ps / pl) ** (1.0 / g)
        cs = cl * (ps / pl) ** ((g - 1.0) / (2.0 * g))
        if xi <= ul - cl:
            return rl, ul, pl
        if xi >= us - cs:
            return rs, us, ps
        u = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * ul + xi)
        c = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * (ul - xi))
        r = rl * (c / cl) ** (2.0 / (g - 1.0))
        return r, u, pl * (c / cl) ** (2.0 * g / (g - 1.0))
    cr = _sound(g, rr, pr)
    if ps > pr:   # right shock
        s = ur + cr * math.sqrt((g + 1.0) / (2.0 * g) * ps / pr + (g - 1.0) / (2.0 * g))
        if xi >= s:
            return rr, ur, pr
        r = rr * (ps / pr + (g - 1.0) / (g + 1.0)) / ((g - 1.0) / (g + 1.0) * ps / pr + 1.0)
        return r, us, ps
    rs = rr * (ps / pr) ** (1.0 / g)
    cs = cr * (ps / pr) ** ((g - 1.0) / (2.0 * g))
    if xi >= ur + cr:
        return rr, ur, pr
    if xi <= us + cs:
        return rs, us, ps
    u = 2.0 / (g + 1.0) * (-cr + 0.5 * (g - 1.0) * ur + xi)
    c = 2.0 / (g + 1.0) * (cr - 0.5 * (g - 1.0) * (ur - xi))
    r = rr * (c / cr) ** (2.0 / (g - 1.0))
    return r, u, pr * (c / cr) ** (2.0 * g / (g - 1.0))


def solution(left, right, x, t, x0=0.5, gamma=1.4):
    """Primitive variables (rho, u, p) at the points x at time t > 0 (arrays)."""
    out = np.array([sample(left, right, (xx - x0) / t, gamma) for xx in np.asarray(x, dtype=float)])
    return out[:, 0], out[:, 1], out[:, 2]
