"""Seeded synthetic inputs for the ACAT workloads (no ACAT arithmetic here).

This module is the only code shared by the oracle tests and the HIP path:
it builds initial states (conserved variables, float64, SoA) and the
problem parameters of each workload.  It knows the physics needed to turn
primitive variables into conserved ones and nothing of the numerical method.

Workloads (the paper's experiments are analytic initial data, so these are
seeded stand-ins of the same kind):
  burgers_1d   Burgers on [-1,1], periodic, smooth data that steepens into a
               shock (cf. Sec. 5.2);
  euler_1d     1D Euler Riemann data with a smooth density perturbation,
               transmissive boundaries (cf. Sec. 5.3);
  euler_2d     2D Euler on a periodic square: isentropic vortices on a
               uniform flow plus straight contact/shock bands (cf. Sec. 5.5);
  batch_1d     many independent euler_1d problems of uneven sizes and P;
  adjoint_2d   euler_2d at 512^2 plus a smooth target perturbation.
"""
from __future__ import annotations

import math

import numpy as np

DEFAULT_SEED = 200701416
GAMMA = 1.4


def _rng(seed, *stream):
    return np.random.default_rng([seed, *stream] if stream else seed)


def centres(a, b, n):
    """Cell-centre nodes x_i = a + (i + 1/2) dx on [a, b]."""
    dx = (b - a) / n
    return a + (np.arange(n) + 0.5) * dx, dx


def euler1d_conserved(rho, v, p, gamma=GAMMA):
    return np.stack([rho, rho * v, p / (gamma - 1.0) + 0.5 * rho * v * v])


def euler2d_conserved(rho, v, w, p, gamma=GAMMA):
    return np.stack([rho, rho * v, rho * w, p / (gamma - 1.0) + 0.5 * rho * (v * v + w * w)])


# ---------------------------------------------------------------------------
def burgers_1d(seed=DEFAULT_SEED + 0, n=200):
    """u0 = 0.5 + sin(pi x) + sum_{k<=4} (a_k cos k pi x + b_k sin k pi x), a, b ~ U[-0.1, 0.1]."""
    rng = _rng(seed)
    x, dx = centres(-1.0, 1.0, n)
    a = rng.uniform(-0.1, 0.1, 4)
    b = rng.uniform(-0.1, 0.1, 4)
    u = 0.5 + np.sin(np.pi * x)
    for k in range(1, 5):
        u += a[k - 1] * np.cos(k * np.pi * x) + b[k - 1] * np.sin(k * np.pi * x)
    return dict(u=u[None, :].copy(), dx=dx, flux="burgers", P=2, bc="periodic", cfl=0.5, t_final=0.6,
                nvar=1, dim=1)


def euler_1d(seed=DEFAULT_SEED + 1, n=4096, P=4, stream=()):
    """Riemann data at x = 0.5 on [0, 1]: rho, p ~ U[0.1, 1], v ~ U[-0.5, 0.5]
    per side, plus 0.2 sin(5x) on the left density (sin(5x) >= 0 there)."""
    rng = _rng(seed, *stream)
    x, dx = centres(0.0, 1.0, n)
    rl, rr = rng.uniform(0.1, 1.0, 2)
    pl, pr = rng.uniform(0.1, 1.0, 2)
    vl, vr = rng.uniform(-0.5, 0.5, 2)
    left = x < 0.5
    rho = np.where(left, rl + 0.2 * np.sin(5 * x), rr)
    v = np.where(left, vl, vr)
    p = np.where(left, pl, pr)
    return dict(u=euler1d_conserved(rho, v, p), dx=dx, flux="euler", P=P, bc="transmissive", cfl=0.5,
                t_final=0.2, nvar=3, dim=1, gamma=GAMMA)


def _vortex_field(X, Y, L, centres_, eps, gamma):
    dv = np.zeros_like(X); dw = np.zeros_like(X); dT = np.zeros_like(X)
    for (xc, yc), e in zip(centres_, eps):
        for sx in (-L, 0.0, L):
            for sy in (-L, 0.0, L):
                xb = X - (xc + sx)
                yb = Y - (yc + sy)
                r2 = xb * xb + yb * yb
                g = np.exp(0.5 * (1.0 - r2))
                dv += -e / (2 * math.pi) * g * yb
                dw += e / (2 * math.pi) * g * xb
                dT += -(gamma - 1.0) * e * e / (8 * gamma * math.pi ** 2) * g * g
    return dv, dw, dT


AXIS_BANDS = [(1, 0), (0, 1), (1, 0), (0, 1)]


def euler_2d(seed=DEFAULT_SEED + 2, n=2048, L=20.0, nvort=8, nbands=4, P=3, cfl=0.4, dirs=None):
    """Uniform flow (1,1,1,1) + nvort isentropic vortices (strength U[1,5],
    centres at periodic distance >= 4, images over 3x3 periods) + nbands
    straight bands with offset U[0,L) and width U[0.1L, 0.3L], inside which
    p *= U[2,10] and rho *= U[0.5,2]; each band gives two straight
    contact/shock lines.  The lines are axis-aligned by default (dirs): the
    2D indicators inspect only the row and the column through an interface,
    which every axis-aligned line crossing a stencil also crosses, while a
    diagonal line can cut a stencil corner unseen."""
    rng = _rng(seed)
    x, dx = centres(0.0, L, n)
    X, Y = np.meshgrid(x, x, indexing="xy")     # X[i2, i1] = x_{i1}
    gamma = GAMMA
    while True:
        cs = []
        while len(cs) < nvort:
            c = rng.uniform(0.0, L, 2)
            ok = True
            for d in cs:
                ddx = abs(c[0] - d[0]); ddx = min(ddx, L - ddx)
                ddy = abs(c[1] - d[1]); ddy = min(ddy, L - ddy)
                if math.hypot(ddx, ddy) < 4.0:
                    ok = False
                    break
            if ok:
                cs.append(c)
        eps = rng.uniform(1.0, 5.0, nvort)
        dv, dw, dT = _vortex_field(X, Y, L, cs, eps, gamma)
        T = 1.0 + dT
        if T.min() >= 0.3:
            break
    rho = T ** (1.0 / (gamma - 1.0))
    p = rho * T
    v = 1.0 + dv
    w = 1.0 + dw
    dirs = dirs or AXIS_BANDS
    for b in range(nbands):
        d = dirs[b % 4]
        off = rng.uniform(0.0, L)
        width = rng.uniform(0.1 * L, 0.3 * L)
        pf = rng.uniform(2.0, 10.0)
        rf = rng.uniform(0.5, 2.0)
        s = np.mod(d[0] * X + d[1] * Y - off, L)
        inside = s < width
        p = np.where(inside, p * pf, p)
        rho = np.where(inside, rho * rf, rho)
    u = euler2d_conserved(rho, v, w, p, gamma)
    return dict(u=np.ascontiguousarray(u), dx=dx, dy=dx, flux="euler", P=P, bc="periodic", cfl=cfl, nsteps=100,
                nvar=4, dim=2, gamma=gamma, L=L)


def batch_1d(seed=DEFAULT_SEED + 3, nprob=256, nmin=512, nmax=16384):
    """nprob euler_1d problems, N_b = round(exp(U[ln nmin, ln nmax])), P_b ~ U{2,3,4},
    problem b drawn from the stream (seed, b)."""
    rng = _rng(seed)
    Ns = np.rint(np.exp(rng.uniform(math.log(nmin), math.log(nmax), nprob))).astype(np.int64)
    Ps = rng.integers(2, 5, nprob)
    probs = [euler_1d(seed, n=int(Ns[b]), P=int(Ps[b]), stream=(b,)) for b in range(nprob)]
    return dict(problems=probs, N=Ns, P=Ps, cfl=0.5, nsteps=500)


def adjoint_2d(seed=DEFAULT_SEED + 4, n=512, nbumps=8, amp=1e-2, sigma=1.5, ndirs=32):
    """euler_2d at n^2 with P = 2; target initial state u0* = u0 + Gaussian
    bumps of amplitude amp on rho and E; ndirs smooth unit-sup-norm directions."""
    base = euler_2d(seed, n=n, P=2, cfl=0.4)
    rng = _rng(seed, 1)
    L = base["L"]
    x, _ = centres(0.0, L, n)
    X, Y = np.meshgrid(x, x, indexing="xy")
    bump = np.zeros_like(X)
    for _ in range(nbumps):
        c = rng.uniform(0.0, L, 2)
        ddx = np.mod(X - c[0] + L / 2, L) - L / 2
        ddy = np.mod(Y - c[1] + L / 2, L) - L / 2
        bump += amp * np.exp(-(ddx * ddx + ddy * ddy) / (2 * sigma * sigma))
    target0 = base["u"].copy()
    target0[0] += bump
    target0[3] += bump
    base.update(target_u0=target0, nsteps=200, checkpoint_every=20)
    base["directions"] = lambda k, shape=base["u"].shape: smooth_direction(seed, k, shape)
    return base


def smooth_direction(seed, k, shape):
    """Seeded smooth random direction (Gaussian noise smoothed by periodic
    averaging along the last two axes), scaled to unit sup norm."""
    rng = _rng(seed, 2, k)
    d = rng.standard_normal(shape)
    for _ in range(4):
        for ax in (-1, -2):
            d = (np.roll(d, 1, axis=ax) + 2 * d + np.roll(d, -1, axis=ax)) / 4
    return d / np.abs(d).max()


# ---------------------------------------------------------------------------
# The paper's own experiments (Sec. 5), with the printed initial data, grids,
# CFL numbers and final times.  Each returns the same dict as above plus
# `t_final` and, for Riemann problems, the primitive left/right states.
RIEMANN_1D = {
    # Sec. 5.3: discontinuity at x = 1/2 on [0, 1], 200 points, CFL 0.8
    "sod": dict(left=(1.0, 0.0, 1.0), right=(0.125, 0.0, 0.1), n=200, cfl=0.8, t_final=0.25),
    "einfeldt123": dict(left=(1.0, -2.0, 0.4), right=(1.0, 2.0, 0.4), n=200, cfl=0.8, t_final=0.15),
    "blast_right": dict(left=(1.0, 0.0, 1000.0), right=(1.0, 0.0, 0.01), n=450, cfl=0.8, t_final=0.012),
}


def paper_riemann_1d(name, n=None, P=3):
    """Shock-tube problems of the 1D Euler experiments (Sec. 5.3); outflow
    (transmissive) boundaries, gamma = 1.4."""
    c = RIEMANN_1D[name]
    n = n or c["n"]
    x, dx = centres(0.0, 1.0, n)
    (rl, ul, pl), (rr, ur, pr) = c["left"], c["right"]
    left = x < 0.5
    u = euler1d_conserved(np.where(left, rl, rr), np.where(left, ul, ur), np.where(left, pl, pr))
    return dict(u=u, dx=dx, flux="euler", P=P, bc="transmissive", cfl=c["cfl"], t_final=c["t_final"], nvar=3,
                dim=1, gamma=GAMMA, left=c["left"], right=c["right"], x=x)


def paper_scalar_1d(name, n=160, P=3):
    """Scalar experiments of Sec. 5.1-5.2 on [0, 2], periodic, CFL 0.9:
    transport of 1/2 sin(pi x) (t = 4) or of the square wave (t = 2),
    Burgers from 1/2 sin(pi x) (t = 1)."""
    x, dx = centres(0.0, 2.0, n)
    if name == "transport_sine":
        u, flux, t = 0.5 * np.sin(np.pi * x), "advection", 4.0
    elif name == "transport_square":
        u = np.where((x >= 0.5) & (x <= 1.0), 1.0, np.where((x > 1.0) & (x <= 1.5), -1.0, 0.0))
        flux, t = "advection", 2.0
    elif name == "burgers_sine":
        u, flux, t = 0.5 * np.sin(np.pi * x), "burgers", 1.0
    else:
        raise KeyError(name)
    return dict(u=u[None, :].copy(), dx=dx, flux=flux, P=P, bc="periodic", cfl=0.9, t_final=t, nvar=1, dim=1,
                x=x, ax=1.0)


LAX_LIU = {
    # Sec. 5.5 tables of the 2D Riemann problems: quadrant -> (rho, u, v, p);
    # quadrant 1: x > 1/2, y > 1/2; 2: x < 1/2, y > 1/2; 3: x < 1/2, y < 1/2; 4: x > 1/2, y < 1/2
    4: dict(q={1: (1.1, 0.0, 0.0, 1.1), 2: (0.5065, 0.8939, 0.0, 0.35), 3: (1.1, 0.8939, 0.8939, 1.1),
               4: (0.5065, 0.0, 0.8939, 0.35)}, t_final=0.25),
    6: dict(q={1: (1.0, 0.75, -0.5, 1.0), 2: (2.0, 0.75, 0.5, 1.0), 3: (1.0, -0.75, 0.5, 1.0),
               4: (3.0, -0.75, -0.5, 1.0)}, t_final=0.3),
    8: dict(q={1: (0.5197, 0.1, 0.1, 0.4), 2: (1.0, -0.6259, 0.1, 1.0), 3: (0.8, 0.1, 0.1, 1.0),
               4: (1.0, 0.1, -0.6259, 1.0)}, t_final=0.25),
}


def paper_lax_liu(config, n=400, P=2):
    """2D Riemann problems of Sec. 5.5 on [0, 1]^2 (free, i.e. transmissive,
    boundaries, CFL 0.475 with the halved 2D rule)."""
    c = LAX_LIU[config]
    x, dx = centres(0.0, 1.0, n)
    X, Y = np.meshgrid(x, x, indexing="xy")
    quad = np.where(X > 0.5, np.where(Y > 0.5, 1, 4), np.where(Y > 0.5, 2, 3))
    prim = np.zeros((4,) + X.shape)
    for q, st in c["q"].items():
        for k in range(4):
            prim[k] = np.where(quad == q, st[k], prim[k])
    u = euler2d_conserved(prim[0], prim[1], prim[2], prim[3])
    return dict(u=np.ascontiguousarray(u), dx=dx, dy=dx, flux="euler", P=P, bc="transmissive", cfl=0.475,
                t_final=c["t_final"], nvar=4, dim=2, gamma=GAMMA)


def paper_transport_2d(n=100, P=2):
    """2D transport u_t + u_x + u_y = 0 on [0, 2]^2 from the indicator of
    x + y <= 1/4, free boundaries, CFL 0.5, t = 1 (Sec. 5.4)."""
    x, dx = centres(0.0, 2.0, n)
    X, Y = np.meshgrid(x, x, indexing="xy")
    u = np.where(X + Y <= 0.25, 1.0, 0.0)[None]
    return dict(u=np.ascontiguousarray(u), dx=dx, dy=dx, flux="advection", P=P, bc="transmissive", cfl=0.5,
                t_final=1.0, nvar=1, dim=2, ax=1.0, ay=1.0)
