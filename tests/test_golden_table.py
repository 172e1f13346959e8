"""Oracle pins from the paper's table of numerical methods (tests/golden/
method_table.txt): the stencil of an ACAT2P update has 2P+1 points (the
Jacobian of the frozen step is banded with half-width exactly P) and its
order of accuracy is 2P (measured on smooth periodic advection); FL-CAT2
has a 3-point stencil and order 2."""
import os
import re

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "method_table.txt")


def table():
    rows = {}
    for line in open(GOLDEN):
        line = line.split("#")[0].strip()
        if line:
            name, pts, order = line.split()
            rows[name] = (pts, order)
    return rows


def expected(P):
    t = table()
    if P == 1:
        pts, order = t["FL-CAT2"]
        return int(pts), int(order)
    pts, order = t["ACAT2P"]

    def ev(expr):   # "2P+1" -> 2 * P + 1
        return int(eval(re.sub(r"(\d)P", r"\1*P", expr), {"P": P}))
    return ev(pts), ev(order)


def jacobian_1d(pb, u, dt, maps):
    n = u.size
    J = np.zeros((n, n))
    e = np.zeros(n)
    for j in range(n):
        e[j] = 1.0
        J[:, j] = oracle.jvp(pb, u, e.reshape(u.shape), dt, maps)[1].ravel()
        e[j] = 0.0
    return J


@pytest.mark.parametrize("P", [1, 2, 3, 4])
def test_stencil_points_match_table(P):
    n = 32
    x = (np.arange(n) + 0.5) / n
    u = (1.0 + 0.3 * np.sin(2 * np.pi * x))[None, :]
    pb = oracle.Problem(dim=1, nvar=1, nx=n, flux=oracle.FLUX_BURGERS, P=P, bc=oracle.BC_PERIODIC, dx=1.0 / n)
    dt = 0.5 / n
    maps = (np.full(n, P, np.int8), np.full(n, 0.5 if P == 1 else -1.0), np.full(n, 1.3 if P == 1 else -1.0))
    J = jacobian_1d(pb, u, dt, maps)
    pts, _ = expected(P)
    half = (pts - 1) // 2
    for i in range(n):
        d = (np.arange(n) - i + n // 2) % n - n // 2          # periodic offset j - i
        nz = np.abs(J[i]) > 0
        assert np.all(np.abs(d[nz]) <= half)
        assert nz[(i + half) % n] and nz[(i - half) % n]


@pytest.mark.parametrize("P", [2, 3])
def test_order_matches_table(P):
    _, order = expected(P)
    Ns = (40, 80) if P == 3 else (80, 160)
    errs = []
    for N in Ns:
        x = -1 + (np.arange(N) + 0.5) * 2 / N
        pb = oracle.Problem(dim=1, nvar=1, nx=N, flux=oracle.FLUX_ADVECTION, P=P, bc=oracle.BC_PERIODIC,
                            dx=2 / N, ax=1.0)
        u, t, n = oracle.run(pb, 0.5 * np.sin(np.pi * x + 0.3)[None], 0.8, t_final=0.5)
        errs.append(np.abs(u[0] - 0.5 * np.sin(np.pi * (x - t) + 0.3)).max())
    rate = np.log2(errs[0] / errs[1])
    assert rate > order - 0.35, (errs, rate)
