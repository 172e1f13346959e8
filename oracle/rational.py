"""Exact-rational ACAT oracle for tiny 1D scalar grids (Burgers, advection).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  Every quantity is a
``fractions.Fraction``: the differentiation weights (obtained here from the
moment conditions, a different derivation from the C++ oracle's expanded
Lagrange basis), the indicators (Sec. 3.2), the superbee limiter (Sec. 3.1),
the Rusanov flux, the CAT recursion (Sec. 2.2) and the conservative update.
With dyadic data, dx and dt, the C++ oracle's fp64 result must agree with
this one up to rounding.

The recursion is also available in its literal (unscaled) form, with the
powers of dt written out as in Sec. 2.2, to pin the scaled variables used
everywhere else.
"""
from __future__ import annotations

from fractions import Fraction as Fr
from functools import lru_cache
from math import factorial


def _solve(A, b):
    """Gaussian elimination over the rationals."""
    n = len(A)
    M = [list(map(Fr, row)) + [Fr(bb)] for row, bb in zip(A, b)]
    for col in range(n):
        piv = next(r for r in range(col, n) if M[r][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        for r in range(n):
            if r != col and M[r][col] != 0:
                f = M[r][col] / M[col][col]
                M[r] = [x - f * y for x, y in zip(M[r], M[col])]
    return [M[r][n] / M[r][r] for r in range(n)]


@lru_cache(maxsize=None)
def weights(nodes: tuple, q: Fr, k: int) -> tuple:
    """w with sum_j w_j g(x_j) = g^(k)(q) for every polynomial of degree < len(nodes):
    sum_j w_j (x_j - q)^m = k! delta_{mk}, m = 0..n-1."""
    n = len(nodes)
    A = [[(Fr(x) - q) ** m for x in nodes] for m in range(n)]
    b = [Fr(factorial(k)) if m == k else Fr(0) for m in range(n)]
    return tuple(_solve(A, b))


def stencil(p):
    return tuple(range(-p + 1, p + 1))


@lru_cache(maxsize=None)
def eta(p: int) -> tuple:
    """Interface weights: (A_i - A_{i-1}) equals the centred (2p+1)-point first
    derivative (Sec. 2.1 relation with k = 1)."""
    d = weights(tuple(range(-p, p + 1)), Fr(0), 1)
    e, out = Fr(0), []
    for m in range(-p, p):
        e = e - d[m + p]
        out.append(e)
    assert e - d[2 * p] == 0
    return tuple(out)


def flux(kind, u, a=Fr(1)):
    return a * u if kind == "advection" else u * u / 2


def speed(kind, u, a=Fr(1)):
    return abs(a) if kind == "advection" else abs(u)


def cat_flux(kind, us, p, lam, a=Fr(1)):
    """CAT2p flux from the 2p values us (nodes -p+1..p), scaled variables."""
    J = stencil(p)
    n = 2 * p
    Fh = [[flux(kind, v, a) for v in us]]
    U = [None]
    for k in range(2, 2 * p + 1):
        Uk = [-lam * sum(weights(J, Fr(j), 1)[l] * Fh[k - 2][l] for l in range(n)) for j in J]
        U.append(Uk)
        gk = weights(J, Fr(0), k - 1)
        row = []
        for aj in range(n):
            s = Fr(0)
            for ri, r in enumerate(J):
                w = us[aj] + sum(Fr(r) ** l / factorial(l) * U[l][aj] for l in range(1, k))
                s += gk[ri] * flux(kind, w, a)
            row.append(s)
        Fh.append(row)
    et = eta(p)
    return sum(Fr(1, factorial(k)) * sum(et[l] * Fh[k - 1][l] for l in range(n)) for k in range(1, 2 * p + 1))


def cat_flux_literal(kind, us, p, dt, dx, a=Fr(1)):
    """The same flux with the powers of dt and dx written out (Sec. 2.2)."""
    J = stencil(p)
    n = 2 * p
    ft = [[flux(kind, v, a) for v in us]]          # f~^(k) at the nodes
    ut = [None]                                    # u~^(k)
    for k in range(2, 2 * p + 1):
        uk = [-sum(weights(J, Fr(j), 1)[l] * ft[k - 2][l] for l in range(n)) / dx for j in J]
        ut.append(uk)
        gk = weights(J, Fr(0), k - 1)
        row = []
        for aj in range(n):
            s = Fr(0)
            for ri, r in enumerate(J):
                w = us[aj] + sum((r * dt) ** l / factorial(l) * ut[l][aj] for l in range(1, k))
                s += gk[ri] * flux(kind, w, a)
            row.append(s / dt ** (k - 1))
        ft.append(row)
    et = eta(p)
    return sum(dt ** (k - 1) / factorial(k) * sum(et[l] * ft[k - 1][l] for l in range(n))
               for k in range(1, 2 * p + 1))


def indicator(v, p, eps):
    """psi^p on the 2p values v (nodes -p+1..p), Sec. 3.2."""
    at = lambda j: v[j + p - 1]
    IL = sum((at(j + 1) - at(j)) ** 2 for j in range(-p + 1, 0)) + eps
    IR = sum((at(j + 1) - at(j)) ** 2 for j in range(1, p)) + eps
    I = IL * IR / (IL + IR)
    w = weights(stencil(p), Fr(1, 2), 2 * p - 1)
    tau = (factorial(2 * p - 1) * sum(w[l] * v[l] for l in range(2 * p))) ** 2
    return I / (I + tau)


def superbee(r):
    return max(Fr(0), min(2 * r, Fr(1)), min(r, Fr(2)))


def limiter(v):
    """psi^1 = min(phi(r+), phi(r-)) on values at offsets -1..2 (Sec. 3.1)."""
    dl = v[2] - v[1]
    if dl == 0:   # ratios undefined: constant on the four points -> 1, else 0
        return Fr(1) if (v[1] == v[0] and v[3] == v[2]) else Fr(0)
    return min(superbee((v[3] - v[2]) / dl), superbee((v[1] - v[0]) / dl))


def step(kind, u, P, dt, dx, bc="periodic", eps=Fr(1, 2 ** 40), theta=Fr(1, 2), a=Fr(1), order=None):
    """One ACAT2P step on the list u of Fractions.  order (optional) forces
    the order of every interface (no indicators, no limiter: CAT2p only).
    Returns (u_new, orders)."""
    N = len(u)
    lam = Fr(dt) / Fr(dx)
    per = bc == "periodic"

    def at(i):
        if per:
            return u[i % N]
        return u[min(max(i, 0), N - 1)]

    nI = N if per else N + 1
    off = 0 if per else -1
    F, ords = [], []
    for k in range(nI):
        i = k + off
        if order is not None:
            ps = order if isinstance(order, int) else order[k]
            psi1 = Fr(1)
        else:
            ps = 1
            for p in range(P, 1, -1):
                if indicator([at(i + j) for j in stencil(p)], p, eps) >= theta:
                    ps = p
                    break
            psi1 = limiter([at(i + j) for j in (-1, 0, 1, 2)]) if ps == 1 else None
        f = cat_flux(kind, [at(i + j) for j in stencil(ps)], ps, lam, a)
        if ps == 1 and order is None:
            uL, uR = at(i), at(i + 1)
            al = max(speed(kind, uL, a), speed(kind, uR, a))
            flo = (flux(kind, uL, a) + flux(kind, uR, a)) / 2 - al / 2 * (uR - uL)
            f = psi1 * f + (1 - psi1) * flo
        F.append(f)
        ords.append(ps)
    out = []
    for i in range(N):
        kr = i - off
        kl = (i - 1) % N if per else i
        out.append(u[i] + lam * (F[kl] - F[kr]))
    return out, ords
