"""Algorithmic FP64 operation counts of the ACAT flux computations.

Convention: add, sub, mul, div and sqrt count 1 flop each, a fused
multiply-add counts 2.  The counts are those of the method's own steps for
the order actually selected at each interface or corner (Sec. 2.2 recursion
in 1D; Sec. 4 corner recursion on the rectangle J_q1 x J_q2, with the last
recursion step restricted to the nodes the final fluxes read, i.e. row
j2 = 0 for F and column j1 = 0 for G, as Sec. 4 allows).  A time node whose
weight in the time-derivative approximation of a level is exactly zero (on
the 2q nodes -q+1..q the even-order weights of node r = q vanish) adds
nothing to that level's sum: its flux evaluation and weighted term are not
counted, as the forward kernels skip them; its Taylor prediction is, since
later levels read it.  The adjoint's count keeps every time node: its
kernels evaluate them all.  The Taylor
predictions u + sum_{l<k} (r dt)^l/l! u~^(l) at the time nodes are counted
in their incremental form, one term added per level (the same sums: each
level extends the previous level's partial sum), not re-summed from u at
every level.  They do not count work an implementation adds (idle lanes,
recomputation, index arithmetic).

Flux evaluations (distinct operations, shared subexpressions once):
  2D Euler f and g at one state: 1/rho, v, w, mx v, my w, their sum, 1/2,
      E -, (gamma-1) x  -> p (9); E + p; mx v + p; my v; v (E+p); mx w;
      my w + p; w (E+p)                                       = 16
  2D Euler f only (or g only)                                  = 13
  1D Euler f: v = m/rho, m v, 1/2, E -, (gamma-1) x, m v + p, E + p, v (E+p) = 8
  Burgers f = (u u)/2                                          = 2
  advection f = a u                                            = 1 per variable

Adjoint (reverse mode) of one 2D corner, adjoint_corner_flops_2d: the
forward recursion up to U^{T-1} (its values are the linearisation points;
U^{T-1} only on the row and column the fluxes read),
then the reverse sweep: per level and node, the time-derivative weights
applied to the incoming adjoint, the Jacobian-transpose products at the
T-1 predicted states, the adjoint of the Taylor predictions, and the
transposed centred differences; the last level only on the row and column
the fluxes read; finally the Jacobian-transpose products at the node
state.  Predictions the reverse sweep recomputes instead of storing are not
counted.
  2D Euler f'(u)^T fb + g'(u)^T gb (analytic, primitive variables once) = 58
  2D advection                                                          = 3
"""
from __future__ import annotations

from fractions import Fraction
from functools import lru_cache

C_FG_EULER2D = 16
C_F_EULER2D = 13
C_F = {("euler", 1): 8, ("burgers", 1): 2, ("advection", 1): 1}
V_FG_EULER2D = 58


@lru_cache(maxsize=None)
def time_nodes(qt: int, k: int):
    """(weighted nodes, weighted nodes other than r = 0) of the order-k
    time-derivative approximation at r = 0 on the nodes r = -qt+1..qt: the
    weight of node r is k! times the x^k coefficient of its Lagrange basis
    polynomial, computed exactly."""
    nodes = list(range(-qt + 1, qt + 1))
    nz = nzf = 0
    for r in nodes:
        poly = [Fraction(1)]                     # coefficients, lowest degree first
        for m in nodes:
            if m == r:
                continue
            nxt = [Fraction(0)] * (len(poly) + 1)
            for i, a in enumerate(poly):         # poly * (x - m) / (r - m)
                nxt[i + 1] += a / (r - m)
                nxt[i] -= a * m / (r - m)
            poly = nxt
        if poly[k] != 0:
            nz += 1
            nzf += r != 0
    return nz, nzf


def _pass_2d(n1, n2, qt, do_f, do_g, s, cfg, cf):
    """One corner recursion on an n1 x n2 rectangle, time half-width qt."""
    T = 2 * qt
    R = n1 * n2
    u_cost = s * (2 * n1 + 2 * n2 + 3)           # x and y derivatives, two scalings, one subtraction
    total = 0
    for kk in range(2, T + 1):
        w_cost = 2 * s                           # one more term of the Taylor prediction of one state
        nz, nzf = time_nodes(qt, kk - 1)
        if kk < T:
            total += R * u_cost
            total += R * ((T - 1) * w_cost + nzf * cfg)
            total += R * 2 * (2 * s * nz)        # Fh and Gh time derivatives
        else:
            a1c = n1 // 2 - 1                    # column index of j1 = 0
            a2c = n2 // 2 - 1                    # row index of j2 = 0
            for a2 in range(n2):
                for a1 in range(n1):
                    need_f = do_f and a2 == a2c
                    need_g = do_g and a1 == a1c
                    if not (need_f or need_g):
                        continue
                    total += u_cost
                    total += (T - 1) * w_cost + nzf * (cfg if (need_f and need_g) else cf)
                    total += (int(need_f) + int(need_g)) * 2 * s * nz
    if do_f:
        total += T * s * (2 * n1 + 2)            # sum_k (1/k!) sum_l eta_l Fh^{k-1}
    if do_g:
        total += T * s * (2 * n2 + 2)
    return total


def corner_flops_2d(q1: int, q2: int, s: int = 4, cfg: int = C_FG_EULER2D, cf: int = C_F_EULER2D) -> int:
    """Algorithmic flops of the F and G fluxes of one 2D corner of class (q1, q2)."""
    n1, n2 = 2 * q1, 2 * q2
    total = n1 * n2 * cfg                        # f, g at the stencil nodes
    if q1 == q2:
        total += _pass_2d(n1, n2, q1, True, True, s, cfg, cf)
    else:
        total += _pass_2d(n1, n2, q1, True, False, s, cfg, cf)
        total += _pass_2d(n1, n2, q2, False, True, s, cfg, cf)
    blend = cf + 10 * s                          # f at the neighbour, Rusanov flux, psi blend
    if q1 == 1:
        total += blend
    if q2 == 1:
        total += blend
    return total


def interface_flops_1d(p: int, s: int, cf: int) -> int:
    """Algorithmic flops of one 1D interface flux of order p."""
    n = T = 2 * p
    total = n * cf
    for kk in range(2, T + 1):
        nz, nzf = time_nodes(p, kk - 1)
        total += n * s * (2 * n + 1)             # spatial derivative and scaling
        total += n * ((T - 1) * 2 * s + nzf * cf)   # one more prediction term; flux at the weighted ones
        total += n * s * 2 * nz
    total += T * s * (2 * n + 2)
    if p == 1:
        total += cf + 10 * s
    return total


def classify_flops(P: int, s: int, dim: int) -> int:
    """Indicators for p = P..2 (upper bound: all evaluated) per interface."""
    per = 0
    for p in range(2, P + 1):
        n = 2 * p
        # 2(p-1) differences squared and summed, 2 eps adds, I, tau sum, tau scale/square, psi
        per += s * (3 * 2 * (p - 1) + 2 + 4 + 2 * n + 2 + 2)
    return per * (2 if dim == 2 else 1)


def update_flops(s: int, dim: int) -> int:
    return s * (3 if dim == 1 else 6)


def _adj_pass_2d(n1, n2, qt, do_f, do_g, s, cfg, vfg):
    """Reverse of one corner recursion (forward part up to U^{T-1} included)."""
    T = 2 * qt
    R = n1 * n2
    u_cost = s * (2 * n1 + 2 * n2 + 3)
    ut_cost = s * (2 * n1 + 2 * n2 + 4)          # transposed differences, scalings, series term
    nlast = (n1 if do_f else 0) + (n2 if do_g else 0) - (1 if (do_f and do_g) else 0)
    total = 0
    # forward: U^1 .. U^{T-1} (U^{T-1} only where the last level's predictions
    # are read: the row and column of the fluxes), Fh/Gh up to level T-2,
    # predictions up to level T-1
    for kk in range(2, T + 1):
        total += (R if kk < T else nlast) * u_cost
        if kk < T:
            total += R * (T - 1) * (2 * s + cfg)
            total += R * 2 * (2 * s * T)
    # reverse; the incremental predictions W_r(k) = W_r(k-1) + r^{k-1}/(k-1)! U^{k-1}
    # reverse into a running adjoint of W_r (s adds) and one term of U's adjoint (2s)
    for kk in range(T, 1, -1):
        nodes = nlast if kk == T else R
        w = 2 * s if kk == T else 0              # last prediction term (the forward stopped at T-1)
        per_r = 2 * s + w + vfg + s + 2 * s      # scale, prediction, vjp, running adjoint, U term
        total += nodes * ((T - 1) * per_r + 4 * s)
        total += (nlast if kk == T else R) * ut_cost
    total += R * (T - 1) * s                     # prediction adjoints into u
    return total


def adjoint_corner_flops_2d(q1: int, q2: int, s: int = 4, cfg: int = C_FG_EULER2D,
                            vfg: int = V_FG_EULER2D) -> int:
    """Algorithmic flops of the adjoint of one 2D corner of class (q1, q2)."""
    n1, n2 = 2 * q1, 2 * q2
    total = n1 * n2 * (cfg + vfg + 4 * s)        # f, g at the nodes; final transpose products; f0b/g0b sums
    if q1 == q2:
        total += _adj_pass_2d(n1, n2, q1, True, True, s, cfg, vfg)
    else:
        total += _adj_pass_2d(n1, n2, q1, True, False, s, cfg, vfg)
        total += _adj_pass_2d(n1, n2, q2, False, True, s, cfg, vfg)
    total += 2 * 3 * s                           # flux adjoints from the update transpose
    if q1 == 1:
        total += 2 * 4 * s
    if q2 == 1:
        total += 2 * 4 * s
    return total


def adjoint_corner_bytes_2d(q1: int, q2: int, s: int = 4) -> int:
    """Compulsory HBM bytes per corner of the 2D adjoint kernel of class
    (q1, q2), as a launch over a grid with about one corner per cell moves
    them: the state and the incoming adjoint of one cell (each cell is read
    once if neighbouring corners share it in cache), the recorded superbee
    weight and Rusanov speed of each order-1 direction, the list entry, and
    the written per-node contributions, one value per component at each of
    the (2 q1)(2 q2) stencil nodes."""
    nodes = (2 * q1) * (2 * q2)
    dec = 16 * ((q1 == 1) + (q2 == 1))
    return 8 * s + 8 * s + dec + 4 + 8 * s * nodes
