"""Algorithmic FP64 operation counts of the ACAT flux computations.

Convention: add, sub, mul, div and sqrt count 1 flop each, a fused
multiply-add counts 2.  The counts are those of the method's own steps for
the order actually selected at each interface or corner (Sec. 2.2 recursion
in 1D; Sec. 4 corner recursion on the rectangle J_q1 x J_q2, with the last
recursion step restricted to the nodes the final fluxes read, i.e. row
j2 = 0 for F and column j1 = 0 for G, as Sec. 4 allows).  They do not count
work an implementation adds (idle lanes, recomputation, index arithmetic).

Flux evaluations (distinct operations, shared subexpressions once):
  2D Euler f and g at one state: 1/rho, v, w, mx v, my w, their sum, 1/2,
      E -, (gamma-1) x  -> p (9); E + p; mx v + p; my v; v (E+p); mx w;
      my w + p; w (E+p)                                       = 16
  2D Euler f only (or g only)                                  = 13
  1D Euler f: v = m/rho, m v, 1/2, E -, (gamma-1) x, m v + p, E + p, v (E+p) = 8
  Burgers f = (u u)/2                                          = 2
  advection f = a u                                            = 1 per variable
"""
from __future__ import annotations

C_FG_EULER2D = 16
C_F_EULER2D = 13
C_F = {("euler", 1): 8, ("burgers", 1): 2, ("advection", 1): 1}


def _pass_2d(n1, n2, qt, do_f, do_g, s, cfg, cf):
    """One corner recursion on an n1 x n2 rectangle, time half-width qt."""
    T = 2 * qt
    R = n1 * n2
    u_cost = s * (2 * n1 + 2 * n2 + 3)           # x and y derivatives, two scalings, one subtraction
    total = 0
    for kk in range(2, T + 1):
        w_cost = 2 * s * (kk - 1)                # Taylor prediction of one state
        if kk < T:
            total += R * u_cost
            total += R * (T - 1) * (w_cost + cfg)
            total += R * 2 * (2 * s * T)         # Fh and Gh time derivatives
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
                    total += (T - 1) * (w_cost + (cfg if (need_f and need_g) else cf))
                    total += (int(need_f) + int(need_g)) * 2 * s * T
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
        total += n * s * (2 * n + 1)             # spatial derivative and scaling
        total += n * (T - 1) * (2 * s * (kk - 1) + cf)
        total += n * s * 2 * T
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
