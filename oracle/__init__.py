"""ACAT oracle: plain CPU reference of one ACAT time step (arXiv:2007.01416).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the HIP library in ``paper_2007_01416_amd``: its arithmetic lives in
``acat_oracle.cpp`` (plain C++ loops, fp64, built with -ffp-contract=off so
the compiler fuses nothing) and in ``rational.py`` (exact rationals for tiny
scalar grids).

Two frozen rounding modes (``Problem.rounding``): "fixed" (default) writes
the recursion's weighted sums, the 2D U^k and the 2D Euler flux's
product-sums as explicit fused multiply-adds in index order and sums the
final flux node by node; "plain" rounds every product and every sum
separately, in the order the paper writes the formulas (final flux k-outer,
U^k as -lamx sum - lamy sum, velocities m / rho).  The two agree to rounding;
parity at a tolerance against "plain" checks arithmetic whose rounding no
implementation chose.

Functions here marshal numpy arrays to the C++ oracle and implement the time
step rules (1D: dt = CFL dx / max spectral radius; 2D: Sec. 5.5,
dt = CFL/2 min(dx/sx, dy/sy)).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "acat_oracle.cpp")
_LIB = os.path.join(_HERE, "_oracle.so")

FLUX_ADVECTION, FLUX_BURGERS, FLUX_EULER = 0, 1, 2
BC_PERIODIC, BC_TRANSMISSIVE = 0, 1
# variants (Problem.flags): first-order flux Lax-Friedrichs / HLL instead of
# Rusanov, modified p = 2 indicator, Roe-speed upwind psi^1 (scalar laws)
FLAG_FLO_LF, FLAG_FLO_HLL, FLAG_PSI2_MODIFIED, FLAG_PSI1_ROE, FLAG_SQUARE_2D = 1, 2, 4, 8, 16
_FLAG_PLAIN_ROUNDING = 256      # set from Problem.rounding == "plain"


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (-O2, no implicit FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB):
        cmd = ["g++", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-shared", "-fPIC",
               "-o", _LIB + ".tmp", _SRC]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Problem(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("nvar", ctypes.c_int32),
                ("nx", ctypes.c_int64), ("ny", ctypes.c_int64),
                ("flux", ctypes.c_int32), ("P", ctypes.c_int32), ("bc", ctypes.c_int32),
                ("flags", ctypes.c_int32),
                ("gamma", ctypes.c_double), ("ax", ctypes.c_double), ("ay", ctypes.c_double),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double),
                ("eps", ctypes.c_double), ("theta", ctypes.c_double)]


@dataclass
class Problem:
    dim: int
    nvar: int
    nx: int
    ny: int = 1
    flux: int = FLUX_EULER
    P: int = 2
    bc: int = BC_PERIODIC
    gamma: float = 1.4
    ax: float = 1.0
    ay: float = 1.0
    dx: float = 1.0
    dy: float = 1.0
    eps: float = 1e-12
    theta: float = 0.5
    flags: int = 0      # FLAG_* variants (default method: 0)
    rounding: str = "fixed"   # "fixed" or "plain" (see the module docstring)

    def c(self) -> _Problem:
        if self.rounding not in ("fixed", "plain"):
            raise ValueError(f"rounding {self.rounding!r}")
        flags = self.flags | (_FLAG_PLAIN_ROUNDING if self.rounding == "plain" else 0)
        return _Problem(self.dim, self.nvar, self.nx, self.ny, self.flux, self.P, self.bc, flags,
                        self.gamma, self.ax, self.ay, self.dx, self.dy, self.eps, self.theta)

    @property
    def n_interfaces(self):
        """(x-interfaces per row, y-interfaces per column)."""
        ext = 0 if self.bc == BC_PERIODIC else 1
        return self.nx + ext, (self.ny + ext if self.dim == 2 else 0)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        d, i8, i64 = P(ctypes.c_double), P(ctypes.c_int8), P(ctypes.c_int64)
        L.oracle_coeffs.argtypes = [ctypes.c_int, d, d, d, d, d]
        L.oracle_indicator.argtypes = [d, ctypes.c_int, ctypes.c_double]
        L.oracle_indicator.restype = ctypes.c_double
        L.oracle_limiter.argtypes = [d]
        L.oracle_limiter.restype = ctypes.c_double
        L.oracle_indicator2_modified.argtypes = [d, ctypes.c_double]
        L.oracle_indicator2_modified.restype = ctypes.c_double
        L.oracle_step1d.argtypes = [P(_Problem), d, d, ctypes.c_double, ctypes.c_int, i8, d, d, d, ctypes.c_int]
        L.oracle_step1d_jvp.argtypes = [P(_Problem), d, d, d, d, ctypes.c_double, i8, d, d, ctypes.c_int]
        L.oracle_step2d.argtypes = [P(_Problem), d, d, ctypes.c_double, ctypes.c_int, i8, i8, d, d, d, d, d, d,
                                    ctypes.c_int]
        L.oracle_step2d_jvp.argtypes = [P(_Problem), d, d, d, d, ctypes.c_double, i8, i8, d, d, d, d, ctypes.c_int]
        L.oracle_step2d_jvp2.argtypes = [P(_Problem), d, d, d, d, ctypes.c_double, i8, i8, d, d, d, d, ctypes.c_int,
                                         ctypes.c_int]
        L.oracle_update_cells.argtypes = [P(_Problem), d, ctypes.c_double, ctypes.c_int64, i64, d, i8, ctypes.c_int]
        L.oracle_max_speed.argtypes = [P(_Problem), d, d]
        _lib = L
    return _lib


def _p(a, ct=ctypes.c_double):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _chk(rc):
    if rc != 0:
        raise ValueError(f"oracle returned {rc}")


def coeffs(p: int) -> dict:
    """Coefficient tables for half-width p: g1[j][l], gt[k][r], eta, tau, d1."""
    n = 2 * p
    g1 = np.zeros((n, n)); gt = np.zeros((n, n)); eta = np.zeros(n); tau = np.zeros(n)
    d1 = np.zeros(2 * p + 1)
    _chk(lib().oracle_coeffs(p, _p(g1), _p(gt), _p(eta), _p(tau), _p(d1)))
    return dict(g1=g1, gt=gt, eta=eta, tau=tau, d1=d1)


def indicator(v, p: int, eps: float = 1e-12) -> float:
    v = np.ascontiguousarray(v, dtype=np.float64)
    assert v.shape == (2 * p,)
    return lib().oracle_indicator(_p(v), p, eps)


def limiter(v) -> float:
    v = np.ascontiguousarray(v, dtype=np.float64)
    assert v.shape == (4,)
    return lib().oracle_limiter(_p(v))


def indicator2_modified(v, eps: float = 1e-12) -> float:
    """Modified p = 2 indicator (Sec. 3.2) on values at offsets -1..2."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    assert v.shape == (4,)
    return lib().oracle_indicator2_modified(_p(v), eps)


def _state(prob: Problem, u):
    u = np.ascontiguousarray(u, dtype=np.float64)
    shape = (prob.nvar, prob.nx) if prob.dim == 1 else (prob.nvar, prob.ny, prob.nx)
    if u.shape != shape:
        raise ValueError(f"state shape {u.shape} != {shape}")
    return u


def step1d(prob: Problem, u, dt: float, order=None, psi1=None, alpha=None, nthreads: int = 0):
    """One 1D ACAT step.  With order/psi1/alpha given: frozen replay."""
    u = _state(prob, u)
    nI = prob.n_interfaces[0]
    out = np.empty_like(u)
    flux = np.empty((prob.nvar, nI))
    replay = order is not None
    if replay:
        order = np.ascontiguousarray(order, dtype=np.int8)
        psi1 = np.ascontiguousarray(psi1, dtype=np.float64)
        alpha = np.ascontiguousarray(alpha, dtype=np.float64)
    else:
        order = np.zeros(nI, np.int8); psi1 = np.zeros(nI); alpha = np.zeros(nI)
    pc = prob.c()
    _chk(lib().oracle_step1d(ctypes.byref(pc), _p(u), _p(out), dt, 1 if replay else 0, _p(order, ctypes.c_int8),
                             _p(psi1), _p(alpha), _p(flux), nthreads))
    return dict(u=out, order=order, psi1=psi1, alpha=alpha, flux=flux)


def step2d(prob: Problem, u, dt: float, maps=None, nthreads: int = 0):
    """One 2D ACAT step.  maps = (ordx, ordy, psix, psiy, alx, aly) replays."""
    u = _state(prob, u)
    nIx, nIy = prob.n_interfaces
    out = np.empty_like(u)
    F = np.empty((prob.nvar, prob.ny, nIx)); G = np.empty((prob.nvar, nIy, prob.nx))
    replay = maps is not None
    if replay:
        ox, oy, px, py, ax, ay = [np.ascontiguousarray(m, dtype=t) for m, t in
                                  zip(maps, (np.int8, np.int8) + (np.float64,) * 4)]
    else:
        ox = np.zeros((prob.ny, nIx), np.int8); oy = np.zeros((nIy, prob.nx), np.int8)
        px = np.zeros((prob.ny, nIx)); py = np.zeros((nIy, prob.nx))
        ax = np.zeros((prob.ny, nIx)); ay = np.zeros((nIy, prob.nx))
    pc = prob.c()
    i8 = ctypes.c_int8
    _chk(lib().oracle_step2d(ctypes.byref(pc), _p(u), _p(out), dt, 1 if replay else 0, _p(ox, i8), _p(oy, i8),
                             _p(px), _p(py), _p(ax), _p(ay), _p(F), _p(G), nthreads))
    return dict(u=out, ordx=ox, ordy=oy, psix=px, psiy=py, alx=ax, aly=ay, F=F, G=G)


def step(prob: Problem, u, dt: float, nthreads: int = 0):
    return step1d(prob, u, dt, nthreads=nthreads) if prob.dim == 1 else step2d(prob, u, dt, nthreads=nthreads)


def jvp(prob: Problem, u, du, dt: float, maps, nthreads: int = 0):
    """Tangent of the frozen replay step (dual numbers): returns (u_out, du_out)."""
    u = _state(prob, u)
    du = _state(prob, du)
    out = np.empty_like(u); dout = np.empty_like(u)
    pc = prob.c()
    if prob.dim == 1:
        o, p1, a = maps
        o = np.ascontiguousarray(o, np.int8); p1 = np.ascontiguousarray(p1, np.float64)
        a = np.ascontiguousarray(a, np.float64)
        _chk(lib().oracle_step1d_jvp(ctypes.byref(pc), _p(u), _p(du), _p(out), _p(dout), dt,
                                     _p(o, ctypes.c_int8), _p(p1), _p(a), nthreads))
    else:
        ox, oy, px, py, ax, ay = [np.ascontiguousarray(m, dtype=t) for m, t in
                                  zip(maps, (np.int8, np.int8) + (np.float64,) * 4)]
        i8 = ctypes.c_int8
        _chk(lib().oracle_step2d_jvp(ctypes.byref(pc), _p(u), _p(du), _p(out), _p(dout), dt, _p(ox, i8),
                                     _p(oy, i8), _p(px), _p(py), _p(ax), _p(ay), nthreads))
    return out, dout


def jvp2(prob: Problem, u, du2, dt: float, maps=None, nthreads: int = 0):
    """2D tangent of the frozen replay step along two directions at once
    (du2 of shape (2, nvar, ny, nx)): returns (u_out, du_out of the same
    shape).  maps=None: the step's own decisions (taken from the values)."""
    u = _state(prob, u)
    if prob.dim != 2:
        raise ValueError("jvp2 is 2D only")
    du2 = np.ascontiguousarray(du2, dtype=np.float64)
    if du2.shape != (2,) + u.shape:
        raise ValueError(f"directions {du2.shape} != {(2,) + u.shape}")
    out = np.empty_like(u); dout = np.empty_like(du2)
    pc = prob.c()
    decide = maps is None
    if decide:
        nIx, nIy = prob.n_interfaces
        maps = (np.zeros((prob.ny, nIx), np.int8), np.zeros((nIy, prob.nx), np.int8), np.zeros((prob.ny, nIx)),
                np.zeros((nIy, prob.nx)), np.zeros((prob.ny, nIx)), np.zeros((nIy, prob.nx)))
    ox, oy, px, py, ax, ay = [np.ascontiguousarray(m, dtype=t) for m, t in
                              zip(maps, (np.int8, np.int8) + (np.float64,) * 4)]
    i8 = ctypes.c_int8
    _chk(lib().oracle_step2d_jvp2(ctypes.byref(pc), _p(u), _p(du2), _p(out), _p(dout), dt, _p(ox, i8), _p(oy, i8),
                                  _p(px), _p(py), _p(ax), _p(ay), nthreads, 1 if decide else 0))
    return out, dout


def vjp_dense(prob: Problem, u, ubar, dt: float, maps, nthreads: int = 0):
    """Adjoint of the frozen replay step by its definition, ubar_in = J^T ubar
    with J the Jacobian of the replay step assembled column by column from
    jvp: entry j of ubar_in is <ubar, J e_j>.  Small problems only."""
    u = _state(prob, u)
    ubar = _state(prob, ubar)
    e = np.zeros(u.size)
    out = np.empty(u.size)
    for j in range(u.size):
        e[j] = 1.0
        _, col = jvp(prob, u, e.reshape(u.shape), dt, maps, nthreads)
        out[j] = float(np.dot(col.ravel(), ubar.ravel()))
        e[j] = 0.0
    return out.reshape(u.shape)


def maps_of(prob: Problem, r: dict):
    """The frozen decisions of a step result, in the form jvp / step2d take."""
    if prob.dim == 1:
        return (r["order"], r["psi1"], r["alpha"])
    return tuple(r[k] for k in ("ordx", "ordy", "psix", "psiy", "alx", "aly"))


def update_cells(prob: Problem, u, dt: float, cells, nthreads: int = 0):
    """Updated state at the given cells ([n,2] of (i1, i2)); returns (vals [n,nvar], orders [n,4])."""
    u = _state(prob, u)
    cells = np.ascontiguousarray(cells, dtype=np.int64).reshape(-1, 2)
    n = cells.shape[0]
    out = np.empty((n, prob.nvar)); ords = np.zeros((n, 4), np.int8)
    pc = prob.c()
    _chk(lib().oracle_update_cells(ctypes.byref(pc), _p(u), dt, n, _p(cells, ctypes.c_int64), _p(out),
                                   _p(ords, ctypes.c_int8), nthreads))
    return out, ords


def max_speed(prob: Problem, u) -> np.ndarray:
    u = _state(prob, u)
    s = np.zeros(2)
    pc = prob.c()
    _chk(lib().oracle_max_speed(ctypes.byref(pc), _p(u), _p(s)))
    return s[:prob.dim]


def dt_cfl(prob: Problem, u, cfl: float) -> float:
    """1D: CFL dx / s_max.  2D (Sec. 5.5): CFL/2 min(dx/s_x, dy/s_y)."""
    s = max_speed(prob, u)
    if prob.dim == 1:
        return cfl * prob.dx / s[0]
    return 0.5 * cfl * min(prob.dx / s[0], prob.dy / s[1])


def run(prob: Problem, u0, cfl: float, t_final: float | None = None, nsteps: int | None = None,
        nthreads: int = 0, record: bool = False):
    """Advance with the CFL rule until t_final (last step clipped) or for nsteps."""
    u = np.array(u0, dtype=np.float64)
    t, n, hist = 0.0, 0, []
    while True:
        if nsteps is not None and n >= nsteps:
            break
        if t_final is not None and t >= t_final:
            break
        dt = dt_cfl(prob, u, cfl)
        if t_final is not None and t + dt > t_final:
            dt = t_final - t
        r = step(prob, u, dt, nthreads=nthreads)
        if record:
            hist.append(dict(u=u, dt=dt, **{k: v for k, v in r.items() if k not in ("u",)}))
        u = r["u"]
        t += dt
        n += 1
    return (u, t, n, hist) if record else (u, t, n)
