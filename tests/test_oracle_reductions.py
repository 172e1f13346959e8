"""Oracle pins: exact-rational brute force, scaled vs literal recursion, the
ACAT reduction cases (Sec. 3.3), JVP vs finite differences."""
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle
from oracle import rational as R

ADV, BURG, EUL = oracle.FLUX_ADVECTION, oracle.FLUX_BURGERS, oracle.FLUX_EULER


def prob1d(nx, flux, P, bc=0, dx=1.0, ax=1.0, eps=1e-12):
    return oracle.Problem(dim=1, nvar=3 if flux == EUL else 1, nx=nx, flux=flux, P=P, bc=bc, dx=dx, ax=ax,
                          eps=eps)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_scaled_recursion_equals_literal_form(p):
    """The scaled variables U^l = dt^l u~^(l) leave the flux unchanged (exact)."""
    us = [Fr(v, 9) for v in (3, -4, 7, 1, 0, 5)][: 2 * p]
    dt, dx = Fr(1, 40), Fr(1, 8)
    assert R.cat_flux("burgers", us, p, dt / dx) == R.cat_flux_literal("burgers", us, p, dt, dx)


def _dyadic(rng, n, scale=64):
    return [Fr(int(v), scale) for v in rng.integers(-2 * scale, 2 * scale, n)]


@pytest.mark.parametrize("kind,flux", [("burgers", BURG), ("advection", ADV)])
@pytest.mark.parametrize("P", [1, 2, 3])
@pytest.mark.parametrize("bc", ["periodic", "transmissive"])
def test_exact_rational_brute_force(kind, flux, P, bc):
    """fp64 oracle step == exact rational step up to rounding, same orders."""
    rng = np.random.default_rng(100 * P + len(kind) + len(bc))
    N = 12
    eps = Fr(1, 2 ** 40)
    for trial in range(3):
        u = _dyadic(rng, N)
        if trial == 1:   # a smooth piece and a jump
            u = [Fr(int(8 * np.sin(i / 2)), 16) + (Fr(3) if i > 6 else 0) for i in range(N)]
        dt, dx = Fr(1, 64), Fr(1, 8)
        new, ords = R.step(kind, u, P, dt, dx, bc=bc, eps=eps)
        pb = prob1d(N, flux, P, bc=0 if bc == "periodic" else 1, dx=float(dx), eps=float(eps))
        r = oracle.step1d(pb, np.array([[float(v) for v in u]]), float(dt))
        assert list(r["order"]) == ords
        exact = np.array([float(v) for v in new])
        assert np.allclose(r["u"][0], exact, rtol=1e-14, atol=1e-14)


def test_P1_is_fl_cat2_everywhere():
    rng = np.random.default_rng(4)
    N = 30
    u = rng.uniform(-1, 1, (1, N))
    dx, dt = 0.1, 0.04
    r = oracle.step1d(prob1d(N, BURG, 1, dx=dx), u, dt)
    assert (r["order"] == 1).all()
    lam = dt / dx
    for i in range(N):
        v = [u[0, (i + j) % N] for j in (-1, 0, 1, 2)]
        dl = v[2] - v[1]
        sb = lambda q: max(0.0, min(2 * q, 1.0), min(q, 2.0))
        psi = 1.0 if dl == 0 else min(sb((v[3] - v[2]) / dl), sb((v[1] - v[0]) / dl))
        f = lambda w: 0.5 * w * w
        f0, f1 = f(v[1]), f(v[2])
        cat2 = 0.25 * (f(v[2] - lam * (f1 - f0)) + f(v[1] - lam * (f1 - f0)) + f1 + f0)
        rus = 0.5 * (f0 + f1) - 0.5 * max(abs(v[1]), abs(v[2])) * (v[2] - v[1])
        assert abs(r["flux"][0, i] - (psi * cat2 + (1 - psi) * rus)) < 1e-15
        assert abs(r["psi1"][i] - psi) < 1e-15


@pytest.mark.parametrize("P", [2, 3, 4])
def test_smooth_polynomial_selects_P(P):
    # degree <= 2P-2 polynomial data: tau_p = 0 for every p <= P
    N = 40
    x = np.arange(N, dtype=float) - N / 2
    u = (0.01 * x ** 2 + 0.2 * x + 1.0)[None]
    pb = prob1d(N, ADV, P, bc=1, dx=1.0)
    r = oracle.step1d(pb, u, 0.5)
    inner = r["order"][P + 1:-P - 1]
    assert (inner == P).all()


def test_zigzag_reduces_to_rusanov():
    """psi^1 = 0 and A empty: the flux is the robust first-order one."""
    N = 20
    u = np.where(np.arange(N) % 2 == 0, 1.0, -0.5)[None] + 0.0
    dx, dt = 0.1, 0.02
    r = oracle.step1d(prob1d(N, BURG, 3, dx=dx), u, dt)
    assert (r["order"] == 1).all() and (r["psi1"] == 0).all()
    for i in range(N):
        a, b = u[0, i], u[0, (i + 1) % N]
        rus = 0.25 * (a * a + b * b) - 0.5 * max(abs(a), abs(b)) * (b - a)
        assert abs(r["flux"][0, i] - rus) < 1e-15


@pytest.mark.parametrize("P", [2, 4])
def test_jvp_matches_central_difference_1d(P):
    import workloads
    w = workloads.euler_1d(n=64, P=P)
    pb = prob1d(64, EUL, P, bc=1, dx=w["dx"])
    u = w["u"]
    dt = 0.5 * oracle.dt_cfl(pb, u, 0.5)
    r = oracle.step1d(pb, u, dt)
    maps = (r["order"], r["psi1"], r["alpha"])
    d = np.random.default_rng(0).standard_normal(u.shape)
    _, jv = oracle.jvp(pb, u, d, dt, maps)
    h = 1e-6
    up = oracle.step1d(pb, u + h * d, dt, order=maps[0], psi1=maps[1], alpha=maps[2])["u"]
    um = oracle.step1d(pb, u - h * d, dt, order=maps[0], psi1=maps[1], alpha=maps[2])["u"]
    fd = (up - um) / (2 * h)
    assert np.abs(fd - jv).max() < 1e-7 * np.abs(jv).max()


@pytest.mark.parametrize("P", [2, 3, 4])
def test_vjp_of_periodic_advection_is_reversed_advection(P):
    """Linear advection, periodic, every interface frozen at order P: the
    step is u -> A u with A circulant and centred, so A^T is the same step
    with the speed reversed (mirror symmetry of the order-2P Lax-Wendroff
    stencil).  Pins the transpose the dense oracle adjoint assembles."""
    n = 24
    rng = np.random.default_rng(P)
    pb = prob1d(n, ADV, P, dx=0.1, ax=1.3)
    pr = prob1d(n, ADV, P, dx=0.1, ax=-1.3)
    u = rng.standard_normal((1, n))
    ub = rng.standard_normal((1, n))
    dt = 0.6 * 0.1 / 1.3
    maps = (np.full(n, P, np.int8), np.full(n, -1.0), np.full(n, -1.0))
    got = oracle.vjp_dense(pb, u, ub, dt, maps)
    want = oracle.step1d(pr, ub, dt, order=maps[0], psi1=maps[1], alpha=maps[2])["u"]
    assert np.abs(got - want).max() < 1e-13


def test_vjp_dense_inner_product_euler_2d():
    """<J^T w, v> = <w, J v> for the dense oracle adjoint of a frozen 2D
    Euler step with mixed orders."""
    import workloads
    rng = np.random.default_rng(5)
    w = workloads.euler_2d(n=12, P=2)
    pb = oracle.Problem(dim=2, nvar=4, nx=12, ny=12, flux=EUL, P=2, bc=0, dx=w["dx"], dy=w["dy"])
    u = w["u"]
    dt = oracle.dt_cfl(pb, u, 0.4)
    maps = oracle.maps_of(pb, oracle.step2d(pb, u, dt))
    wb = rng.standard_normal(u.shape)
    v = rng.standard_normal(u.shape)
    lhs = np.vdot(oracle.vjp_dense(pb, u, wb, dt, maps), v)
    rhs = np.vdot(wb, oracle.jvp(pb, u, v, dt, maps)[1])
    assert abs(lhs - rhs) < 1e-11 * abs(rhs)
