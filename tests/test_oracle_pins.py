"""Pins of the 1D oracle against what the paper and the mathematics fix.

Each test names the property it checks; none re-types the oracle's
recursion.  Small sizes only: the whole file runs in seconds.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle
from oracle import rational as R

ADV, BURG, EUL = oracle.FLUX_ADVECTION, oracle.FLUX_BURGERS, oracle.FLUX_EULER


def prob1d(nx, flux, P, bc=0, dx=1.0, ax=1.0, nvar=None, eps=1e-12):
    nv = nvar or (3 if flux == EUL else 1)
    return oracle.Problem(dim=1, nvar=nv, nx=nx, flux=flux, P=P, bc=bc, dx=dx, ax=ax, eps=eps)


def forced(nI, p):
    return dict(order=np.full(nI, p, np.int8), psi1=np.ones(nI), alpha=np.ones(nI))


def euler_f(u, g=1.4):
    rho, m, E = u
    v = m / rho
    p = (g - 1) * (E - 0.5 * m * v)
    return np.array([m, m * v + p, v * (E + p)])


# --------------------------------------------------------------------- CAT2
@pytest.mark.parametrize("flux", [BURG, EUL])
def test_cat2_closed_form(flux):
    """p = 1 recursion = the CAT2 closed form of Sec. 2.2 (four flux values)."""
    rng = np.random.default_rng(1)
    N = 16
    if flux == BURG:
        u = rng.uniform(-1, 1, (1, N)); f = lambda w: 0.5 * w * w
    else:
        rho = rng.uniform(0.5, 1.5, N); v = rng.uniform(-0.5, 0.5, N); p = rng.uniform(0.5, 1.5, N)
        u = np.stack([rho, rho * v, p / 0.4 + 0.5 * rho * v * v]); f = euler_f
    dx, dt = 0.1, 0.03
    lam = dt / dx
    r = oracle.step1d(prob1d(N, flux, 1, dx=dx), u, dt, **forced(N, 1))
    for i in range(N):
        u0, u1 = u[:, i], u[:, (i + 1) % N]
        f0, f1 = f(u0), f(u1)
        pred = lambda w: f(w - lam * (f1 - f0))
        F = 0.25 * (pred(u1) + pred(u0) + f1 + f0)
        assert np.allclose(r["flux"][:, i], F, rtol=1e-14, atol=1e-15)


# ------------------------------------------------------------ Lax-Wendroff
@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("c", [0.37, 0.9, -0.6])
def test_linear_reduces_to_lax_wendroff(p, c):
    """Linear flux, uniform order p: u_i^{n+1} = sum_m l_m(-c) u_{i+m}, the
    order-2p Lax-Wendroff scheme (Sec. 2.2 claim)."""
    rng = np.random.default_rng(p)
    N = 40
    u = rng.standard_normal((1, N))
    dx = 1.0 / N
    r = oracle.step1d(prob1d(N, ADV, p, dx=dx, ax=c), u, dx, **forced(N, p))
    cf = Fr(c).limit_denominator(1000)
    w = [float(x) for x in R.weights(tuple(range(-p, p + 1)), -cf, 0)]
    lw = sum(w[m + p] * np.roll(u[0], -m) for m in range(-p, p + 1))
    assert np.abs(r["u"][0] - lw).max() < 1e-14 * 10 ** p


@pytest.mark.parametrize("p", [1, 2, 3])
def test_linear_lax_wendroff_exact_rational(p):
    """The same reduction in exact arithmetic (rational oracle)."""
    N = 10
    u = [Fr(int(v), 7) for v in np.random.default_rng(5).integers(-20, 20, N)]
    c = Fr(3, 8)
    new, _ = R.step("advection", u, p, c / 16, Fr(1, 16), order=p)
    w = R.weights(tuple(range(-p, p + 1)), -c, 0)
    lw = [sum(w[m + p] * u[(i + m) % N] for m in range(-p, p + 1)) for i in range(N)]
    assert new == lw


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_unit_courant_number_is_exact_shift(p):
    rng = np.random.default_rng(7)
    N = 24
    u = rng.standard_normal((1, N))
    r = oracle.step1d(prob1d(N, ADV, p, dx=0.5), u, 0.5, **forced(N, p))
    assert np.abs(r["u"][0] - np.roll(u[0], 1)).max() < 1e-13


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_linear_l2_stability(p):
    """|amplification factor| <= 1 for every Fourier mode, 0 < c <= 1 (Sec. 2.2)."""
    N = 64
    j = np.arange(N)
    for c in (0.25, 0.5, 0.8, 1.0):
        for k in range(1, N // 2 + 1):
            th = 2 * np.pi * k / N
            outs = []
            for base in (np.cos(th * j), np.sin(th * j)):
                outs.append(oracle.step1d(prob1d(N, ADV, p, dx=1.0, ax=c), base[None], 1.0, **forced(N, p))["u"][0])
            z = outs[0] + 1j * outs[1]
            g = z / np.exp(1j * th * j)
            assert np.allclose(g, g[0], atol=1e-12)
            assert abs(g[0]) <= 1 + 1e-12


# ------------------------------------------------------------- convergence
def _adv_error(N, P, T=0.5):
    x = -1 + (np.arange(N) + 0.5) * 2 / N
    u0 = 0.5 * np.sin(np.pi * x + 0.3)
    u, t, n = oracle.run(prob1d(N, ADV, P, dx=2 / N), u0[None], 0.8, t_final=T)
    return np.abs(u[0] - 0.5 * np.sin(np.pi * (x - T) + 0.3)).max()


@pytest.mark.parametrize("P,Ns", [(2, (160, 320, 640)), (3, (40, 80, 160)), (4, (40, 80)), (5, (24, 32)),
                                  (6, (24, 32))])
def test_convergence_order_advection(P, Ns):
    e = np.array([_adv_error(N, P) for N in Ns])
    rates = np.log2(e[:-1] / e[1:])
    assert np.all(rates > 2 * P - 0.35), rates


def _burgers_exact(x, t, u0, du0):
    # characteristics: u = u0(xi), x = xi + u0(xi) t; Newton on xi
    xi = x.copy()
    for _ in range(60):
        xi -= (xi + u0(xi) * t - x) / (1 + du0(xi) * t)
    return u0(xi)


@pytest.mark.parametrize("P", [2, 3])
def test_convergence_order_burgers_before_shock(P):
    u0 = lambda s: 0.5 + 0.25 * np.sin(np.pi * s + 0.3)
    du0 = lambda s: 0.25 * np.pi * np.cos(np.pi * s + 0.3)
    T = 0.3   # shock time 1/(0.25 pi) ~ 1.27
    # coarser P = 2 grids still fall back near the moving extrema
    Ns = (640, 1280) if P == 2 else (160, 320)
    errs = []
    for N in Ns:
        x = -1 + (np.arange(N) + 0.5) * 2 / N
        u, t, n = oracle.run(prob1d(N, BURG, P, dx=2 / N), u0(x)[None], 0.8, t_final=T)
        errs.append(np.abs(u[0] - _burgers_exact(x, T, u0, du0)).max())
    rate = np.log2(errs[0] / errs[1])
    assert rate > 2 * P - 0.4, (errs, rate)


@pytest.mark.parametrize("P", [2, 3])
def test_convergence_order_euler_entropy_wave(P):
    """rho = 1 + 0.2 sin(pi x), v = 1, p = 1 translates exactly."""
    Ns = (160, 320) if P == 2 else (80, 160)
    T = 0.25
    errs = []
    for N in Ns:
        x = -1 + (np.arange(N) + 0.5) * 2 / N
        mk = lambda s: np.stack([1 + 0.2 * np.sin(np.pi * s + 0.3), 1 + 0.2 * np.sin(np.pi * s + 0.3),
                                 1 / 0.4 + 0.5 * (1 + 0.2 * np.sin(np.pi * s + 0.3))])
        u, t, n = oracle.run(prob1d(N, EUL, P, dx=2 / N), mk(x), 0.6, t_final=T)
        errs.append(np.abs(u - mk(x - T)).max())
    rate = np.log2(errs[0] / errs[1])
    assert rate > 2 * P - 0.4, (errs, rate)


# ------------------------------------------------- conservation, free stream
def test_periodic_conservation_burgers_with_shock():
    import workloads
    w = workloads.burgers_1d()
    pb = prob1d(200, BURG, 2, dx=w["dx"])
    u, t, n = oracle.run(pb, w["u"], w["cfl"], t_final=w["t_final"])
    m0, m1 = w["u"].sum(), u.sum()
    assert abs(m1 - m0) <= 200 * n * 2.0 ** -52 * np.abs(w["u"]).max() * 4
    assert np.isfinite(u).all()


@pytest.mark.parametrize("bc", [0, 1])
def test_free_stream_bitwise(bc):
    N = 32
    u = np.tile(np.array([[1.3], [0.4], [2.9]]), (1, N))
    for P in (1, 2, 3, 4, 5, 6):
        r = oracle.step1d(prob1d(N, EUL, P, bc=bc, dx=0.1), u, 0.01)
        assert np.array_equal(r["u"], u)
        assert (r["order"] == P if P >= 2 else r["order"] == 1).all()


def test_mirror_symmetry_euler():
    rng = np.random.default_rng(3)
    N = 48
    rho = rng.uniform(0.3, 1.5, N); v = rng.uniform(-0.5, 0.5, N); p = rng.uniform(0.3, 1.5, N)
    rho[N // 2:] *= 3
    u = np.stack([rho, rho * v, p / 0.4 + 0.5 * rho * v * v])
    um = u[:, ::-1].copy(); um[1] *= -1
    pb = prob1d(N, EUL, 4, dx=0.02)
    a = oracle.step1d(pb, u, 0.004)["u"]
    b = oracle.step1d(pb, um, 0.004)["u"]
    b = b[:, ::-1]; b[1] *= -1
    assert np.allclose(a, b, rtol=1e-13, atol=1e-13)


# ------------------------------------------------------------- indicators
def test_indicator_step_closed_forms():
    eps = 1e-12
    # (0,0,1,1): tau = (3! * -2)^2 = 144, I = eps/2
    assert oracle.indicator([0, 0, 1, 1], 2, eps) == (eps / 2) / (eps / 2 + 144)
    # (0,1,1,1): tau = 36, I = (1+eps) eps / (1 + 2 eps)
    I = (1 + eps) * eps / (1 + 2 * eps)
    assert abs(oracle.indicator([0, 1, 1, 1], 2, eps) - I / (I + 36)) < 1e-28


@pytest.mark.parametrize("p", [2, 3, 4, 5, 6])
def test_indicator_is_one_on_low_degree_polynomials(p):
    j = np.arange(-p + 1, p + 1, dtype=float)
    for deg in range(2 * p - 1):
        v = (j + 0.5) ** deg * 3 - 2 * j
        assert oracle.indicator(v, p) == 1.0


@pytest.mark.parametrize("p", [2, 3, 4])
def test_indicator_homothety(p):
    """psi is invariant under g = alpha f with eps -> alpha^2 eps (Sec. 3.2)."""
    rng = np.random.default_rng(p)
    for _ in range(20):
        v = rng.standard_normal(2 * p)
        a = 10.0 ** rng.uniform(-3, 3)
        assert abs(oracle.indicator(a * v, p, 1e-12 * a * a) - oracle.indicator(v, p, 1e-12)) < 1e-12


def test_indicator_detects_jump_and_smoothness():
    """psi^p near 1 on smooth data and near 0 across a jump (Sec. 3.2 estimates)."""
    for p in (2, 3, 4):
        for h in (0.05, 0.01):
            j = np.arange(-p + 1, p + 1)
            assert oracle.indicator(np.sin(1 + h * j), p) > 0.99
            jump = np.where(j > 0, 1.0, 0.0) + h * j
            assert oracle.indicator(jump, p) < 0.01


def test_superbee_limiter():
    # r = (du_upw)/(du_loc); values at -1, 0, 1, 2
    assert oracle.limiter([0, 1, 2, 3]) == 1.0              # r = 1 both sides
    assert oracle.limiter([0, 0, 1, 1]) == 0.0              # flat neighbours: r = 0
    assert oracle.limiter([0, 1, 1, 1]) == 0.0              # du_loc = 0 beside a variation: 0
    assert oracle.limiter([1, 1, 1, 1]) == 1.0              # du_loc = 0, locally constant: 1
    assert oracle.limiter([1, 0.4, 0.4, 1]) == 0.0          # du_loc = 0 at an extremum: 0
    assert oracle.limiter([0, 2, 3, 5]) == 2.0              # r = 2 both sides: phi = 2 (not clipped to 1)
    assert oracle.limiter([0, 0.25, 1.25, 1.5]) == 0.5       # r = 1/4: phi = 2r
    assert oracle.limiter([0, 3, 4, 9]) == 2.0               # r- = 3, r+ = 5: phi = 2
    assert oracle.limiter([2, 1, 2, 3]) == 0.0               # r- = -1 < 0
