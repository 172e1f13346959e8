"""Pins of the oracle's variants (Problem.flags): Lax-Friedrichs and HLL as
the first-order flux of the FL-CAT2 blend, the modified p = 2 indicator
(Sec. 3.2) and the Roe-speed upwind limiter ratio for scalar laws
(Sec. 3.1).  Each is checked against a closed form or a property the
definition implies, not against a retyped formula."""
import numpy as np
import pytest

import oracle
import workloads

ADV, BURG, EUL = oracle.FLUX_ADVECTION, oracle.FLUX_BURGERS, oracle.FLUX_EULER
LF, HLL, PSI2M, ROE = oracle.FLAG_FLO_LF, oracle.FLAG_FLO_HLL, oracle.FLAG_PSI2_MODIFIED, oracle.FLAG_PSI1_ROE


def p1(nx, flux, flags, bc=0, dx=0.1, ax=1.0, P=1):
    nv = 3 if flux == EUL else 1
    return oracle.Problem(dim=1, nvar=nv, nx=nx, flux=flux, P=P, bc=bc, dx=dx, ax=ax, flags=flags)


def lowonly(n):
    """Frozen decisions: order 1 with psi^1 = 0 everywhere (pure F^lo)."""
    return dict(order=np.full(n, 1, np.int8), psi1=np.zeros(n), alpha=np.full(n, 7.0))


def euler_f(u, g=1.4):
    rho, m, E = u
    v = m / rho
    p = (g - 1) * (E - 0.5 * m * v)
    return np.array([m, m * v + p, v * (E + p)])


def euler_state(rng, n):
    rho = rng.uniform(0.5, 1.5, n); v = rng.uniform(-0.5, 0.5, n); p = rng.uniform(0.5, 1.5, n)
    return np.stack([rho, rho * v, p / 0.4 + 0.5 * rho * v * v])


@pytest.mark.parametrize("flux", [BURG, EUL])
def test_lf_is_the_lax_friedrichs_scheme_1d(flux):
    """psi^1 = 0: u_i^{n+1} = (u_{i-1} + u_{i+1})/2 - lam/2 (f_{i+1} - f_{i-1})."""
    rng = np.random.default_rng(1)
    n, dx, dt = 24, 0.1, 0.03
    u = rng.uniform(-1, 1, (1, n)) if flux == BURG else euler_state(rng, n)
    f = (lambda w: 0.5 * w * w) if flux == BURG else euler_f
    out = oracle.step1d(p1(n, flux, LF, dx=dx), u, dt, **lowonly(n))["u"]
    fu = f(u)
    want = 0.5 * (np.roll(u, 1, 1) + np.roll(u, -1, 1)) - 0.5 * dt / dx * (np.roll(fu, -1, 1) - np.roll(fu, 1, 1))
    assert np.abs(out - want).max() < 1e-13


def test_lf_is_the_lax_friedrichs_scheme_2d():
    """psi^1 = 0 in both directions: the classical 2D scheme, the average of
    the four neighbours minus the centred flux differences."""
    rng = np.random.default_rng(2)
    n, dx, dy, dt = 12, 0.1, 0.12, 0.02
    pb = oracle.Problem(dim=2, nvar=1, nx=n, ny=n, flux=ADV, P=1, bc=0, dx=dx, dy=dy, ax=0.7, ay=-0.4, flags=LF)
    u = rng.standard_normal((1, n, n))
    maps = (np.ones((n, n), np.int8), np.ones((n, n), np.int8), np.zeros((n, n)), np.zeros((n, n)),
            np.zeros((n, n)), np.zeros((n, n)))
    out = oracle.step2d(pb, u, dt, maps=maps)["u"][0]
    v = u[0]
    E, W = np.roll(v, -1, 1), np.roll(v, 1, 1)
    N, S = np.roll(v, -1, 0), np.roll(v, 1, 0)
    want = 0.25 * (E + W + N + S) - 0.5 * dt / dx * 0.7 * (E - W) - 0.5 * dt / dy * (-0.4) * (N - S)
    assert np.abs(out - want).max() < 1e-13


@pytest.mark.parametrize("a", [0.8, -0.6])
def test_hll_is_upwind_for_linear_advection(a):
    rng = np.random.default_rng(3)
    n, dx, dt = 20, 0.1, 0.05
    u = rng.standard_normal((1, n))
    out = oracle.step1d(p1(n, ADV, HLL, dx=dx, ax=a), u, dt, **lowonly(n))["u"][0]
    c = a * dt / dx
    want = u[0] - c * (u[0] - np.roll(u[0], 1)) if a > 0 else u[0] - c * (np.roll(u[0], -1) - u[0])
    assert np.abs(out - want).max() < 1e-14


def test_hll_euler_consistency_and_supersonic_upwinding():
    rng = np.random.default_rng(4)
    n = 16
    # a constant state is preserved (HLL(u, u) = f(u))
    u = np.tile(np.array([[1.3], [0.4], [2.9]]), (1, n))
    assert np.array_equal(oracle.step1d(p1(n, EUL, HLL), u, 0.01, **lowonly(n))["u"], u)
    # supersonic flow to the right (v > c everywhere): the flux is f(u_left)
    rho = rng.uniform(0.8, 1.2, n); v = rng.uniform(3.0, 3.5, n); p = rng.uniform(0.8, 1.2, n)
    u = np.stack([rho, rho * v, p / 0.4 + 0.5 * rho * v * v])
    r = oracle.step1d(p1(n, EUL, HLL), u, 0.01, **lowonly(n))
    assert np.allclose(r["flux"], euler_f(u), rtol=0, atol=1e-14 * np.abs(euler_f(u)).max())


def test_hll_mirror_symmetry():
    rng = np.random.default_rng(5)
    n = 32
    u = euler_state(rng, n)
    um = u[:, ::-1].copy(); um[1] *= -1
    pb = p1(n, EUL, HLL, P=3, dx=0.02)
    a = oracle.step1d(pb, u, 0.004)["u"]
    b = oracle.step1d(pb, um, 0.004)["u"][:, ::-1]
    b[1] *= -1
    assert np.abs(a - b).max() < 1e-13


def test_modified_psi2_detects_an_extremum_at_a_lateral_midpoint():
    """Sec. 3.2: with the maximum of a smooth f at the midpoint of the left
    sub-interval, psi^2 tends to 0 while the modified indicator tends to 1
    under refinement; on a step both stay small."""
    out = []
    for h in (0.05, 0.025, 0.0125):
        x = h * (np.arange(-1, 3) + 0.5)            # the maximum at 0 is the midpoint of (x_{-1}, x_0)
        f = np.cos(x) + 0.5 * x ** 3                # first derivative 0 at 0, third derivative 3
        out.append((oracle.indicator(f, 2), oracle.indicator2_modified(f)))
    assert max(o[0] for o in out) < 1e-3 and out[-1][1] > 0.9
    # 1 - psi~2 = O(dx^2) at a first-order critical point (Sec. 3.2 estimate, k = 1)
    assert 2.5 < (1 - out[0][1]) / (1 - out[1][1]) and 2.5 < (1 - out[1][1]) / (1 - out[2][1])
    step = np.array([0.0, 0.0, 1.0, 1.0])
    assert oracle.indicator2_modified(step) < 1e-6 and oracle.indicator(step, 2) < 1e-6


def test_modified_psi2_keeps_acat4_accurate_on_the_smooth_transport():
    """Sec. 5.1: with the modified indicator ACAT4 follows the exact solution
    of the smooth transport problem (t = 4, 160 points) at the default
    epsilon, where the plain psi^2 falls back at extrema."""
    errs = {}
    for flags in (0, PSI2M):
        w = workloads.paper_scalar_1d("transport_sine", P=2)
        pb = oracle.Problem(dim=1, nvar=1, nx=160, flux=ADV, P=2, bc=0, dx=w["dx"], ax=1.0, flags=flags)
        u, t, _ = oracle.run(pb, w["u"], w["cfl"], t_final=w["t_final"])
        errs[flags] = np.abs(u[0] - 0.5 * np.sin(np.pi * (w["x"] - t))).max()
    assert errs[PSI2M] < 1e-6 < 1e-4 < errs[0], errs


@pytest.mark.parametrize("flux,a", [(ADV, 0.9), (ADV, -0.9), (BURG, None)])
def test_roe_psi1_reads_only_the_upwind_side(flux, a):
    """The Roe form uses r^- when the Roe speed is positive and r^+ otherwise:
    changing the value on the downwind side of the 4-point window does not
    change psi^1, changing the upwind one does."""
    rng = np.random.default_rng(6)
    n, k = 16, 7                      # interface k: between cells 7 and 8 (periodic)
    u = (0.2 + 0.1 * np.arange(n) + 0.03 * rng.uniform(0, 1, n))[None, :]   # increasing, positive
    pb = p1(n, flux, ROE, ax=a if a is not None else 1.0)
    speed_pos = (a > 0) if a is not None else True     # Burgers data positive: Roe speed > 0
    base = oracle.step1d(pb, u, 1e-3)["psi1"][k]
    down, up = (k + 2, k - 1) if speed_pos else (k - 1, k + 2)
    ud = u.copy(); ud[0, down] += 0.37
    uu = u.copy(); uu[0, up] += 0.37
    assert oracle.step1d(pb, ud, 1e-3)["psi1"][k] == base
    assert oracle.step1d(pb, uu, 1e-3)["psi1"][k] != base
    # the default min form reads both sides
    pm = p1(n, flux, 0, ax=a if a is not None else 1.0)
    bm = oracle.step1d(pm, u, 1e-3)["psi1"][k]
    assert oracle.step1d(pm, ud, 1e-3)["psi1"][k] != bm or oracle.step1d(pm, uu, 1e-3)["psi1"][k] != bm


def test_flag_validation():
    lib = oracle.lib()
    u = np.ones((3, 16)); out = np.empty_like(u)
    import ctypes
    for flags, ok in ((LF, True), (HLL, True), (LF | HLL, False), (ROE, False), (64, False), (PSI2M | LF, True)):
        pb = p1(16, EUL, flags)
        o = np.zeros(16, np.int8); ps = np.zeros(16); al = np.zeros(16); F = np.zeros((3, 16))
        rc = lib.oracle_step1d(ctypes.byref(pb.c()), oracle._p(u), oracle._p(out), 0.01, 0, oracle._p(o, ctypes.c_int8),
                               oracle._p(ps), oracle._p(al), oracle._p(F), 1)
        assert (rc == 0) == ok, flags
