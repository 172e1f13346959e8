"""Pins of the oracle's wave speeds, time-step rule and Rusanov flux against
hand-computed values.

The states are chosen so that every quantity is a short dyadic number: with
gamma = 1.5, rho = 1, p = 1.5 and rho = 4, p = 6 both give the sound speed
c = sqrt(gamma p / rho) = 1.5 exactly.  A slip in the wave speed (c without
gamma, |(v, w)| + c instead of |v| + c per direction, the maximum over the
wrong cells), in the 2D time-step rule (Sec. 5.5: CFL/2 min(dx/s_x, dy/s_y))
or in the Rusanov speed alpha = max of the two cells' spectral radii changes
these numbers.  Every expected value below was worked out by hand from the
textbook Euler flux f = (m, m v + p, v (E + p)) in 1D and
f = (m, m v + p, n v, v (E + p)), g = (n, m w, n w + p, w (E + p)) in 2D.
Both rounding modes of the oracle must give them exactly.
"""
import numpy as np
import pytest

import oracle

EUL, BURG, ADV = oracle.FLUX_EULER, oracle.FLUX_BURGERS, oracle.FLUX_ADVECTION
GAMMA = 1.5

# 1D states (rho, m, E): L = (rho 1, v 0.5, p 1.5), R = (rho 4, v -1, p 6)
L1 = np.array([1.0, 0.5, 3.125])        # E = 1.5 / 0.5 + 0.5 * 1 * 0.25
R1 = np.array([4.0, -4.0, 14.0])        # E = 6 / 0.5 + 0.5 * 4 * 1
# 2D states (rho, m, n, E): L = (1, v 0.5, w -0.25, p 1.5), R = (4, v -1, w 0.5, p 6),
# Q = (1, v 0, w -2, p 1.5)
L2 = np.array([1.0, 0.5, -0.25, 3.15625])
R2 = np.array([4.0, -4.0, 2.0, 14.5])
Q2 = np.array([1.0, 0.0, -2.0, 5.0])


@pytest.fixture(params=["fixed", "plain"])
def rounding(request):
    return request.param


def p1d(nx, P=1, flux=EUL, nvar=3, rounding="fixed", dx=1.0):
    return oracle.Problem(dim=1, nvar=nvar, nx=nx, flux=flux, P=P, bc=oracle.BC_PERIODIC, gamma=GAMMA, dx=dx,
                          rounding=rounding)


def p2d(n, P=1, rounding="fixed", dx=1.0, dy=1.0):
    return oracle.Problem(dim=2, nvar=4, nx=n, ny=n, flux=EUL, P=P, bc=oracle.BC_PERIODIC, gamma=GAMMA, dx=dx,
                          dy=dy, rounding=rounding)


def test_spectral_radius_1d_hand_values(rounding):
    # |v| + c: L 0.5 + 1.5 = 2, R 1 + 1.5 = 2.5
    assert oracle.max_speed(p1d(4, rounding=rounding), np.tile(L1[:, None], 4))[0] == 2.0
    assert oracle.max_speed(p1d(4, rounding=rounding), np.tile(R1[:, None], 4))[0] == 2.5
    u = np.stack([L1, L1, R1, L1], 1)
    assert oracle.max_speed(p1d(4, rounding=rounding), u)[0] == 2.5
    # Burgers |u|, advection |a|
    assert oracle.max_speed(p1d(4, flux=BURG, nvar=1), np.array([[-3.0, 1.0, 2.0, 0.5]]))[0] == 3.0
    pa = oracle.Problem(dim=1, nvar=1, nx=4, flux=ADV, P=1, ax=-0.75)
    assert oracle.max_speed(pa, np.zeros((1, 4)))[0] == 0.75


def test_spectral_radius_2d_per_direction(rounding):
    # s_x = |v| + c, s_y = |w| + c: L (2, 1.75), R (2.5, 2), Q (1.5, 3.5)
    pb = p2d(4, rounding=rounding)
    for st, sx, sy in ((L2, 2.0, 1.75), (R2, 2.5, 2.0), (Q2, 1.5, 3.5)):
        s = oracle.max_speed(pb, np.tile(st[:, None, None], (1, 4, 4)))
        assert (s[0], s[1]) == (sx, sy)
    # mixed grid: the maxima come from different cells (R in x, Q in y);
    # the speed magnitude |(v, w)| + c would give 2.618... in x
    u = np.tile(L2[:, None, None], (1, 4, 4))
    u[:, 1, 2] = R2
    u[:, 3, 0] = Q2
    s = oracle.max_speed(pb, u)
    assert (s[0], s[1]) == (2.5, 3.5)


def test_time_step_rules():
    u1 = np.stack([L1, R1, L1, L1], 1)
    # 1D: CFL dx / s = 0.625 * 1 / 2.5 = 0.25
    assert oracle.dt_cfl(p1d(4), u1, 0.625) == 0.25
    # 2D (Sec. 5.5): CFL/2 min(dx/s_x, dy/s_y); s = (2.5, 3.5), dx = 1, dy = 0.5:
    # 0.2 min(0.4, 1/7) = 1/35
    u = np.tile(L2[:, None, None], (1, 4, 4))
    u[:, 1, 2] = R2
    u[:, 3, 0] = Q2
    dt = oracle.dt_cfl(p2d(4, dy=0.5), u, 0.4)
    assert dt == pytest.approx(1.0 / 35.0, rel=2e-16)
    # with dy = 1 the x-direction binds: 0.2 min(0.4, 1/3.5) = 0.2 / 3.5
    assert oracle.dt_cfl(p2d(4), u, 0.4) == pytest.approx(0.2 / 3.5, rel=2e-16)


@pytest.mark.parametrize("P", [1, 2, 3])
def test_euler_1d_fl_cat2_is_rusanov_on_alternating_data(P, rounding):
    """Cells alternate L, R: at every interface the superbee ratios are -1, so
    psi^1 = 0 and the FL-CAT2 flux is the Rusanov flux with alpha = 2.5
    (Sec. 3.1 blend); no wider stencil is smooth, so every order is 1."""
    N = 8
    u = np.stack([L1 if i % 2 == 0 else R1 for i in range(N)], 1)
    r = oracle.step1d(p1d(N, P=P, rounding=rounding), u, 0.25)
    assert np.all(r["order"] == 1)
    assert np.all(r["psi1"] == 0.0)
    assert np.all(r["alpha"] == 2.5)
    # F(L|R) = (f_L + f_R)/2 - 1.25 (u_R - u_L); F(R|L) = (f_R + f_L)/2 - 1.25 (u_L - u_R)
    FLR = np.array([-5.5, 11.5, -22.4375])
    FRL = np.array([2.0, 0.25, 4.75])
    for k in range(N):
        np.testing.assert_array_equal(r["flux"][:, k], FLR if k % 2 == 0 else FRL)
    # update with lambda = 0.25
    newL = np.array([2.875, -2.3125, 9.921875])
    newR = np.array([2.125, -1.1875, 7.203125])
    for i in range(N):
        np.testing.assert_array_equal(r["u"][:, i], newL if i % 2 == 0 else newR)


@pytest.mark.parametrize("P", [1, 2, 3])
def test_euler_2d_fl_cat2_is_rusanov_on_checkerboard(P, rounding):
    """Checkerboard of L and R: psi^1 = 0 in both directions, F and G are the
    Rusanov fluxes with alpha_x = 2.5 (|v| + c) and alpha_y = 2 (|w| + c)."""
    N = 8
    u = np.empty((4, N, N))
    for j in range(N):
        for i in range(N):
            u[:, j, i] = L2 if (i + j) % 2 == 0 else R2
    r = oracle.step2d(p2d(N, P=P, rounding=rounding), u, 0.125)
    for k in ("ordx", "ordy"):
        assert np.all(r[k] == 1)
    assert np.all(r["psix"] == 0.0) and np.all(r["psiy"] == 0.0)
    assert np.all(r["alx"] == 2.5) and np.all(r["aly"] == 2.0)
    FLR = np.array([-5.5, 11.5, -3.875, -23.265625])
    FRL = np.array([2.0, 0.25, 1.75, 5.09375])
    GLR = np.array([-2.125, 3.4375, 2.03125, -6.80078125])
    GRL = np.array([3.875, -5.5625, 6.53125, 15.88671875])
    for j in range(N):
        for i in range(N):
            left_is_L = (i + j) % 2 == 0
            np.testing.assert_array_equal(r["F"][:, j, i], FLR if left_is_L else FRL)
            np.testing.assert_array_equal(r["G"][:, j, i], GLR if left_is_L else GRL)
    newL = np.array([2.6875, -2.03125, 1.015625, 9.537109375])
    newR = np.array([2.3125, -1.46875, 0.734375, 8.119140625])
    for j in range(N):
        for i in range(N):
            np.testing.assert_array_equal(r["u"][:, j, i], newL if (i + j) % 2 == 0 else newR)
