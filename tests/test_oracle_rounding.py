"""The oracle's two rounding modes (fixed: explicit fused multiply-adds in a
fixed order; plain: every operation rounded on its own, sums in the order the
paper writes them) compute the same method: one step from the same state
gives identical decisions and states equal to a few ulp, in 1D and 2D, at
every order and both boundaries.  The plain mode also keeps the exact
properties that do not depend on rounding (free stream, conservation, the
Lax-Wendroff reduction to rounding)."""
import dataclasses

import numpy as np
import pytest

import oracle
import workloads
from gpu_helpers import from_workload, rel_err


def plain(po):
    return dataclasses.replace(po, rounding="plain")


@pytest.mark.parametrize("P", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("bc", ["periodic", "transmissive"])
def test_modes_agree_1d(P, bc):
    w = workloads.euler_1d(n=256, P=P)
    po, _ = from_workload(w, bc=bc)
    u = w["u"]
    for _ in range(3):
        dt = oracle.dt_cfl(po, u, w["cfl"])
        a, b = oracle.step(po, u, dt), oracle.step(plain(po), u, dt)
        for k in ("order", "psi1", "alpha"):
            assert np.array_equal(a[k], b[k]), k
        assert rel_err(b["u"], a["u"]) <= 1e-14
        u = a["u"]


@pytest.mark.parametrize("P", [1, 2, 3, 4])
@pytest.mark.parametrize("bc", ["periodic", "transmissive"])
def test_modes_agree_2d(P, bc):
    w = workloads.euler_2d(n=40, P=P)
    po, _ = from_workload(w, bc=bc)
    u = w["u"]
    diff = 0
    for _ in range(2):
        dt = oracle.dt_cfl(po, u, w["cfl"])
        a, b = oracle.step(po, u, dt), oracle.step(plain(po), u, dt)
        for k in ("ordx", "ordy", "psix", "psiy", "alx", "aly"):
            assert np.array_equal(a[k], b[k]), k
        assert rel_err(b["u"], a["u"]) <= 1e-14
        diff += int((a["u"] != b["u"]).sum())
        u = a["u"]
    assert diff > 0      # the modes do round differently


@pytest.mark.parametrize("bc", [0, 1])
def test_plain_mode_free_stream_and_conservation(bc):
    po = oracle.Problem(dim=2, nvar=4, nx=24, ny=20, P=3, bc=bc, dx=0.1, dy=0.12, rounding="plain")
    c = np.tile(np.array([1.3, 0.4, -0.7, 2.9])[:, None, None], (1, 20, 24))
    assert np.array_equal(oracle.step2d(po, c, 1e-3)["u"], c)
    if bc == 0:
        w = workloads.euler_2d(n=48, P=3)
        pp, _ = from_workload(w)
        pp = plain(pp)
        r = oracle.step2d(pp, w["u"], oracle.dt_cfl(pp, w["u"], w["cfl"]))
        s0, s1 = w["u"].reshape(4, -1).sum(1), r["u"].reshape(4, -1).sum(1)
        assert np.all(np.abs(s1 - s0) <= 1e-12 * np.abs(w["u"]).reshape(4, -1).max(1) * w["u"][0].size)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_plain_mode_lax_wendroff(p):
    """Linear flux, uniform order p: the order-2p Lax-Wendroff stencil
    sum_m l_m(-c) u_{i+m} (Lagrange interpolation at the characteristic's
    foot), to rounding."""
    N, c = 40, 0.43
    rng = np.random.default_rng(p)
    u = rng.standard_normal((1, N))
    po = oracle.Problem(dim=1, nvar=1, nx=N, flux=oracle.FLUX_ADVECTION, P=p, ax=1.0, dx=1.0, rounding="plain")
    r = oracle.step1d(po, u, c, order=np.full(N, p, np.int8), psi1=np.ones(N), alpha=np.ones(N))
    m = np.arange(-p, p + 1)
    lw = np.array([np.prod([(-c - b) / (a - b) for b in m if b != a]) for a in m])
    want = sum(lw[k] * np.roll(u[0], -m[k]) for k in range(len(m)))
    assert np.abs(r["u"][0] - want).max() <= 1e-13 * np.abs(u).max()
