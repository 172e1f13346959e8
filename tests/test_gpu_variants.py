"""GPU parity of the variants (acat_problem.flags) against the oracle:
Lax-Friedrichs or HLL as the first-order flux, the modified p = 2
indicator, the Roe-speed limiter ratio for scalar laws, the square-stencil
2D corners.  Lockstep, bit for
bit, on shocked data where the fallback and all orders occur; the adjoint
with Lax-Friedrichs against the dense oracle adjoint."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from gpu_helpers import both_problems, from_workload
from test_gpu_parity import lockstep

pytestmark = pytest.mark.gpu

LF, HLL, PSI2M, ROE, SQUARE = 1, 2, 4, 8, 16


@pytest.mark.parametrize("flags", [LF, HLL, PSI2M, PSI2M | LF, PSI2M | HLL])
@pytest.mark.parametrize("bc", ["periodic", "transmissive"])
def test_variants_lockstep_euler1d(acat, flags, bc):
    w = workloads.euler_1d(n=600, P=4)
    po, pg = from_workload(w, bc=bc, flags=flags)
    lockstep(acat, po, pg, w["u"], 0.5, 12, label=f"euler1d flags={flags} {bc}")


@pytest.mark.parametrize("flags", [ROE, ROE | PSI2M, ROE | HLL])
def test_variants_lockstep_burgers(acat, flags):
    w = workloads.burgers_1d(n=300)
    po, pg = from_workload(w, P=3, flags=flags)
    lockstep(acat, po, pg, w["u"], 0.5, 20, label=f"burgers flags={flags}")


@pytest.mark.parametrize("name", ["einfeldt123", "blast_right"])
@pytest.mark.parametrize("flags", [LF, HLL])
def test_variants_shock_tubes_lockstep(acat, name, flags):
    w = workloads.paper_riemann_1d(name, P=3)
    po, pg = from_workload(w, flags=flags)
    lockstep(acat, po, pg, w["u"], w["cfl"], 15, label=f"{name} flags={flags}")


@pytest.mark.parametrize("flags", [LF, HLL, PSI2M])
@pytest.mark.parametrize("bc", ["periodic", "transmissive"])
def test_variants_lockstep_euler2d(acat, flags, bc):
    w = workloads.euler_2d(n=64, P=3)
    po, pg = from_workload(w, bc=bc, flags=flags)
    lockstep(acat, po, pg, w["u"], 0.4, 4, label=f"euler2d flags={flags} {bc}")


@pytest.mark.parametrize("P,flags", [(3, SQUARE), (4, SQUARE), (3, SQUARE | LF)])
@pytest.mark.parametrize("bc", ["periodic", "transmissive"])
def test_square_variant_lockstep_euler2d(acat, P, flags, bc):
    """Corners with q1 != q2 computed on two squares: their entries are
    listed twice (F only in class (q1, q1), G only in (q2, q2))."""
    w = workloads.euler_2d(n=64, P=P)
    po, pg = from_workload(w, bc=bc, flags=flags)
    r = oracle.step2d(po, w["u"], oracle.dt_cfl(po, w["u"], 0.4))
    assert (r["ordx"][:, :64] != r["ordy"][:64, :]).any()      # mixed corners occur
    lockstep(acat, po, pg, w["u"], 0.4, 4, label=f"euler2d square P={P} flags={flags} {bc}")


@pytest.mark.parametrize("bc", ["periodic", "transmissive"])
@pytest.mark.parametrize("q1,q2", [(a, b) for a in range(1, 5) for b in range(1, 5) if a != b])
def test_square_variant_every_class_forced(acat, q1, q2, bc):
    from test_gpu_adjoint import gpu_decisions
    nx, ny = 21, 17
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    X, Y = np.meshgrid(x, y, indexing="xy")
    rho = 1 + 0.1 * np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y)
    v, wv = 0.3 + 0.05 * np.sin(2 * np.pi * Y), -0.2 + 0.05 * np.cos(2 * np.pi * X)
    p = 1 + 0.05 * np.sin(2 * np.pi * (X + Y))
    u = np.stack([rho, rho * v, rho * wv, p / 0.4 + 0.5 * rho * (v * v + wv * wv)])
    po, pg = both_problems(2, 4, nx, "euler", 4, bc, 1.0 / nx, ny=ny, dy=1.0 / ny, flags=SQUARE)
    nIx, nIy = po.n_interfaces
    r = dict(ordx=np.full((ny, nIx), q1, np.int8), ordy=np.full((nIy, nx), q2, np.int8),
             psix=np.full((ny, nIx), 0.6), psiy=np.full((nIy, nx), 0.6),
             alx=np.full((ny, nIx), 2.0), aly=np.full((nIy, nx), 2.0))
    maps = (r["ordx"], r["ordy"], r["psix"], r["psiy"], r["alx"], r["aly"])
    dt = oracle.dt_cfl(po, u, 0.4)
    want = oracle.step2d(po, u, dt, maps=maps)["u"]
    got = acat.step_replay(pg, torch.from_numpy(u).cuda(), dt, gpu_decisions(acat, pg, po, r)).cpu().numpy()
    assert np.array_equal(got, want), (q1, q2, bc, np.abs(got - want).max())


@pytest.mark.parametrize("bc", ["periodic", "transmissive"])
@pytest.mark.parametrize("flags", [0, LF, HLL])
@pytest.mark.parametrize("q1,q2", [(1, 1), (1, 2), (2, 1), (1, 3), (3, 1)])
def test_order1_corners_forced_every_first_order_flux(acat, q1, q2, flags, bc):
    """Every corner of class (q1, q2) with an order-1 direction and blend
    weights in (0,1), so that both the CAT2 part and the first-order flux
    enter (the small classes take the blend's states and point fluxes from
    their own node lanes, the others reload them); Rusanov, Lax-Friedrichs
    and HLL, both boundaries, bitwise against the oracle."""
    from test_gpu_adjoint import gpu_decisions
    nx, ny = 23, 19
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    X, Y = np.meshgrid(x, y, indexing="xy")
    rho = 1 + 0.2 * np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y) + 0.3 * (X > 0.5)
    v, wv = 0.3 + 0.1 * np.sin(2 * np.pi * Y), -0.2 + 0.1 * np.cos(2 * np.pi * X)
    p = 1 + 0.1 * np.sin(2 * np.pi * (X + Y)) + 0.5 * (Y > 0.4)
    u = np.stack([rho, rho * v, rho * wv, p / 0.4 + 0.5 * rho * (v * v + wv * wv)])
    po, pg = both_problems(2, 4, nx, "euler", 3, bc, 1.0 / nx, ny=ny, dy=1.0 / ny, flags=flags)
    nIx, nIy = po.n_interfaces
    rng = np.random.default_rng(31 + flags)
    r = dict(ordx=np.full((ny, nIx), q1, np.int8), ordy=np.full((nIy, nx), q2, np.int8),
             psix=rng.uniform(0.1, 0.9, (ny, nIx)), psiy=rng.uniform(0.1, 0.9, (nIy, nx)),
             alx=rng.uniform(1.5, 3.0, (ny, nIx)), aly=rng.uniform(1.5, 3.0, (nIy, nx)))
    maps = (r["ordx"], r["ordy"], r["psix"], r["psiy"], r["alx"], r["aly"])
    dt = oracle.dt_cfl(po, u, 0.4)
    want = oracle.step2d(po, u, dt, maps=maps)["u"]
    got = acat.step_replay(pg, torch.from_numpy(u).cuda(), dt, gpu_decisions(acat, pg, po, r)).cpu().numpy()
    assert np.array_equal(got, want), (q1, q2, flags, bc, np.abs(got - want).max())


def test_variants_lockstep_advection2d_roe(acat):
    rng = np.random.default_rng(9)
    n = 40
    u = np.where(rng.uniform(size=(1, n, n)) > 0.5, 1.0, 0.0) + 0.1 * rng.standard_normal((1, n, n))
    po, pg = both_problems(2, 1, n, "advection", 3, "periodic", 0.1, ny=n, dy=0.1, ax=0.7, ay=-0.4,
                           flags=ROE | HLL)
    lockstep(acat, po, pg, u, 0.4, 5, label="advection2d roe+hll")


def _dense(acat, po, pg, u, dt):
    r = oracle.step1d(po, u, dt) if po.dim == 1 else oracle.step2d(po, u, dt)
    maps = oracle.maps_of(po, r)
    ub = np.random.default_rng(3).standard_normal(u.shape)
    want = oracle.vjp_dense(po, u, ub, dt, maps)
    dec = acat.Decisions(pg)
    names = ("order", "psi1", "alpha") if po.dim == 1 else ("ordx", "psix", "alx", "ordy", "psiy", "aly")
    dst = (dec.order_x, dec.psi1_x, dec.alpha_x) if po.dim == 1 else \
        (dec.order_x, dec.psi1_x, dec.alpha_x, dec.order_y, dec.psi1_y, dec.alpha_y)
    for nm, t in zip(names, dst):
        t.copy_(torch.from_numpy(np.ascontiguousarray(r[nm])))
    got = acat.step_adjoint(pg, torch.from_numpy(np.ascontiguousarray(u)).cuda(), dt, dec,
                            torch.from_numpy(ub).cuda()).cpu().numpy()
    return got, want


def test_adjoint_with_lax_friedrichs_1d(acat):
    w = workloads.euler_1d(n=32, P=3)
    po, pg = from_workload(w, bc="transmissive", flags=LF | PSI2M)
    dt = oracle.dt_cfl(po, w["u"], 0.5)
    got, want = _dense(acat, po, pg, w["u"], dt)
    assert np.abs(got - want).max() <= 1e-11 * np.abs(want).max()


def test_adjoint_with_lax_friedrichs_2d(acat):
    from test_gpu_adjoint import smooth_2d
    n = 20
    u = smooth_2d(n)
    po, pg = both_problems(2, 4, n, "euler", 2, "periodic", 1.0 / n, ny=n, dy=1.0 / n, flags=LF)
    dt = oracle.dt_cfl(po, u, 0.4)
    got, want = _dense(acat, po, pg, u, dt)
    assert np.abs(got - want).max() <= 1e-11 * np.abs(want).max()
