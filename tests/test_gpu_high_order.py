"""GPU parity at the higher orders: P = 5, 6 in 1D (orders 10, 12) and P = 4
in 2D (order 8, corner rectangles up to 8 x 8 nodes), bit for bit against
the oracle in lockstep and over free-running runs."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_helpers import both_problems, from_workload
from test_gpu_parity import lockstep

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("P", [5, 6])
@pytest.mark.parametrize("bc", ["periodic", "transmissive"])
def test_lockstep_euler1d_high_order(acat, P, bc):
    w = workloads.euler_1d(n=800, P=P)
    po, pg = from_workload(w, bc=bc)
    lockstep(acat, po, pg, w["u"], 0.5, 10, label=f"euler1d P={P} {bc}")


def test_lockstep_burgers_p6(acat):
    w = workloads.burgers_1d(n=300)
    po, pg = from_workload(w, P=6)
    lockstep(acat, po, pg, w["u"], 0.5, 20, label="burgers P=6")


def test_free_running_euler1d_p6(acat):
    w = workloads.euler_1d(n=1024, P=6)
    po, pg = from_workload(w)
    uo, t, n = oracle.run(po, w["u"], w["cfl"], t_final=0.05)
    s = acat.Solver(pg, w["u"], w["cfl"], t_final=0.05)
    s.run_to_end(check_every=32)
    assert abs(s.time() - t) == 0.0 and np.array_equal(s.u.cpu().numpy(), uo)


@pytest.mark.parametrize("bc", ["periodic", "transmissive"])
def test_lockstep_euler2d_p4(acat, bc):
    w = workloads.euler_2d(n=64, P=4)
    po, pg = from_workload(w, bc=bc)
    lockstep(acat, po, pg, w["u"], 0.4, 4, label=f"euler2d P=4 {bc}")


def test_lockstep_advection2d_p4(acat):
    rng = np.random.default_rng(4)
    n = 48
    x = (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(x, x, indexing="xy")
    u = (np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y) + (X > 0.5) * 0.5 + 0.01 * rng.standard_normal(X.shape))[None]
    po, pg = both_problems(2, 1, n, "advection", 4, "periodic", 1.0 / n, ny=n, dy=1.0 / n, ax=0.7, ay=-0.4)
    lockstep(acat, po, pg, u, 0.4, 6, label="advection2d P=4")


def test_free_running_euler2d_p4(acat):
    w = workloads.paper_lax_liu(6, n=80, P=4)
    po, pg = from_workload(w)
    uo, t, n = oracle.run(po, w["u"], w["cfl"], t_final=0.1, nthreads=16)
    s = acat.Solver(pg, w["u"], w["cfl"], t_final=0.1)
    s.run_to_end(check_every=32)
    assert s.time() == t and np.array_equal(s.u.cpu().numpy(), uo)


@pytest.mark.parametrize("bc", ["periodic", "transmissive"])
@pytest.mark.parametrize("q1,q2", [(a, b) for a in range(1, 5) for b in range(1, 5)])
def test_forward_every_corner_class_forced(acat, q1, q2, bc):
    """Every 2D corner class of P = 4 forced through replay maps (psi^1 =
    0.6, alpha = 2 where an order is 1) on smooth Euler data, non-square
    grid: the replayed GPU step equals the oracle's bit for bit."""
    import torch
    from test_gpu_adjoint import gpu_decisions
    nx, ny = 21, 17
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    X, Y = np.meshgrid(x, y, indexing="xy")
    rho = 1 + 0.1 * np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y)
    v, w = 0.3 + 0.05 * np.sin(2 * np.pi * Y), -0.2 + 0.05 * np.cos(2 * np.pi * X)
    p = 1 + 0.05 * np.sin(2 * np.pi * (X + Y))
    u = np.stack([rho, rho * v, rho * w, p / 0.4 + 0.5 * rho * (v * v + w * w)])
    po, pg = both_problems(2, 4, nx, "euler", 4, bc, 1.0 / nx, ny=ny, dy=1.0 / ny)
    nIx, nIy = po.n_interfaces
    r = dict(ordx=np.full((ny, nIx), q1, np.int8), ordy=np.full((nIy, nx), q2, np.int8),
             psix=np.full((ny, nIx), 0.6), psiy=np.full((nIy, nx), 0.6),
             alx=np.full((ny, nIx), 2.0), aly=np.full((nIy, nx), 2.0))
    maps = (r["ordx"], r["ordy"], r["psix"], r["psiy"], r["alx"], r["aly"])
    dt = oracle.dt_cfl(po, u, 0.4)
    want = oracle.step2d(po, u, dt, maps=maps)["u"]
    dec = gpu_decisions(acat, pg, po, r)
    got = acat.step_replay(pg, torch.from_numpy(u).cuda(), dt, dec).cpu().numpy()
    assert np.array_equal(got, want), (q1, q2, bc, np.abs(got - want).max())
