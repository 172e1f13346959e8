"""GPU parity at the edges of the problem space, bit for bit against the
oracle: the smallest grids each order admits (the stencil of 2 max(P, 2)
nodes covers the whole periodic grid), sizes around the number of
interfaces or corners one block takes per round (so that class lists end
in ragged tails and some lanes are idle), odd non-square 2D grids, single
discontinuities (order classes with one or two items), and states where
every order class but one is empty."""
import numpy as np
import pytest

import oracle
from gpu_helpers import both_problems
from test_gpu_parity import lockstep

pytestmark = pytest.mark.gpu


def euler1d_data(n):
    x = (np.arange(n) + 0.5) / n
    rho = 1.0 + 0.3 * np.sin(2 * np.pi * x) + 0.5 * (x > 0.6)
    v = 0.2 * np.cos(2 * np.pi * x)
    p = 1.0 + 0.2 * np.sin(4 * np.pi * x) + 1.0 * (x < 0.3)
    return np.stack([rho, rho * v, p / 0.4 + 0.5 * rho * v * v])


def euler2d_data(nx, ny):
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    X, Y = np.meshgrid(x, y, indexing="xy")
    rho = 1.0 + 0.3 * np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y) + 0.4 * (X > 0.55)
    v = 0.2 * np.cos(2 * np.pi * Y)
    w = -0.15 * np.sin(2 * np.pi * X)
    p = 1.0 + 0.2 * np.sin(2 * np.pi * (X + Y)) + 0.8 * (Y < 0.35)
    return np.stack([rho, rho * v, rho * w, p / 0.4 + 0.5 * rho * (v * v + w * w)])


def G(P):
    return max(P, 2)


# interfaces per 256-lane block and round: 2p lanes per interface, whole
# interfaces per 64-lane wavefront (4 lanes idle for p = 3, 5, 6)
ROUND_1D = {1: 128, 2: 64, 3: 40, 4: 32, 5: 24, 6: 20}


@pytest.mark.parametrize("P", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("bc", ["periodic", "transmissive"])
def test_euler1d_smallest_and_ragged_grids(acat, P, bc):
    sizes = sorted({2 * G(P), 2 * G(P) + 1, ROUND_1D[P] - 1, ROUND_1D[P] + 1, 2 * ROUND_1D[P] + 3})
    for n in sizes:
        po, pg = both_problems(1, 3, n, "euler", P, bc, 1.0 / n)
        lockstep(acat, po, pg, euler1d_data(n), 0.4, 3, label=f"euler1d P={P} {bc} n={n}")


@pytest.mark.parametrize("P", [1, 2, 3, 4, 5, 6])
def test_burgers_smallest_grid(acat, P):
    """Amplitude 0.1: on the smallest periodic grids a unit-amplitude sine
    is so under-resolved that the order-8 and order-12 predictions (up to P
    time steps ahead, through stencils that wrap the whole grid) diverge in
    the oracle itself within one step (2.9e3 at P = 4, 1e104 at P = 6)."""
    n = 2 * G(P)
    x = (np.arange(n) + 0.5) / n
    u = (0.5 + 0.1 * np.sin(2 * np.pi * x))[None]
    for bc in ("periodic", "transmissive"):
        po, pg = both_problems(1, 1, n, "burgers", P, bc, 1.0 / n)
        lockstep(acat, po, pg, u, 0.5, 4, label=f"burgers P={P} {bc} n={n}")


@pytest.mark.parametrize("P", [1, 2, 3, 4])
@pytest.mark.parametrize("bc", ["periodic", "transmissive"])
def test_euler2d_smallest_and_odd_grids(acat, P, bc):
    g = 2 * G(P)
    for nx, ny in ((g, g), (g + 1, g + 3), (13, 29), (31, 10)):
        if min(nx, ny) < g:
            continue
        po, pg = both_problems(2, 4, nx, "euler", P, bc, 1.0 / nx, ny=ny, dy=1.0 / ny)
        lockstep(acat, po, pg, euler2d_data(nx, ny), 0.4, 2, label=f"euler2d P={P} {bc} {nx}x{ny}")


@pytest.mark.parametrize("P", [2, 3, 4, 6])
def test_single_jump_gives_sparse_low_order_classes(acat, P):
    """A constant state with one density jump (a contact at rest): the low
    order classes hold only the few interfaces next to the jump."""
    n = 257
    rho = np.where(np.arange(n) < 100, 1.0, 0.5)
    u = np.stack([rho, np.zeros(n), np.full(n, 2.5)])
    po, pg = both_problems(1, 3, n, "euler", P, "transmissive", 1.0 / n)
    dec = acat.Decisions(pg)
    import torch
    acat.step(pg, torch.as_tensor(u, device="cuda"), 1e-3, dec=dec)
    counts = np.bincount(dec.order_x.cpu().numpy().astype(np.int64), minlength=P + 1)[1:]
    assert counts[-1] > n - 2 * P * 2 and counts[:-1].sum() <= 4 * P, counts
    lockstep(acat, po, pg, u, 0.5, 5, label=f"single jump P={P}")


@pytest.mark.parametrize("dim", [1, 2])
def test_all_items_in_one_class(acat, dim):
    """A smooth single-mode state: every item in the top order class, the
    other class lists empty."""
    if dim == 1:
        n = 96
        x = (np.arange(n) + 0.5) / n
        rho = 1.0 + 0.1 * np.sin(2 * np.pi * x)
        u = np.stack([rho, rho * 0.3, 1.0 / 0.4 + 0.5 * rho * 0.09])
        po, pg = both_problems(1, 3, n, "euler", 4, "periodic", 1.0 / n)
    else:
        n = 48
        x = (np.arange(n) + 0.5) / n
        X, Y = np.meshgrid(x, x, indexing="xy")
        rho = 1.0 + 0.1 * np.sin(2 * np.pi * (X + Y))
        u = np.stack([rho, 0.3 * rho, -0.2 * rho, 3.0 + 0.5 * rho * 0.13])
        po, pg = both_problems(2, 4, n, "euler", 3, "periodic", 1.0 / n, ny=n, dy=1.0 / n)
    r = oracle.step(po, u, 1e-3)
    orders = [r["order"]] if dim == 1 else [r["ordx"], r["ordy"]]
    assert all(np.all(o == po.P) for o in orders)
    lockstep(acat, po, pg, u, 0.5, 3, label=f"one class dim={dim}")
