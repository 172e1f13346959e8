"""GPU adjoint (acat_step_adjoint, AdjointRun / ACATRun) against the oracle.

Per step, element by element: the kernel's ubar_in = J^T ubar_out against
the oracle's dense adjoint (J assembled column by column from the oracle's
dual-number JVP of the frozen replay step), with the decisions taken from
the oracle's own step.  Bound: max |gpu - oracle| <= 1e-11 max |oracle|
(the two sum the same products in different orders; the Jacobian entries
are O(1) and the sums have at most a few hundred terms).

At the adjoint workload's size (2D Euler 512^2, P = 2): the inner product
<J^T w, v> against the oracle's <w, J v> (<= 1e-10 relative), and central
finite differences of the GPU replay step (<= 1e-6 relative).  Over many
steps: the checkpointed ACATRun gradient against the oracle's tangent run
and against finite differences of the frozen replay run.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads
from gpu_helpers import both_problems, from_workload

pytestmark = pytest.mark.gpu

TOL_DENSE = 1e-11
TOL_JVP = 1e-10
TOL_FD = 1e-6


def gpu_decisions(acat, pg, po, r):
    dec = acat.Decisions(pg)
    names = ("order", "psi1", "alpha") if po.dim == 1 else ("ordx", "psix", "alx", "ordy", "psiy", "aly")
    dst = (dec.order_x, dec.psi1_x, dec.alpha_x) if po.dim == 1 else \
        (dec.order_x, dec.psi1_x, dec.alpha_x, dec.order_y, dec.psi1_y, dec.alpha_y)
    for n, t in zip(names, dst):
        t.copy_(torch.from_numpy(np.ascontiguousarray(r[n])))
    return dec


def smooth_2d(n, jump=True, amp=0.2):
    """Smooth periodic Euler state on [0,1]^2 with an x-band of higher
    density: at n = 24 and P = 3 every order class (q1, q2) occurs."""
    x = (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(x, x, indexing="xy")
    rho = 1 + amp * np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y)
    v = 0.3 + 0.1 * np.sin(2 * np.pi * Y)
    w = -0.2 + 0.1 * np.cos(2 * np.pi * X)
    p = 1 + 0.1 * np.sin(2 * np.pi * (X + Y))
    if jump:
        rho = rho + 0.5 * ((X > 0.4) & (X < 0.7))
    E = p / 0.4 + 0.5 * rho * (v * v + w * w)
    return np.stack([rho, rho * v, rho * w, E])


def dense_case(acat, po, pg, u, dt, seed=0):
    r = oracle.step1d(po, u, dt) if po.dim == 1 else oracle.step2d(po, u, dt)
    maps = oracle.maps_of(po, r)
    ub = np.random.default_rng(seed).standard_normal(u.shape)
    want = oracle.vjp_dense(po, u, ub, dt, maps)
    dec = gpu_decisions(acat, pg, po, r)
    ug = torch.from_numpy(np.ascontiguousarray(u)).cuda()
    got = acat.step_adjoint(pg, ug, dt, dec, torch.from_numpy(ub).cuda()).cpu().numpy()
    return got, want, r


def orders_seen(po, r):
    if po.dim == 1:
        return set(np.unique(r["order"]).tolist())
    return set(zip(r["ordx"].ravel().tolist(), r["ordy"].ravel().tolist()))


@pytest.mark.parametrize("P", [2, 3, 4, 5, 6])
@pytest.mark.parametrize("bc", ["periodic", "transmissive"])
def test_adjoint_1d_euler_matches_dense_oracle(acat, P, bc):
    w = workloads.euler_1d(n=32, P=P)
    po, pg = from_workload(w, bc=bc)
    dt = oracle.dt_cfl(po, w["u"], 0.5)
    got, want, r = dense_case(acat, po, pg, w["u"], dt, seed=P)
    assert orders_seen(po, r) >= {1, P}
    err = np.abs(got - want).max()
    print(f"1D euler P={P} {bc}: max err {err:.3e} (scale {np.abs(want).max():.3e})", flush=True)
    assert err <= TOL_DENSE * np.abs(want).max()


@pytest.mark.parametrize("flux,P,bc", [("burgers", 3, "transmissive"), ("burgers", 4, "periodic"),
                                       ("advection", 2, "periodic"), ("advection", 3, "transmissive")])
def test_adjoint_1d_scalar_matches_dense_oracle(acat, flux, P, bc):
    n = 32
    rng = np.random.default_rng(P)
    x = (np.arange(n) + 0.5) / n
    u = (np.sin(2 * np.pi * x) + 0.5 * (x > 0.5) + 0.01 * rng.standard_normal(n))[None, :]
    po, pg = both_problems(1, 1, n, flux, P, bc, 1.0 / n, ax=0.7)
    dt = oracle.dt_cfl(po, u, 0.5)
    got, want, _ = dense_case(acat, po, pg, u, dt, seed=P + 10)
    assert np.abs(got - want).max() <= TOL_DENSE * np.abs(want).max()


@pytest.mark.parametrize("P", [2, 3, 4])
def test_adjoint_2d_euler_matches_dense_oracle(acat, P):
    n = 24
    u = smooth_2d(n)
    po, pg = both_problems(2, 4, n, "euler", P, "periodic", 1.0 / n, ny=n, dy=1.0 / n)
    dt = oracle.dt_cfl(po, u, 0.4)
    got, want, r = dense_case(acat, po, pg, u, dt, seed=20 + P)
    if P == 3:
        assert len(orders_seen(po, r)) == 9      # every corner class (q1, q2)
    err = np.abs(got - want).max()
    print(f"2D euler P={P}: max err {err:.3e} (scale {np.abs(want).max():.3e})", flush=True)
    assert err <= TOL_DENSE * np.abs(want).max()


@pytest.mark.parametrize("P", [1, 2, 3, 4])
def test_adjoint_2d_transmissive_matches_dense_oracle(acat, P):
    """Transmissive 2D: the edge fluxes enter one cell each, ghost-row and
    ghost-column corners carry one flux, and the clamped ghost reads add
    their adjoints to the edge cells.  Non-square grid, every order class."""
    nx, ny = 30, 27
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    X, Y = np.meshgrid(x, y, indexing="xy")
    rho = 1 + 0.2 * np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y) + 0.5 * ((X > 0.4) & (X < 0.7))
    v, w = 0.3 + 0.1 * np.sin(2 * np.pi * Y), -0.2 + 0.1 * np.cos(2 * np.pi * X)
    p = 1 + 0.1 * np.sin(2 * np.pi * (X + Y)) + 0.6 * (Y < 0.3)
    u = np.stack([rho, rho * v, rho * w, p / 0.4 + 0.5 * rho * (v * v + w * w)])
    po, pg = both_problems(2, 4, nx, "euler", P, "transmissive", 1.0 / nx, ny=ny, dy=1.0 / ny)
    dt = oracle.dt_cfl(po, u, 0.4)
    got, want, r = dense_case(acat, po, pg, u, dt, seed=40 + P)
    # corner (i1, i2) takes the orders of x-interface (i1 + 1/2, i2) and y-interface (i1, i2 + 1/2)
    corners = {(int(r["ordx"][i2, i1 + 1]), int(r["ordy"][i2 + 1, i1])) for i2 in range(ny) for i1 in range(nx)}
    assert len(corners) == P * P, corners
    err = np.abs(got - want).max()
    print(f"2D euler transmissive P={P}: max err {err:.3e} (scale {np.abs(want).max():.3e})", flush=True)
    assert err <= TOL_DENSE * np.abs(want).max()


def test_adjoint_2d_transmissive_advection_lf(acat):
    n = 14
    rng = np.random.default_rng(5)
    u = rng.standard_normal((1, n, n + 3))
    po, pg = both_problems(2, 1, n + 3, "advection", 2, "transmissive", 0.1, ny=n, dy=0.12, ax=0.8, ay=-0.5,
                           flags=oracle.FLAG_FLO_LF)
    dt = oracle.dt_cfl(po, u, 0.4)
    got, want, _ = dense_case(acat, po, pg, u, dt, seed=9)
    assert np.abs(got - want).max() <= TOL_DENSE * np.abs(want).max()


def test_adjoint_2d_advection_matches_dense_oracle(acat):
    n = 16
    rng = np.random.default_rng(3)
    u = rng.standard_normal((1, n, n))
    po, pg = both_problems(2, 1, n, "advection", 3, "periodic", 0.1, ny=n, dy=0.12, ax=0.8, ay=-0.5)
    dt = oracle.dt_cfl(po, u, 0.4)
    got, want, _ = dense_case(acat, po, pg, u, dt, seed=7)
    assert np.abs(got - want).max() <= TOL_DENSE * np.abs(want).max()


def test_adjoint_in_place_device_dt_and_zero_dt(acat):
    n = 24
    u = smooth_2d(n)
    po, pg = both_problems(2, 4, n, "euler", 3, "periodic", 1.0 / n, ny=n, dy=1.0 / n)
    dt = oracle.dt_cfl(po, u, 0.4)
    r = oracle.step2d(po, u, dt)
    dec = gpu_decisions(acat, pg, po, r)
    ug = torch.from_numpy(u).cuda()
    ub = torch.from_numpy(np.random.default_rng(1).standard_normal(u.shape)).cuda()
    ref = acat.step_adjoint(pg, ug, dt, dec, ub)
    dt_dev = torch.tensor([dt], dtype=torch.float64, device="cuda")
    inplace = ub.clone()
    acat.step_adjoint(pg, ug, dt_dev, dec, inplace, ubar_in=inplace)
    assert torch.equal(inplace, ref)
    # dt = 0: the step is the identity, and so is its adjoint
    assert torch.equal(acat.step_adjoint(pg, ug, 0.0, dec, ub), ub)
    # deterministic: a second call gives the same bits
    assert torch.equal(acat.step_adjoint(pg, ug, dt, dec, ub), ref)
    assert acat.device_status() == 0


@pytest.mark.parametrize("case", ["1d P=3", "1d P=6", "2d P=2", "2d P=3", "2d P=4"])
@pytest.mark.parametrize("bc", ["periodic", "transmissive"])
@pytest.mark.parametrize("fwd", ["cfl", "replay"])
def test_adjoint_reusing_step_lists_equals_adjoint(acat, case, bc, fwd):
    """acat_step_adjoint_lists after the forward step (recording, or replaying
    the recorded decisions) gives acat_step_adjoint's result bit for bit, and
    leaves the step workspace unchanged."""
    dim, P = int(case[0]), int(case[-1])
    if dim == 1:
        w = workloads.euler_1d(n=200, P=P)
        po, pg = from_workload(w, bc=bc)
        u = w["u"]
    else:
        n = 40
        u = smooth_2d(n)
        po, pg = both_problems(2, 4, n, "euler", P, bc, 1.0 / n, ny=n, dy=1.0 / n)
    ug = torch.from_numpy(np.ascontiguousarray(u)).cuda()
    dec = acat.Decisions(pg)
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    sws = acat.workspace(pg)
    out = torch.empty_like(ug)
    acat.step_cfl(pg, ug, 0.4, dt, out=out, ws=sws, dec=dec)
    if fwd == "replay":
        sws = acat.workspace(pg)
        acat.step_replay(pg, ug, dt, dec, out=out, ws=sws)
    ub = torch.from_numpy(np.random.default_rng(P).standard_normal(u.shape)).cuda()
    ref = acat.step_adjoint(pg, ug, dt, dec, ub)
    before = sws.clone()
    got = acat.step_adjoint_lists(pg, ug, dt, dec, ub, sws)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
    assert torch.equal(sws, before)
    assert acat.device_status() == 0


def test_adjoint_1d_bad_recorded_order_is_flagged(acat):
    w = workloads.euler_1d(n=32, P=3)
    po, pg = from_workload(w)
    dt = oracle.dt_cfl(po, w["u"], 0.5)
    r = oracle.step1d(po, w["u"], dt)
    dec = gpu_decisions(acat, pg, po, r)
    dec.order_x[5] = 7                       # outside 1..P: taken as 1, flagged
    ug = torch.from_numpy(w["u"]).cuda()
    out = acat.step_adjoint(pg, ug, dt, dec, torch.ones_like(ug))
    assert torch.isfinite(out).all()
    assert acat.device_status() & 4


# ---------------------------------------------------------------- C5 scale
@pytest.fixture(scope="module")
def c5():
    return workloads.adjoint_2d()


def test_adjoint_step_c5_inner_product_and_fd(acat, c5):
    w = c5
    po, pg = from_workload(w)
    u = w["u"]
    dt = oracle.dt_cfl(po, u, w["cfl"])
    r = oracle.step2d(po, u, dt, nthreads=16)
    maps = oracle.maps_of(po, r)
    dec = gpu_decisions(acat, pg, po, r)
    rng = np.random.default_rng(11)
    wb = rng.standard_normal(u.shape)
    ug = torch.from_numpy(u).cuda()
    adj = acat.step_adjoint(pg, ug, dt, dec, torch.from_numpy(wb).cuda()).cpu().numpy()
    for k in range(2):
        v = w["directions"](k)
        lhs = float(np.vdot(adj, v))
        rhs = float(np.vdot(wb, oracle.jvp(po, u, v, dt, maps, nthreads=16)[1]))
        assert abs(lhs - rhs) <= TOL_JVP * abs(rhs), (k, lhs, rhs)
        h = 1e-6
        vg = torch.from_numpy(v).cuda()
        up = acat.step_replay(pg, ug + h * vg, dt, dec).cpu().numpy()
        um = acat.step_replay(pg, ug - h * vg, dt, dec).cpu().numpy()
        fd = float(np.vdot(wb, (up - um) / (2 * h)))
        assert abs(fd - lhs) <= TOL_FD * abs(lhs), (k, fd, lhs)


def misfit_grad(w, u_T, rho_star):
    """dL/du_T of L = 1/2 dx dy sum (rho_T - rho*_T)^2."""
    g = torch.zeros_like(u_T)
    g[0] = w["dx"] * w["dy"] * (u_T[0] - rho_star)
    return g


@pytest.mark.parametrize("n,nsteps,k,bc,P", [(64, 12, 5, "periodic", 2), (64, 10, 10, "periodic", 2),
                                             (48, 8, 3, "transmissive", 2), (40, 6, 4, "transmissive", 4)])
def test_checkpointed_run_matches_oracle_tangent(acat, n, nsteps, k, bc, P):
    """Gradient of a misfit after nsteps through ACATRun (checkpoint every k)
    against the oracle's tangent run along two directions; both boundaries,
    orders 4 and 8."""
    w = workloads.adjoint_2d(n=n)
    po, pg = from_workload(w, bc=bc, P=P)
    uT_o, _, _, hist = oracle.run(po, w["u"], w["cfl"], nsteps=nsteps, nthreads=16, record=True)
    star = oracle.run(po, w["target_u0"], w["cfl"], nsteps=nsteps, nthreads=16)[0][0]
    run = acat.AdjointRun(pg, w["cfl"], nsteps, checkpoint_every=k)
    u0 = torch.from_numpy(w["u"]).cuda().requires_grad_(True)
    uT = acat.ACATRun.apply(u0, run)
    assert torch.equal(uT.detach().cpu(), torch.from_numpy(uT_o))     # forward: bitwise
    loss = 0.5 * w["dx"] * w["dy"] * ((uT[0] - torch.from_numpy(star).cuda()) ** 2).sum()
    loss.backward()
    grad = u0.grad.cpu().numpy()
    gT = misfit_grad(w, torch.from_numpy(uT_o), torch.from_numpy(star)).numpy()
    for j in range(2):
        v = w["directions"](j)
        dv = v.copy()
        for hstep in hist:
            dv = oracle.jvp(po, hstep["u"], dv, hstep["dt"], oracle.maps_of(po, hstep), nthreads=16)[1]
        rhs = float(np.vdot(gT, dv))
        lhs = float(np.vdot(grad, v))
        assert abs(lhs - rhs) <= TOL_JVP * abs(rhs), (j, lhs, rhs)


def test_checkpointed_run_matches_fd_of_replay(acat):
    """ACATRun gradient against central differences of the frozen replay run
    (decisions and time steps of the forward run), 4 directions."""
    w = workloads.adjoint_2d(n=128)
    po, pg = from_workload(w)
    nsteps = 20
    star = torch.from_numpy(oracle.run(po, w["target_u0"], w["cfl"], nsteps=nsteps, nthreads=16)[0][0]).cuda()
    run = acat.AdjointRun(pg, w["cfl"], nsteps, checkpoint_every=5, record_all=True)
    u0 = torch.from_numpy(w["u"]).cuda()
    uT = run.forward(u0)
    gT = misfit_grad(w, uT, star)
    grad = run.backward(gT)

    def loss(u):
        return 0.5 * w["dx"] * w["dy"] * float(((u[0] - star) ** 2).sum())

    for j in range(4):
        v = torch.from_numpy(w["directions"](j)).cuda()
        ad = float((grad * v).sum())
        best = min(abs((loss(run.replay(u0 + h * v)) - loss(run.replay(u0 - h * v))) / (2 * h) - ad)
                   for h in (1e-4, 1e-5, 1e-6))
        assert best <= TOL_FD * abs(ad), (j, best, ad)


def test_graph_captured_segments_match_eager(acat):
    """AdjointRun with graph-captured segments (k = 4, 10 steps: lengths 4
    and 2) gives the same forward state and gradient, bit for bit, as the
    eager run; a second backward after one forward (whose last segment is
    then no longer resident) gives the same gradient."""
    import torch
    w = workloads.adjoint_2d(n=64)
    po, pg = from_workload(w)
    u0 = torch.from_numpy(w["u"]).cuda()
    res = []
    for graphs in (False, True):
        run = acat.AdjointRun(pg, w["cfl"], 10, checkpoint_every=4, graphs=graphs)
        uT = run.forward(u0)
        g = run.backward(uT * 0.5)
        uT2 = run.forward(u0)                       # replayed graphs the second time
        g2 = run.backward(uT2 * 0.5)
        g3 = run.backward(uT2 * 0.5)
        assert torch.equal(uT, uT2) and torch.equal(g, g2) and torch.equal(g, g3)
        res.append((uT, g))
    assert torch.equal(res[0][0], res[1][0]) and torch.equal(res[0][1], res[1][1])


@pytest.mark.parametrize("graphs", [False, True])
def test_overlapped_reverse_pass_equals_serial(acat, graphs):
    """The reverse pass with the recomputation of segment s - 1 on a second
    stream (two buffer sets, the default) gives the serial pass's gradient
    bit for bit, with the recomputed decisions verified against the forward
    run; 23 steps, checkpoints every 5 (segments 5, 5, 5, 5, 3), backward
    twice after one forward; the per-step class counts agree too."""
    import torch
    w = workloads.adjoint_2d(n=64)
    po, pg = from_workload(w)
    u0 = torch.from_numpy(w["u"]).cuda()
    ser = acat.AdjointRun(pg, w["cfl"], 23, checkpoint_every=5, graphs=False, overlap=False)
    ser.class_log = torch.zeros((23, 16), dtype=torch.int32, device="cuda")
    g_ser = ser.backward(ser.forward(u0) * 0.5)
    ovl = acat.AdjointRun(pg, w["cfl"], 23, checkpoint_every=5, graphs=graphs)
    assert ovl.overlap and len(ovl.segs) == 2
    ovl.class_log = torch.zeros((23, 16), dtype=torch.int32, device="cuda")
    uT = ovl.forward(u0)
    g1 = ovl.backward(uT * 0.5)
    g2 = ovl.backward(uT * 0.5)
    assert torch.equal(g_ser, g1) and torch.equal(g_ser, g2)
    # the per-step class counts of each adjoint step land on the same steps
    # (P = 2: classes 0..3; the later entries of a log row are not defined)
    ncls = w["P"] * w["P"]
    assert torch.equal(ser.class_log[:, :ncls], ovl.class_log[:, :ncls]) and int(ser.class_log[:, :ncls].sum()) > 0


def test_auto_checkpoint_gives_the_same_gradient(acat):
    """checkpoint_every="auto" (the whole 10-step run resident: no
    recomputation) and a budget of six steps (two alternating buffer sets of
    three: segments 3, 3, 3, 1) give the gradient of checkpoint_every=4 bit
    for bit."""
    import torch
    w = workloads.adjoint_2d(n=64)
    po, pg = from_workload(w)
    u0 = torch.from_numpy(w["u"]).cuda()
    ref = acat.AdjointRun(pg, w["cfl"], 10, checkpoint_every=4)
    g_ref = ref.backward(ref.forward(u0) * 0.5)
    auto = acat.AdjointRun(pg, w["cfl"], 10, checkpoint_every="auto")
    assert auto.k == 10
    g_auto = auto.backward(auto.forward(u0) * 0.5)
    per = acat.resident_bytes_per_step(pg)
    small = acat.AdjointRun(pg, w["cfl"], 10, checkpoint_every="auto", memory_budget=6 * per + 1)
    assert small.k == 3
    g_small = small.backward(small.forward(u0) * 0.5)
    assert torch.equal(g_ref, g_auto) and torch.equal(g_ref, g_small)


@pytest.mark.parametrize("bc", ["periodic", "transmissive"])
@pytest.mark.parametrize("q1,q2", [(a, b) for a in range(1, 5) for b in range(1, 5)])
def test_adjoint_every_corner_class_forced(acat, q1, q2, bc):
    """Every 2D corner class of P = 4, forced through replay maps on smooth
    data (psi^1 = 0.6 and alpha = 2 where an order is 1), on a non-square
    grid with both boundaries: the GPU adjoint against the oracle's dense
    adjoint of the same frozen step."""
    nx, ny = 10, 9
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
    dt = 0.2 * oracle.dt_cfl(po, u, 0.4)
    ub = np.random.default_rng(10 * q1 + q2).standard_normal(u.shape)
    want = oracle.vjp_dense(po, u, ub, dt, maps)
    dec = gpu_decisions(acat, pg, po, r)
    got = acat.step_adjoint(pg, torch.from_numpy(u).cuda(), dt, dec, torch.from_numpy(ub).cuda()).cpu().numpy()
    bad = np.argwhere(~np.isfinite(got))
    err = np.abs(got - want).max()
    print(f"class ({q1},{q2}) {bc}: max err {err:.3e}, non-finite {len(bad)} first {bad[:3].tolist()}", flush=True)
    assert np.all(np.isfinite(got)) and err <= TOL_DENSE * np.abs(want).max()


def test_checkpointed_gradient_full_size_c5_matches_oracle_tangent(acat):
    """The adjoint workload as the benchmark runs it: 2D Euler 512^2, P = 2,
    200 CFL steps, checkpoint every 20 steps, graph-captured segments
    (ACATRun).  <grad, d_j> for two smooth directions against the oracle's
    tangent run (its own CFL steps and decisions, both tangents carried in
    one pass): within 1e-10 relative; the GPU's final state equals the
    oracle's bit for bit.  The misfit's target is the initial density (the
    target only fixes the cotangent at the final time)."""
    import time
    w = workloads.adjoint_2d()
    po, pg = from_workload(w)
    nsteps, k = w["nsteps"], w["checkpoint_every"]
    star = w["u"][0].copy()
    run = acat.AdjointRun(pg, w["cfl"], nsteps, checkpoint_every=k)
    u0 = torch.from_numpy(w["u"]).cuda().requires_grad_(True)
    uT = acat.ACATRun.apply(u0, run)
    loss = 0.5 * w["dx"] * w["dy"] * ((uT[0] - torch.from_numpy(star).cuda()) ** 2).sum()
    loss.backward()
    grad = u0.grad.cpu().numpy()
    uT = uT.detach().cpu().numpy()
    t0 = time.time()
    u = w["u"].copy()
    dirs = np.stack([w["directions"](0), w["directions"](1)])
    dv = dirs.copy()
    for n in range(nsteps):
        dt = oracle.dt_cfl(po, u, w["cfl"])
        u, dv = oracle.jvp2(po, u, dv, dt, nthreads=16)
        if n % 50 == 49:
            print(f"[C5 oracle tangent] step {n + 1} ({time.time() - t0:.0f} s)", flush=True)
    assert np.array_equal(uT, u)
    gT = w["dx"] * w["dy"] * (u[0] - star)
    for j in range(2):
        rhs = float(np.vdot(gT, dv[j][0]))
        lhs = float(np.vdot(grad, dirs[j]))
        print(f"[C5 full size] direction {j}: adjoint {lhs:.15e} tangent {rhs:.15e} "
              f"rel {abs(lhs - rhs) / abs(rhs):.2e}", flush=True)
        assert abs(lhs - rhs) <= TOL_JVP * abs(rhs), (j, lhs, rhs)
