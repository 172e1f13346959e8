"""Batched step (many independent 1D problems, one launch per order class):
bitwise equal to per-problem steps and to the oracle."""
import sys

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def T(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def concat(states):
    return np.concatenate(states, axis=1)


def make_batch(acat, probs):
    return acat.Batch([p["u"].shape[1] for p in probs], [p["P"] for p in probs], [p["bc"] for p in probs],
                      [p["dx"] for p in probs], flux=probs[0]["flux"], nvar=probs[0]["nvar"])


def test_batched_c4_equals_per_instance_steps(acat):
    """256 Euler problems, N log-uniform in [512, 16384], P in {2,3,4}."""
    import torch
    w = workloads.batch_1d()
    probs = w["problems"]
    batch = make_batch(acat, probs)
    bs = acat.BatchSolver(batch, concat([p["u"] for p in probs]), w["cfl"])
    singles = []
    for p in probs:
        pg = acat.Problem(dim=1, nvar=3, nx=p["u"].shape[1], flux="euler", P=p["P"], bc=p["bc"], dx=p["dx"])
        singles.append(acat.Solver(pg, p["u"], w["cfl"]))
    for n in range(3):
        # the time steps this step uses, by the separate reduction; after the
        # first step the solver holds them already (reduced inside the last step)
        used = torch.empty_like(bs.dt)
        batch.cfl_dt(bs.u, w["cfl"], used)
        if bs.dt_valid:
            assert torch.equal(used, bs.dt), f"fused time steps before step {n}"
        bs.step()
        for s in singles:
            s.step()
        torch.cuda.synchronize()
        got = bs.u.cpu().numpy()
        parts = batch.split(got)
        dts = used.cpu().numpy()
        for b, s in enumerate(singles):
            assert float(s.dt.item()) == dts[b], f"dt problem {b} step {n}"
            assert np.array_equal(parts[b], s.u.cpu().numpy()), f"state problem {b} step {n}"
    say(f"[batched C4] {batch.nprob} problems, {batch.ncell} cells: 3 steps bitwise equal to per-problem steps")


@pytest.mark.parametrize("flux", ["euler", "burgers"])
def test_batched_lockstep_oracle(acat, flux):
    rng = np.random.default_rng(3)
    probs = []
    for b in range(12):
        n = int(rng.integers(16, 300))
        P = int(rng.integers(1, 5))
        bc = "periodic" if b % 3 == 0 else "transmissive"
        if flux == "euler":
            p = workloads.euler_1d(n=n, P=P, stream=(b,))
        else:
            x = np.arange(n) / n
            p = dict(u=(np.sin(2 * np.pi * x + b) + (x > 0.5))[None].copy(), dx=1.0 / n, flux="burgers", P=P,
                     nvar=1)
        p["bc"] = bc
        p["P"] = P
        probs.append(p)
    batch = make_batch(acat, probs)
    us = [p["u"].copy() for p in probs]
    u = T(concat(us))
    import torch
    dt = torch.zeros(batch.nprob, dtype=torch.float64, device="cuda")
    fid = oracle.FLUX_EULER if flux == "euler" else oracle.FLUX_BURGERS
    for step in range(8):
        batch.cfl_dt(u, 0.6, dt)
        u = batch.step(u, dt)
        dts = dt.cpu().numpy()
        parts = batch.split(u.cpu().numpy())
        for b, p in enumerate(probs):
            po = oracle.Problem(dim=1, nvar=p["nvar"], nx=us[b].shape[1], flux=fid, P=p["P"],
                                bc=oracle.BC_PERIODIC if p["bc"] == "periodic" else oracle.BC_TRANSMISSIVE,
                                dx=p["dx"])
            assert dts[b] == oracle.dt_cfl(po, us[b], 0.6)
            us[b] = oracle.step1d(po, us[b], dts[b])["u"]
            assert np.array_equal(parts[b], us[b]), f"problem {b} step {step}"


def test_batched_c4_full_size_sampled_oracle(acat):
    """The full batched workload (256 Euler problems, 1.2 M cells) through
    BatchSolver, as the benchmark runs it (the second step's time steps come
    from the fused reduction): sampled problems (the largest, the smallest,
    and two more at each P) against the oracle's own time steps and steps,
    bitwise."""
    import torch
    w = workloads.batch_1d()
    probs = w["problems"]
    batch = make_batch(acat, probs)
    bs = acat.BatchSolver(batch, concat([p["u"] for p in probs]), w["cfl"])
    Ns = np.array([p["u"].shape[1] for p in probs])
    Ps = np.array([p["P"] for p in probs])
    pick = {int(np.argmax(Ns)), int(np.argmin(Ns))}
    for P in (2, 3, 4):
        pick.update(int(b) for b in np.flatnonzero(Ps == P)[:2])
    pick = sorted(pick)
    us = {b: probs[b]["u"].copy() for b in pick}
    po = {b: oracle.Problem(dim=1, nvar=3, nx=int(Ns[b]), flux=oracle.FLUX_EULER, P=int(Ps[b]),
                            bc=oracle.BC_TRANSMISSIVE if probs[b]["bc"] == "transmissive" else oracle.BC_PERIODIC,
                            dx=probs[b]["dx"]) for b in pick}
    for step in range(2):
        dts = {b: oracle.dt_cfl(po[b], us[b], w["cfl"]) for b in pick}
        if bs.dt_valid:
            got_dt = bs.dt.cpu().numpy()
            for b in pick:
                assert got_dt[b] == dts[b], f"fused time step, problem {b} before step {step}"
        bs.step()
        torch.cuda.synchronize()
        parts = batch.split(bs.u.cpu().numpy())
        for b in pick:
            us[b] = oracle.step1d(po[b], us[b], dts[b])["u"]
            assert np.array_equal(parts[b], us[b]), f"problem {b} (N={Ns[b]}, P={Ps[b]}) step {step}"
    say(f"[batched C4 full size] problems {pick}: 2 steps bitwise equal to the oracle")


@pytest.mark.parametrize("flux", ["euler", "burgers"])
def test_batched_fused_cfl_equals_separate_reduction(acat, flux):
    """acat_step_batched_cfl: the same states as acat_step_batched, and the time
    steps it leaves equal acat_batched_cfl_dt of the new state, over several
    steps (ragged sizes, problems shorter than a wave, periodic and
    transmissive, every P)."""
    import torch
    rng = np.random.default_rng(11)
    sizes = [8, 9, 40, 63, 64, 65, 130, 777, 2049, 16]
    probs = []
    for b, n in enumerate(sizes):
        P = 1 + b % 4
        n = max(n, 2 * max(P, 2))
        if flux == "euler":
            p = workloads.euler_1d(n=n, P=P, stream=(100 + b,))
        else:
            x = np.arange(n) / n
            p = dict(u=(np.sin(2 * np.pi * x + b) - 0.3 * (x > 0.4))[None].copy(), dx=1.0 / n, flux="burgers",
                     P=P, nvar=1)
        p["bc"] = "periodic" if b % 2 else "transmissive"
        p["P"] = P
        probs.append(p)
    batch = make_batch(acat, probs)
    u0 = T(concat([p["u"] for p in probs]))
    cfl = 0.55
    ua, dta = u0.clone(), torch.zeros(batch.nprob, dtype=torch.float64, device="cuda")
    ub, dtb = u0.clone(), torch.zeros_like(dta)
    batch.cfl_dt(ua, cfl, dta)
    for step in range(6):
        batch.cfl_dt(ub, cfl, dtb)
        assert torch.equal(dta, dtb), f"dt before step {step}"
        ua = batch.step_cfl(ua, dta, cfl)
        ub = batch.step(ub, dtb)
        torch.cuda.synchronize()
        assert torch.equal(ua, ub), f"state after step {step}"
    batch.cfl_dt(ub, cfl, dtb)
    assert torch.equal(dta, dtb)
    say(f"[batched fused CFL] {flux}: 6 steps, states and time steps bitwise equal to the separate reduction")


def test_batched_graph_replay_matches_eager(acat):
    import torch
    w = workloads.batch_1d(nprob=32, nmin=64, nmax=2048)
    probs = w["problems"]
    batch = make_batch(acat, probs)
    u0 = concat([p["u"] for p in probs])
    a = acat.BatchSolver(batch, u0, 0.5)
    a.capture(2)
    b = acat.BatchSolver(batch, u0, 0.5)
    b.run(2)
    for rep in range(3):
        a.replay(1)
        b.run(2)
        torch.cuda.synchronize()
        assert np.array_equal(a.u.cpu().numpy(), b.u.cpu().numpy()), f"replay {rep}"


def test_batched_launch_shapes_and_autotuner_keep_results(acat, tmp_path):
    """Every launch shape of the per-order flux kernels gives the same bits;
    the autotuner picks one per order and caches it."""
    import torch
    from paper_2007_01416_amd import autotune
    w = workloads.batch_1d(nprob=32, nmin=256, nmax=2048)
    probs = w["problems"]
    batch = make_batch(acat, probs)
    u = T(concat([p["u"] for p in probs]))
    dt = torch.empty(batch.nprob, dtype=torch.float64, device="cuda")
    batch.cfl_dt(u, w["cfl"], dt)
    ref = batch.step(u, dt)
    for wv in (1, 2, 4):
        for pc in (0, 1, 3):
            batch.set_launch({p: (wv, pc) for p in batch.orders})
            assert torch.equal(batch.step(u, dt), ref), (wv, pc)
    cache = str(tmp_path / "tune.json")
    best = autotune.tune(batch, u, dt, reps=2, cache=cache)
    assert set(best) == set(batch.orders)
    assert torch.equal(batch.step(u, dt), ref)
    again = autotune.tune(batch, u, dt, cache=cache)           # from the cache
    assert {p: v[:2] for p, v in again.items()} == {p: tuple(v[:2]) for p, v in best.items()}
    say(f"[autotune] {best}")


def test_batched_c4_full_run_500_graph_replayed_steps(acat):
    """The whole batched workload run: 256 problems through BatchSolver,
    2 eager steps then 249 replays of a captured 2-step graph (500 steps, the
    time steps of each step reduced inside the previous one).  Sampled
    problems (the largest, the smallest, two at each P) against 500 oracle
    steps from the same initial data with the oracle's own CFL time steps:
    bit for bit (so within 1e-11)."""
    import torch
    w = workloads.batch_1d()
    probs = w["problems"]
    batch = make_batch(acat, probs)
    bs = acat.BatchSolver(batch, concat([p["u"] for p in probs]), w["cfl"])
    bs.capture(2)
    bs.replay(249)
    torch.cuda.synchronize()
    assert bs.nsteps == 500
    parts = batch.split(bs.u.cpu().numpy())
    Ns = np.array([p["u"].shape[1] for p in probs])
    Ps = np.array([p["P"] for p in probs])
    pick = {int(np.argmax(Ns)), int(np.argmin(Ns))}
    for P in (2, 3, 4):
        pick.update(int(b) for b in np.flatnonzero(Ps == P)[:2])
    for b in sorted(pick):
        po = oracle.Problem(dim=1, nvar=3, nx=int(Ns[b]), flux=oracle.FLUX_EULER, P=int(Ps[b]),
                            bc=oracle.BC_TRANSMISSIVE if probs[b]["bc"] == "transmissive" else oracle.BC_PERIODIC,
                            dx=probs[b]["dx"])
        uo, _, nst = oracle.run(po, probs[b]["u"], w["cfl"], nsteps=500, nthreads=16)
        scale = np.abs(uo).max(axis=1)
        err = (np.abs(parts[b] - uo).max(axis=1) / scale).max()
        say(f"[batched C4 500 steps] problem {b} N={Ns[b]} P={Ps[b]}: rel_err={err:.3e} "
            f"bitwise={np.array_equal(parts[b], uo)}")
        assert err <= 1e-11
        assert np.array_equal(parts[b], uo), f"problem {b}"
