"""Benchmark: ACAT FP64 cell-updates/s on the 2D Euler 2048^2 workload (one GPU).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

One step is the whole hot path on the device: max wave speed reduction,
CFL time step, classification (indicators, orders, limiter), the per-class
flux kernels and the conservative update.  The state starts resident in
HBM; W untimed steps run first, then K steps are timed between two device
synchronisations.  Prints one JSON line (see the `roofline` and
`cpu_baseline` objects for the dominant kernel and the CPU oracle).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6      # MI355X FP64 vector: 256 CU x 128 flop/clk x 2.4 GHz
PEAK_HBM_GBS = 8000.0
WORKLOAD = ("2D Euler gamma=1.4, 2048x2048, periodic, ACAT P=3, CFL 0.4, 8 isentropic vortices + "
            "4 axis-aligned contact/shock lines (p jumps U[2,10])")


# the sources the single-problem step kernels are compiled from
STEP_SOURCES = ("acat_step.hip", "step_common.hpp", "physics.hpp", "coeffs.hpp", "acat_internal.hpp")


def kernel_source_digest() -> str:
    h = hashlib.sha256()
    for f in STEP_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2007_01416_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


COUNTER_WINDOW = (2048, 20, 5)     # grid size, timed steps, warm-up steps of the counter runs


def traffic_from_profiles(kernel: str, n: int, steps: int, warmup: int):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    if it was taken on the current kernel source and on the same grid and
    step window (the class mix, and so the bytes per launch, change along
    a run)."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_c3_counters.txt")
    if (n, steps, warmup) != COUNTER_WINDOW or not os.path.exists(path):
        return None
    digest = kernel_source_digest()
    vals = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != digest:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _oracle_step_rate(w, nthreads):
    """cell-updates/s of one oracle step (CFL time step included) of workload w."""
    import numpy as np
    import oracle
    n = w["u"].shape[-1]
    po = oracle.Problem(dim=2, nvar=4, nx=n, ny=n, flux=oracle.FLUX_EULER, P=w["P"], bc=oracle.BC_PERIODIC,
                        dx=w["dx"], dy=w["dy"], gamma=w["gamma"])
    u = np.ascontiguousarray(w["u"])
    t0 = time.perf_counter()
    dt = oracle.dt_cfl(po, u, w["cfl"])
    oracle.step2d(po, u, dt, nthreads=nthreads)
    el = time.perf_counter() - t0
    return n * n / el, el


def cpu_baseline(w, workloads):
    """The oracle, as it stands, on one full step of the same workload with
    every host core this process may run on; beside it, one step of the same
    recipe at 512^2 on one thread and on all of them (the single-thread
    sample, bounded in time)."""
    cores = len(os.sched_getaffinity(0))
    n = w["u"].shape[-1]
    rate, el = _oracle_step_rate(w, cores)
    small = workloads.euler_2d(n=512, P=w["P"])
    r1, e1 = _oracle_step_rate(small, 1)
    rn, en = _oracle_step_rate(small, cores)
    return {"value": rate, "unit": "cell-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"1 full {n}x{n} P={w['P']} step of the same workload from its initial state ({el:.1f} s, "
                      f"{cores} OpenMP threads = all cores of the process's CPU affinity set)",
            "single_thread": {"value": r1, "cores": 1, "seconds": e1, "all_cores_value_same_sample": rn,
                              "sample": "1 step of the same recipe at 512x512 (P=%d) from its initial state" % w["P"]}}


def bench_batched(acat, workloads, steps_batched=500, steps_single=10):
    """256 independent 1D Euler problems: batched graph-replayed steps vs the
    same problems advanced one acat_step per problem."""
    import numpy as np
    import torch
    w = workloads.batch_1d()
    probs = w["problems"]
    batch = acat.Batch([p["u"].shape[1] for p in probs], [p["P"] for p in probs], [p["bc"] for p in probs],
                       [p["dx"] for p in probs], flux="euler", nvar=3)
    u0 = np.concatenate([p["u"] for p in probs], axis=1)
    from paper_2007_01416_amd import autotune
    ut = torch.from_numpy(u0).cuda()
    dtt = torch.empty(batch.nprob, dtype=torch.float64, device="cuda")
    batch.cfl_dt(ut, w["cfl"], dtt)
    best = autotune.tune(batch, ut, dtt, reps=3)
    bs = acat.BatchSolver(batch, u0, w["cfl"])
    bs.capture(2)
    bs.replay(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bs.replay(steps_batched // 2)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    # the same graph-replayed steps with the default launch (every order class
    # in one flux launch: 6 launches per step) and with one flux launch per
    # order class at the default shape (9 launches per step)
    def graph_ms(table):
        batch.set_launch(table)
        bd = acat.BatchSolver(batch, u0, w["cfl"])
        bd.capture(2)
        bd.replay(2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bd.replay(steps_batched // 2)
        torch.cuda.synchronize()
        return time.perf_counter() - t0
    tdef = graph_ms(None)
    tsep = graph_ms({p: (4, 0) for p in batch.orders})
    singles = []
    for p in probs:
        pg = acat.Problem(dim=1, nvar=3, nx=p["u"].shape[1], flux="euler", P=p["P"], bc=p["bc"], dx=p["dx"])
        singles.append(acat.Solver(pg, p["u"], w["cfl"]))
    for s in singles:
        s.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps_single):
        for s in singles:
            s.step()
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    # the same per-problem steps captured into one HIP graph (two steps of every
    # problem per replay, so the ping-pong buffers return to their start):
    # measures the per-instance design without Python launch overhead
    for s in singles:
        s.step()
        s.step()
    torch.cuda.synchronize()
    gi = torch.cuda.CUDAGraph()
    starts = [s.cur for s in singles]
    with torch.cuda.graph(gi):
        for s in singles:
            s.step()
            s.step()
    for s, c in zip(singles, starts):
        s.cur = c
    gi.replay()
    torch.cuda.synchronize()
    reps_g = max(steps_batched // 2, 1)
    t0 = time.perf_counter()
    for _ in range(reps_g):
        gi.replay()
    torch.cuda.synchronize()
    tsg = time.perf_counter() - t0
    steps_single_graph = 2 * reps_g
    # roofline of the dominant per-order flux kernel: a few eager steps with the
    # library's kernel timer and the per-order interface counts of each step
    from paper_2007_01416_amd import flops as F
    batch.set_launch(None if all(v[0] == 0 for v in best.values()) else {p: v[:2] for p, v in best.items()})
    ue = torch.from_numpy(u0).cuda()
    uo = torch.empty_like(ue)
    dte = torch.empty(batch.nprob, dtype=torch.float64, device="cuda")
    counts = batch.ws[:16].view(torch.int32)
    nprof = 20
    hist = torch.zeros((nprof, 4), dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    acat.profile(True)
    for k in range(nprof):
        batch.cfl_dt(ue, w["cfl"], dte)
        batch.step(ue, dte, out=uo)
        hist[k].copy_(counts)
        ue, uo = uo, ue
    prof = acat.profile_read()
    acat.profile(False)
    per_p = hist.cpu().numpy().astype(np.int64).sum(0)
    cf = F.C_F[("euler", 1)]
    if "flux_b_all" in prof:             # the default: every order class in one launch
        dom_name = "flux_b_all"
        dom_launches, dom_ms = prof[dom_name]
        dom_flops = sum(int(per_p[p - 1]) * F.interface_flops_1d(p, 3, cf) for p in batch.orders)
    else:
        kern = {p: prof[f"flux_b_p{p}"] for p in batch.orders if f"flux_b_p{p}" in prof}
        dom = max(kern, key=lambda p: kern[p][1])
        dom_name = f"flux_b_p{dom}"
        dom_launches, dom_ms = kern[dom]
        dom_flops = int(per_p[dom - 1]) * F.interface_flops_1d(dom, 3, cf)
    ach = dom_flops / (dom_ms * 1e-3) / 1e12
    launch_kernels = {k: {"launches": c, "avg_us": round(1e3 * ms / max(c, 1), 2)} for k, (c, ms) in prof.items()}
    cells = batch.ncell
    vb = cells * steps_batched / tb
    vs = cells * steps_single / ts
    return {"workload": f"{batch.nprob} independent 1D Euler problems, N log-uniform in [512,16384] "
                        f"(total {cells} cells), P in {{2,3,4}}, transmissive, per-problem CFL 0.5",
            "value": vb, "unit": "cell-updates/s", "steps": steps_batched, "ms_per_step": 1e3 * tb / steps_batched,
            "per_instance_graph_value": cells * steps_single_graph / tsg,
            "per_instance_graph_ms_per_step": 1e3 * tsg / steps_single_graph,
            "per_instance_graph_steps": steps_single_graph,
            "speedup_vs_per_instance_graph": vb / (cells * steps_single_graph / tsg),
            "per_instance_eager_value": vs, "per_instance_eager_steps": steps_single,
            "per_instance_eager_ms_per_step": 1e3 * ts / steps_single, "speedup_vs_per_instance_eager": vb / vs,
            "autotuned_launch": ("default: every order class in one launch (kept: per-class shapes not "
                                 "2 % faster, graph-replayed)" if all(v[0] == 0 for v in best.values()) else
                                 {f"p{p}": {"waves_per_block": v[0], "blocks_per_cu": v[1],
                                            "kernel_us": round(1e3 * v[2], 2)} for p, v in best.items()}),
            "default_launch_ms_per_step": 1e3 * tdef / steps_batched,
            "per_class_launches_ms_per_step": 1e3 * tsep / steps_batched,
            "launches_per_step": launch_kernels,
            "roofline": {"bound": "alu", "kernel": dom_name, "achieved": ach, "peak": PEAK_FP64_TFLOPS,
                         "unit": "TFLOP/s", "frac": ach / PEAK_FP64_TFLOPS,
                         "avg_launch_us": 1e3 * dom_ms / dom_launches}}


def bench_adjoint(acat, workloads, F, fd_dirs=32, fd_h=(1e-4, 1e-5, 1e-6, 1e-7, 1e-8)):
    """2D Euler 512^2 P=2: gradient of the final-density misfit after 200
    steps w.r.t. the initial state (checkpoint every 20, recomputation),
    timed against the plain 200-step forward; central differences of the
    frozen replay run on seeded smooth directions with an h sweep."""
    import numpy as np
    import torch
    w = workloads.adjoint_2d()
    n = w["u"].shape[-1]
    nsteps, k, cfl = w["nsteps"], w["checkpoint_every"], w["cfl"]
    pg = acat.Problem(dim=2, nvar=4, nx=n, ny=n, flux="euler", P=w["P"], bc="periodic", dx=w["dx"], dy=w["dy"],
                      gamma=w["gamma"])
    u0 = torch.from_numpy(w["u"]).cuda()
    star = acat.AdjointRun(pg, cfl, nsteps, k, verify=False).forward(torch.from_numpy(w["target_u0"]).cuda())[0]
    area = w["dx"] * w["dy"]

    def grad_T(uT):
        g = torch.zeros_like(uT)
        g[0] = area * (uT[0] - star)
        return g

    def loss(u):
        return 0.5 * area * float(((u[0] - star) ** 2).sum())

    # plain forward: the same steps with no checkpoints or recording, graph-replayed
    # in blocks of k steps like the checkpointed forward and the backward
    plain = acat.Solver(pg, w["u"], cfl)
    plain.capture(k)
    plain.replay(1)
    plain = acat.Solver(pg, w["u"], cfl)
    plain.capture(k)
    plain.u.copy_(u0)                            # the capture's warm-up steps moved the state
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain.replay(nsteps // k)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    # checkpointed forward + backward
    run = acat.AdjointRun(pg, cfl, nsteps, k, verify=False)
    run.backward(grad_T(run.forward(u0)))         # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    uT = run.forward(u0)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    gT = grad_T(uT)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    grad = run.backward(gT)
    torch.cuda.synchronize()
    t_bwd = time.perf_counter() - t0
    # every step resident: one segment of nsteps, so the forward keeps each
    # step's state, decisions and class lists and the reverse pass recomputes
    # nothing (HBM held instead of time: reported beside the k-step checkpoints)
    rrun = acat.AdjointRun(pg, cfl, nsteps, nsteps, verify=False)
    rrun.backward(grad_T(rrun.forward(u0)))       # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    uT_r = rrun.forward(u0)
    torch.cuda.synchronize()
    t_fwd_r = time.perf_counter() - t0
    gT_r = grad_T(uT_r)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    grad_r = rrun.backward(gT_r)
    torch.cuda.synchronize()
    t_bwd_r = time.perf_counter() - t0
    resident_bytes = sum(t.numel() * t.element_size() for t in rrun.seg_u + rrun.seg_ws) + sum(
        v.numel() * v.element_size() for d in rrun.seg_dec for v in vars(d).values() if torch.is_tensor(v))
    del rrun
    # kernel durations: the same backward launched eagerly (graph replays are not
    # bracketed by the library's events) on one stream (the timed run overlaps
    # recomputation and adjoint steps on two), with the per-step class counts
    erun = acat.AdjointRun(pg, cfl, nsteps, k, verify=False, graphs=False, overlap=False)
    erun.forward(u0)
    erun.class_log = torch.zeros((nsteps, 16), dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    acat.profile(True)
    erun.backward(gT)
    prof = acat.profile_read()
    acat.profile(False)
    hist = erun.class_log.cpu().numpy().astype(np.int64).sum(0)
    P = w["P"]
    kern = {}
    for name, (c, ms) in prof.items():
        cl = corner_classes(name, "adjoint2d_")
        if cl:
            kern[name] = dict(launches=c, ms=ms, classes=cl,
                              flops=sum(int(hist[(q1 - 1) * P + (q2 - 1)]) * F.adjoint_corner_flops_2d(q1, q2)
                                        for q1, q2 in cl))
    ridge = PEAK_FP64_TFLOPS * 1e12 / (PEAK_HBM_GBS * 1e9)
    per_kernel = {}
    for name, v in kern.items():
        cnt = sum(int(hist[(q1 - 1) * P + (q2 - 1)]) for q1, q2 in v["classes"])
        by = sum(int(hist[(q1 - 1) * P + (q2 - 1)]) * F.adjoint_corner_bytes_2d(q1, q2) for q1, q2 in v["classes"])
        sec = v["ms"] * 1e-3
        intensity = v["flops"] / max(by, 1)
        bound = "alu" if intensity >= ridge else "hbm"
        per_kernel[name] = {"ms": round(v["ms"], 3), "corners": cnt, "flops_per_byte": round(intensity, 2),
                            "bound": bound,
                            "frac": (v["flops"] / sec / 1e12 / PEAK_FP64_TFLOPS) if bound == "alu"
                            else (by / sec / 1e9 / PEAK_HBM_GBS),
                            "alu_frac": v["flops"] / sec / 1e12 / PEAK_FP64_TFLOPS,
                            "hbm_frac": by / sec / 1e9 / PEAK_HBM_GBS}
    dom = max(kern, key=lambda x: kern[x]["ms"])
    achieved = kern[dom]["flops"] / (kern[dom]["ms"] * 1e-3) / 1e12
    dom_alu = max((x for x in kern if per_kernel[x]["bound"] == "alu"), key=lambda x: kern[x]["ms"], default=None)
    # verified run (recomputed order maps and time steps checked) recording every step for the replay map
    vrun = acat.AdjointRun(pg, cfl, nsteps, k, record_all=True, verify=True)
    uT2 = vrun.forward(u0)
    grad2 = vrun.backward(grad_T(uT2))
    deterministic = bool(torch.equal(grad, grad2))
    t0 = time.perf_counter()
    errs, per_h = [float("nan")], {h: [] for h in fd_h}
    for j in range(fd_dirs):
        if j % 8 == 0:
            print(f"[bench] adjoint finite differences: direction {j}/{fd_dirs}", file=sys.stderr, flush=True)
        v = torch.from_numpy(w["directions"](j)).cuda()
        ad = float((grad2 * v).sum())
        rel = []
        for h in fd_h:
            fd = (loss(vrun.replay(u0 + h * v)) - loss(vrun.replay(u0 - h * v))) / (2 * h)
            r = abs(fd - ad) / abs(ad)
            per_h[h].append(r)
            rel.append(r)
        errs.append(min(rel))
    errs = errs[1:] or errs
    t_fd = time.perf_counter() - t0
    return {"workload": f"2D Euler {n}x{n} P={P} periodic, {nsteps} steps, CFL {cfl}, loss 1/2 dx dy sum "
                        f"(rho_T - rho*_T)^2, gradient w.r.t. all of u0, checkpoint every {k}",
            "forward_plain_ms": 1e3 * t_plain, "forward_checkpointed_ms": 1e3 * t_fwd, "backward_ms": 1e3 * t_bwd,
            "adjoint_over_forward": t_bwd / t_plain,
            "all_steps_resident": {"forward_ms": 1e3 * t_fwd_r, "backward_ms": 1e3 * t_bwd_r,
                                   "adjoint_over_forward": t_bwd_r / t_plain, "hbm_bytes": resident_bytes,
                                   "grad_equal_to_checkpointed": bool(torch.equal(grad_r, grad))},
            "roofline": ({"bound": "alu", "kernel": dom, "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                          "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS}
                         if per_kernel[dom]["bound"] == "alu" else
                         {"bound": "hbm", "kernel": dom,
                          "achieved": per_kernel[dom]["hbm_frac"] * PEAK_HBM_GBS, "peak": PEAK_HBM_GBS,
                          "unit": "GB/s", "frac": per_kernel[dom]["hbm_frac"]})
                        | {"avg_launch_us": 1e3 * kern[dom]["ms"] / kern[dom]["launches"],
                           "dominant_alu_bound_kernel": dom_alu,
                           "dominant_alu_bound_frac": per_kernel[dom_alu]["alu_frac"] if dom_alu else None},
            "adjoint_kernels": per_kernel,
            "loss": loss(uT), "grad_deterministic": deterministic,
            "fd_check": {"directions": fd_dirs, "h": list(fd_h), "max_rel_err_best_h": max(errs),
                         "median_rel_err_by_h": {f"{h:.0e}": float(np.median(per_h[h])) if per_h[h] else None
                                                 for h in fd_h},
                         "seconds": t_fd}}


def bench_small(acat, workloads, cpu: bool = True):
    """The two 1D configurations to their final times: the Burgers shock
    (200 cells, P = 2, t = 0.6) and the Euler Riemann problem (4096 cells,
    P = 4, t = 0.2).  GPU: steps to t_final counted on one eager run, then
    the per-step time of a captured 64-step graph (steps past t_final have
    dt = 0 and are not counted) and time to solution = steps x that.
    CPU (with cpu): the oracle's full run of the Burgers case on one thread
    and on every core; the Euler case on every core in full and on one
    thread over its first 50 steps, extrapolated to the full step count."""
    import numpy as np
    import torch
    out = {}
    cores = len(os.sched_getaffinity(0))
    for name, w, kw in (("burgers1d_N200_P2_t0.6", workloads.burgers_1d(), dict(nvar=1, flux="burgers")),
                        ("euler1d_N4096_P4_t0.2", workloads.euler_1d(), dict(nvar=3, flux="euler"))):
        n = w["u"].shape[-1]
        bc = w["bc"]
        prob = acat.Problem(dim=1, nx=n, P=w["P"], bc=bc, dx=w["dx"], gamma=w.get("gamma", 1.4), **kw)
        s = acat.Solver(prob, w["u"], w["cfl"], t_final=w["t_final"])
        nsteps = 0
        while s.time() < w["t_final"]:
            s.step()
            nsteps += 1
        g = acat.Solver(prob, w["u"], w["cfl"], t_final=w["t_final"])
        g.capture(64)
        g.replay(1)
        torch.cuda.synchronize()
        reps = 10
        t0 = time.perf_counter()
        g.replay(reps)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / (reps * 64)
        o = {"steps_to_t_final": nsteps, "graph_ms_per_step": ms, "time_to_solution_ms": nsteps * ms,
             "value": n * nsteps / (nsteps * ms * 1e-3), "unit": "cell-updates/s"}
        if cpu:
            import oracle
            po = oracle.Problem(dim=1, nvar=kw["nvar"], nx=n, flux=oracle.FLUX_BURGERS if kw["flux"] == "burgers"
                                else oracle.FLUX_EULER, P=w["P"], bc=oracle.BC_PERIODIC if bc == "periodic"
                                else oracle.BC_TRANSMISSIVE, dx=w["dx"], gamma=w.get("gamma", 1.4))
            t0 = time.perf_counter()
            _, _, on = oracle.run(po, w["u"], w["cfl"], t_final=w["t_final"], nthreads=cores)
            t_all = time.perf_counter() - t0
            o["oracle_all_cores"] = {"cores": cores, "steps": on, "seconds": t_all, "value": n * on / t_all}
            one_steps = on if n <= 1024 else min(on, 50)
            t0 = time.perf_counter()
            oracle.run(po, w["u"], w["cfl"], nsteps=one_steps, nthreads=1)
            t1 = time.perf_counter() - t0
            o["oracle_one_thread"] = {"cores": 1, "steps_timed": one_steps, "seconds": t1,
                                      "value": n * one_steps / t1,
                                      "time_to_solution_s": t1 * on / one_steps,
                                      "extrapolated": one_steps < on}
        out[name] = o
    return out


def bench_paper(acat, workloads):
    """Cost of ACAT2 / ACAT4 / ACAT6 (P = 1, 2, 3) on the paper's two timed
    experiments, next to the paper's CPU-time ratios (Matlab, Sec. 5.3 and
    Sec. 5.5 tables): the right blast wave (450 points, t = 0.012) and the
    2D Riemann problem of configuration 8 (400 x 400, t = 0.25), each run to
    its final time from a cold state (graph-free time loop)."""
    import torch
    out = {}
    cases = [("blast_right_1d_450", lambda P: workloads.paper_riemann_1d("blast_right", P=P),
              {"ACAT2": 1.0, "ACAT4": 5.88, "ACAT6": 12.46}),
             ("lax_liu_8_2d_400x400", lambda P: workloads.paper_lax_liu(8, n=400, P=P),
              {"ACAT2": 1.0, "ACAT4": 9.98, "ACAT6": 96.91})]
    for name, make, paper in cases:
        res = {}
        for P in (1, 2, 3):
            w = make(P)
            kw = dict(dim=w["dim"], nvar=w["nvar"], nx=w["u"].shape[-1], flux="euler", P=P, bc=w["bc"], dx=w["dx"],
                      gamma=w["gamma"])
            if w["dim"] == 2:
                kw.update(ny=w["u"].shape[1], dy=w["dy"])
            prob = acat.Problem(**kw)
            s = acat.Solver(prob, w["u"], w["cfl"], t_final=w["t_final"])
            s.step()
            s = acat.Solver(prob, w["u"], w["cfl"], t_final=w["t_final"])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.run_to_end(check_every=32)
            torch.cuda.synchronize()
            res[f"ACAT{2 * P}"] = {"ms": 1e3 * (time.perf_counter() - t0), "steps": s.nsteps}
        base = res["ACAT2"]["ms"]
        out[name] = {k: dict(v, ratio=round(v["ms"] / base, 3), paper_ratio=paper[k]) for k, v in res.items()}
    return out


def _class_profile(acat, s, nclass, steps, warmup):
    """Steps a Solver under the kernel profiler; returns (seconds, per-class
    item totals, kernel table)."""
    import numpy as np
    import torch
    for _ in range(warmup):
        s.step()
    counts = s.ws[:64].view(torch.int32)
    hist = torch.zeros((steps, 16), dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    acat.profile(True)
    t0 = time.perf_counter()
    for k in range(steps):
        s.step()
        hist[k].copy_(counts)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = acat.profile_read()
    acat.profile(False)
    return el, hist.cpu().numpy().astype(np.int64)[:, :nclass].sum(0), prof


def bench_high_order(acat, workloads, F, steps=20, warmup=3, n1d=1 << 22, n2d=2048):
    """Orders above the headline's: 1D Euler with P = 5 and 6 (orders 10 and
    12) on the Riemann-plus-sine data, and 2D Euler with P = 4 (order 8,
    corner rectangles up to 8 x 8 nodes) on the vortex-and-band data.  For
    each: cell-updates/s, the order classes selected and each flux kernel's
    share of the FP64 peak under the algorithmic flop count."""
    out = {}
    for P in (5, 6):
        w = workloads.euler_1d(n=n1d, P=P)
        prob = acat.Problem(dim=1, nvar=3, nx=n1d, flux="euler", P=P, bc="transmissive", dx=w["dx"],
                            gamma=w["gamma"])
        s = acat.Solver(prob, w["u"], w["cfl"])
        el, per, prof = _class_profile(acat, s, P, steps, warmup)
        kern = {}
        for p in range(1, P + 1):
            name = f"flux1d_p{p}"
            if name in prof and per[p - 1] > 0:
                c, ms = prof[name]
                fl = per[p - 1] * F.interface_flops_1d(p, 3, F.C_F[("euler", 1)])
                kern[name] = {"avg_us": round(1e3 * ms / c, 2), "items": int(per[p - 1]),
                              "frac": round(fl / (ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS, 4)}
        out[f"euler1d_P{P}_n{n1d}"] = {"value": n1d * steps / el, "unit": "cell-updates/s",
                                       "ms_per_step": 1e3 * el / steps, "kernels": kern,
                                       "device_status": acat.device_status()}
    P = 4
    w = workloads.euler_2d(n=n2d, P=P)
    prob = acat.Problem(dim=2, nvar=4, nx=n2d, ny=n2d, flux="euler", P=P, bc="periodic", dx=w["dx"], dy=w["dy"],
                        gamma=w["gamma"])
    s = acat.Solver(prob, w["u"], w["cfl"])
    el, per, prof = _class_profile(acat, s, P * P, steps, warmup)
    kern = {}
    for name, (c, ms) in prof.items():
        cl = corner_classes(name)
        cnt = sum(int(per[(q1 - 1) * P + (q2 - 1)]) for q1, q2 in cl)
        if cl and cnt > 0:
            fl = sum(int(per[(q1 - 1) * P + (q2 - 1)]) * F.corner_flops_2d(q1, q2) for q1, q2 in cl)
            kern[name] = {"avg_us": round(1e3 * ms / c, 2), "items": cnt,
                          "frac": round(fl / (ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS, 4)}
    out[f"euler2d_P4_{n2d}x{n2d}"] = {"value": n2d * n2d * steps / el, "unit": "cell-updates/s",
                                      "ms_per_step": 1e3 * el / steps, "kernels": kern,
                                      "device_status": acat.device_status()}
    return out


def corner_classes(name, prefix="flux2d_"):
    """Order classes (q1, q2) a 2D corner kernel's profile name covers:
    flux2d_q33 -> [(3, 3)], flux2d_q12q21 -> [(1, 2), (2, 1)]; [] otherwise."""
    if not name.startswith(prefix):
        return []
    tags = name[len(prefix):].split("q")[1:]
    return [(int(t[0]), int(t[1])) for t in tags]


def measured_peaks(acat, reps=5):
    """FP64 FMA rate (acat_fp64_fma_rate: 16 independent FMA chains per lane,
    8 blocks of 256 threads per CU) and HBM copy bandwidth (1 GiB device to
    device copy, read + write bytes), each the best of `reps` launches timed
    with events on the current stream, at the running clock."""
    import torch
    blocks, iters = 256 * 8, 4096
    out = torch.empty(blocks * acat.FMA_THREADS, dtype=torch.float64, device="cuda")
    acat.fp64_fma_rate(out, blocks, 64)
    best_fma = float("inf")
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        flops = acat.fp64_fma_rate(out, blocks, iters)
        b.record()
        torch.cuda.synchronize()
        best_fma = min(best_fma, a.elapsed_time(b) * 1e-3)
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best_copy = float("inf")
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        torch.cuda.synchronize()
        best_copy = min(best_copy, a.elapsed_time(b) * 1e-3)
    finite = bool(torch.isfinite(out).all().item())
    del src, dst
    return {"fp64_fma_tflops": flops / best_fma / 1e12, "hbm_copy_tb_s": 2 * (1 << 30) / best_copy / 1e12,
            "fma_output_finite": finite,
            "method": "best of %d: FMA-chain kernel %d blocks x 256 threads x %d iterations x 16 chains; "
                      "1 GiB device-to-device copy" % (reps, blocks, iters)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the batched and adjoint workloads")
    ap.add_argument("--fd-dirs", type=int, default=32, help="finite-difference directions of the adjoint check")
    ap.add_argument("--only", choices=["batched", "adjoint", "paper", "high", "small"],
                    help="run only that workload and print its object (for profiling runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 1 GiB device-to-device copy (reference dispatch for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        sys.exit("bench.py runs on one GPU only: the library has no multi-GPU path (--gpus must be 1)")

    import numpy as np
    import torch

    import paper_2007_01416_amd as acat
    from paper_2007_01416_amd import flops as F
    import workloads

    acat.load()
    if args.only == "batched":
        print(json.dumps(bench_batched(acat, workloads)), flush=True)
        return
    if args.only == "small":
        print(json.dumps(bench_small(acat, workloads, cpu=not args.no_cpu_baseline)), flush=True)
        return
    if args.only == "paper":
        print(json.dumps(bench_paper(acat, workloads)), flush=True)
        return
    if args.only == "high":
        print(json.dumps(bench_high_order(acat, workloads, F)), flush=True)
        return
    if args.only == "adjoint":
        print(json.dumps(bench_adjoint(acat, workloads, F, fd_dirs=args.fd_dirs)), flush=True)
        return
    w = workloads.euler_2d(n=args.n)
    n = args.n
    prob = acat.Problem(dim=2, nvar=4, nx=n, ny=n, flux="euler", P=w["P"], bc="periodic", dx=w["dx"], dy=w["dy"],
                        gamma=w["gamma"])
    s = acat.Solver(prob, w["u"], w["cfl"])
    for _ in range(args.warmup):
        s.step()
    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    counts = s.ws[:64].view(torch.int32)          # per-class item counts of the last step
    hist = torch.zeros((args.steps, 16), dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    acat.profile(True)
    t0 = time.perf_counter()
    for k in range(args.steps):
        s.step()
        hist[k].copy_(counts)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = acat.profile_read()
    acat.profile(False)
    hist = hist.cpu().numpy().astype(np.int64)
    flags = acat.device_status()
    # the same step window again, captured once into a HIP graph and replayed
    # (no per-launch events, no host launch gaps)
    g = acat.Solver(prob, w["u"], w["cfl"])
    g.run(max(args.warmup - 2, 0))
    g.capture(args.steps if args.steps % 2 == 0 else args.steps + 1)   # its two warm-up steps run eagerly
    gsteps = g.graph_steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.replay(1)
    torch.cuda.synchronize()
    el_graph = time.perf_counter() - t0
    graph_ok = bool(torch.equal(g.u, s.u)) if gsteps == args.steps and args.warmup >= 2 else None

    cells = n * n
    value = cells * args.steps / el
    P = w["P"]
    class_flops = {}      # per corner kernel (one class, or a mirror pair of classes)
    for name in prof:
        cl = corner_classes(name)
        if cl:
            class_flops[name] = sum(int(hist[:, (q1 - 1) * P + (q2 - 1)].sum()) * F.corner_flops_2d(q1, q2)
                                    for q1, q2 in cl)
    kernels = {k: {"launches": c, "avg_us": 1e3 * ms / max(c, 1), "total_ms": ms} for k, (c, ms) in prof.items()}
    dom = max((k for k in kernels if k.startswith("flux2d")), key=lambda k: kernels[k]["total_ms"])
    dom_launches = kernels[dom]["launches"]
    achieved = class_flops[dom] / (kernels[dom]["total_ms"] * 1e-3) / 1e12
    traffic = traffic_from_profiles(dom, n, args.steps, args.warmup)
    alg_total = sum(class_flops.values()) + args.steps * cells * (F.classify_flops(P, 4, 2) + F.update_flops(4, 2))
    kern_ms = sum(v["total_ms"] for v in kernels.values())
    hist_cls = hist[:, :P * P].sum(0)
    peaks = measured_peaks(acat)
    out = {
        "metric": f"ACAT FP64 cell-updates/s, 2D Euler {n}^2",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * el / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded generator, workloads.euler_2d)",
        "config": {"workload": WORKLOAD.replace("2048x2048", f"{n}x{n}"), "nx": n, "ny": n, "P": P, "cfl": w["cfl"],
                   "first_timed_step": args.warmup},
        "roofline": {"bound": "alu", "kernel": dom, "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                     "traffic": traffic,
                     "traffic_window": "2048^2, steps %d-%d (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated); "
                                       "null for another grid or window" % (COUNTER_WINDOW[2],
                                                                            sum(COUNTER_WINDOW[1:]) - 1),
                     "launches": dom_launches,
                     "avg_launch_us": kernels[dom]["avg_us"],
                     "alg_flops_per_launch": class_flops[dom] / max(dom_launches, 1),
                     "frac_of_measured_fp64": achieved / peaks["fp64_fma_tflops"]},
        "graph_replayed": {"value": cells * gsteps / el_graph, "unit": "cell-updates/s",
                           "ms_per_step": 1e3 * el_graph / gsteps, "steps": gsteps,
                           "first_step": max(args.warmup - 2, 0) + 2, "same_final_state_as_eager": graph_ok,
                           "note": "the timed window replayed from one captured HIP graph, without the "
                                   "library's per-launch event timer"},
        "measured_peaks": peaks,
        "step_alg_tflops": alg_total / el / 1e12,
        "kernel_time_fraction": kern_ms / (1e3 * el),
        "order_classes": {f"q{q1}{q2}": int(hist_cls[(q1 - 1) * P + (q2 - 1)]) for q1 in range(1, P + 1)
                          for q2 in range(1, P + 1)},
        "kernels": {k: {"launches": v["launches"], "avg_us": round(v["avg_us"], 2)} for k, v in kernels.items()},
        "device_status": flags,
    }
    if not args.no_extra:
        print("[bench] batched 1D workload", file=sys.stderr, flush=True)
        out["batched"] = bench_batched(acat, workloads)
        print("[bench] 1D configurations to their final times", file=sys.stderr, flush=True)
        out["small_configs"] = bench_small(acat, workloads, cpu=not args.no_cpu_baseline)
        print("[bench] paper experiments", file=sys.stderr, flush=True)
        out["paper_cost_ratios"] = bench_paper(acat, workloads)
        print("[bench] higher orders", file=sys.stderr, flush=True)
        out["high_order"] = bench_high_order(acat, workloads, F)
        print("[bench] adjoint workload", file=sys.stderr, flush=True)
        out["adjoint"] = bench_adjoint(acat, workloads, F, fd_dirs=args.fd_dirs)
    if not args.no_cpu_baseline:
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, workloads)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
