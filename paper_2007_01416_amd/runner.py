"""Time loop around the ACAT step: device-side CFL time step, ping-pong state
buffers, and HIP-graph capture of several steps.

Each step is: acat_max_wave_speed -> acat_cfl_dt (dt and t stay on the
device) -> acat_step.  Nothing synchronises with the host, so a block of
steps can be captured once into a HIP graph (torch.cuda.CUDAGraph drives
hipStreamBeginCapture on its capture stream) and replayed.

AdjointRun / ACATRun: gradients of a function of the final state of an
n-step run with respect to the initial state, through acat_step_adjoint,
with the decisions of every step (orders, psi^1, alpha) and its time step
frozen at the forward run's values.  The forward keeps a state checkpoint
every k steps; the backward recomputes each k-step segment from its
checkpoint (recording decisions and time steps) and runs the adjoint steps
of the segment in reverse.  Each recomputed step keeps its own step
workspace, so that its adjoint step reuses the step's order-class lists
(acat_step_adjoint_lists) instead of classifying again.  With
checkpoint_every="auto" the segment is as long as a device-memory budget
allows (every step resident when it fits: no recomputation at all; otherwise
the budget holds the two alternating buffer sets of the overlapped pass).
"""
from __future__ import annotations

import torch

from . import (Batch, Decisions, Problem, adjoint_workspace, cfl_dt, max_wave_speed, step, step_adjoint_lists,
               step_cfl, step_replay, workspace, workspace_bytes)


class Solver:
    def __init__(self, prob: Problem, u0, cfl: float, t_final: float = float("inf"), device="cuda"):
        self.prob = prob
        self.cfl = float(cfl)
        self.t_final = float(t_final)
        u0 = torch.as_tensor(u0, dtype=torch.float64, device=device).contiguous()
        if tuple(u0.shape) != prob.shape:
            raise ValueError(f"initial state {tuple(u0.shape)} != {prob.shape}")
        self.buf = [u0.clone(), torch.empty_like(u0)]
        self.cur = 0
        self.ws = workspace(prob, device)
        self.smax = torch.zeros(2, dtype=torch.float64, device=device)
        self.dt = torch.zeros(1, dtype=torch.float64, device=device)
        self.t = torch.zeros(1, dtype=torch.float64, device=device)
        self.nsteps = 0
        self.graph = None
        self.graph_steps = 0

    @property
    def u(self) -> torch.Tensor:
        return self.buf[self.cur]

    def time(self) -> float:
        return float(self.t.item())

    def step(self, dec: Decisions = None, replay: bool = False):
        """One CFL step (dt from the current state, clipped at t_final)."""
        p = self.prob
        out = self.buf[1 - self.cur]
        if replay:
            max_wave_speed(p, self.u, self.smax)
            cfl_dt(p, self.smax, self.cfl, self.dt, self.t, self.t_final)
            step_replay(p, self.u, self.dt, dec, out=out, ws=self.ws)
        else:
            step_cfl(p, self.u, self.cfl, self.dt, self.t, self.t_final, out=out, ws=self.ws, dec=dec)
        self.cur ^= 1
        self.nsteps += 1

    def run(self, nsteps: int):
        for _ in range(nsteps):
            self.step()
        return self.u

    def run_to_end(self, check_every: int = 64, max_steps: int = 10 ** 7):
        """Advance until t reaches t_final (host checks t every few steps)."""
        while self.nsteps < max_steps:
            for _ in range(check_every):
                self.step()
            if self.time() >= self.t_final:
                break
        return self.u

    # ------------------------------------------------------------ graphs
    def capture(self, nsteps: int):
        """Capture nsteps (even) steps into one HIP graph."""
        if nsteps % 2:
            raise ValueError("capture an even number of steps (ping-pong buffers)")
        self.step()   # warm-up outside capture (kernels loaded)
        self.step()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        start = self.cur
        with torch.cuda.graph(g):
            for _ in range(nsteps):
                self.step()
        self.cur = start
        self.nsteps -= nsteps
        self.graph, self.graph_steps = g, nsteps
        return g

    def replay(self, times: int = 1):
        for _ in range(times):
            self.graph.replay()
            self.nsteps += self.graph_steps
        return self.u


class BatchSolver:
    """Fixed-step time loop of a Batch: per step, per-problem CFL time steps
    and one batched step; `capture(k)` records k steps into one HIP graph.
    After the first step the time steps of step n+1 are reduced inside step n
    (acat_step_batched_cfl)."""

    def __init__(self, batch: Batch, u0, cfl: float, device="cuda"):
        self.batch = batch
        self.cfl = float(cfl)
        u0 = torch.as_tensor(u0, dtype=torch.float64, device=device).contiguous()
        if tuple(u0.shape) != batch.shape:
            raise ValueError(f"initial state {tuple(u0.shape)} != {batch.shape}")
        self.buf = [u0.clone(), torch.empty_like(u0)]
        self.cur = 0
        self.dt = torch.zeros(batch.nprob, dtype=torch.float64, device=device)
        self.dt_valid = False   # dt holds the CFL time steps of the current state
        self.nsteps = 0
        self.graph = None
        self.graph_steps = 0

    @property
    def u(self) -> torch.Tensor:
        return self.buf[self.cur]

    def step(self):
        if not self.dt_valid:
            self.batch.cfl_dt(self.u, self.cfl, self.dt)
            self.dt_valid = True
        self.batch.step_cfl(self.u, self.dt, self.cfl, out=self.buf[1 - self.cur])
        self.cur ^= 1
        self.nsteps += 1

    def run(self, nsteps: int):
        for _ in range(nsteps):
            self.step()
        return self.u

    def capture(self, nsteps: int = 2):
        if nsteps % 2:
            raise ValueError("capture an even number of steps (ping-pong buffers)")
        self.step()
        self.step()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        start = self.cur
        with torch.cuda.graph(g):
            for _ in range(nsteps):
                self.step()
        self.cur = start
        self.nsteps -= nsteps
        self.graph, self.graph_steps = g, nsteps
        return g

    def replay(self, times: int = 1):
        for _ in range(times):
            self.graph.replay()
            self.nsteps += self.graph_steps
        return self.u


def _order_hash(dec: Decisions) -> torch.Tensor:
    """Device checksum of a step's order maps (position-weighted sum)."""
    h = None
    for t in (dec.order_x, dec.order_y):
        if t is None:
            continue
        v = t.reshape(-1).to(torch.int64)
        w = torch.arange(1, v.numel() + 1, device=v.device, dtype=torch.int64) % 8191 + 1
        s = (v * w).sum()
        h = s if h is None else h * 1000003 + s
    return h


def resident_bytes_per_step(prob: Problem) -> int:
    """Device bytes one step of a recomputed segment holds: its input state,
    its step workspace (order-class lists) and its decisions."""
    def numel(shape):
        n = 1
        for d in (shape if isinstance(shape, tuple) else (shape,)):
            n *= d
        return n
    nif = sum(numel(s) for s in prob.interfaces if s is not None)
    return 8 * numel(tuple(prob.shape)) + workspace_bytes(prob) + nif * (1 + 8 + 8)


def auto_checkpoint(nsteps: int, per_step: int, budget: int) -> int:
    """Longest segment (steps between checkpoints) whose resident steps fit
    in `budget` bytes: nsteps when the whole run fits, at least 1."""
    if nsteps < 1 or per_step < 1:
        raise ValueError("nsteps and per_step must be >= 1")
    return int(max(1, min(nsteps, budget // per_step)))


class _Segment:
    """Buffers of one recomputed segment of up to k steps: every step's input
    state, decisions, time step, step workspace (class lists) and class
    counts, and a sink for the segment's last output."""

    def __init__(self, prob: Problem, k: int, device):
        shape = prob.shape
        self.dt = torch.zeros(k, dtype=torch.float64, device=device)
        self.dec = [Decisions(prob, device) for _ in range(k)]
        self.u = [torch.empty(shape, dtype=torch.float64, device=device) for _ in range(k)]
        self.ws = [workspace(prob, device) for _ in range(k)]
        self.cls = torch.zeros((k, 16), dtype=torch.int32, device=device)
        self.tmp = torch.empty(shape, dtype=torch.float64, device=device)


class AdjointRun:
    """n CFL steps of one problem with a reverse pass.

    forward(u0) -> u_n keeps u every `checkpoint_every` steps (and, with
    record_all, the decisions of every step for replay()).  backward(ubar_n)
    -> ubar_0 = (d u_n / d u0)^T ubar_n with the decisions and time steps of
    the forward run frozen; segments are recomputed from their checkpoints.
    The forward runs its last segment into the recomputation buffers (states,
    decisions, class lists of every step), so the first segment of the
    reverse pass needs no recomputation (without record_all).  With overlap
    (the default; more than one segment), two sets of segment buffers
    alternate: the recomputation of segment s - 1 runs on a second stream
    (default priority) while the adjoint steps of segment s run on the
    caller's stream; the results are those of the serial pass, bit for bit.  With verify, the order
    maps and time steps of the recomputation are checked against the forward
    pass.  With graphs, each segment (k forward steps; k recomputed steps; k
    adjoint steps) is captured once per buffer set into a HIP graph on fixed
    buffers and replayed per segment.
    """

    def __init__(self, prob: Problem, cfl: float, nsteps: int, checkpoint_every=20,
                 record_all: bool = False, verify: bool = True, graphs: bool = True, device="cuda",
                 memory_budget: int = None, overlap: bool = True):
        if checkpoint_every == "auto":
            # default budget: half of the device memory free now
            budget = memory_budget if memory_budget is not None else torch.cuda.mem_get_info(device)[0] // 2
            per = resident_bytes_per_step(prob)
            checkpoint_every = auto_checkpoint(int(nsteps), per, int(budget))
            if checkpoint_every < nsteps and overlap:   # two buffer sets alternate
                checkpoint_every = auto_checkpoint(int(nsteps), 2 * per, int(budget))
        if nsteps < 1 or checkpoint_every < 1:
            raise ValueError("nsteps and checkpoint_every must be >= 1")
        self.prob, self.cfl, self.nsteps, self.k = prob, float(cfl), int(nsteps), int(checkpoint_every)
        self.device = device
        k = min(self.k, self.nsteps)
        shape = prob.shape
        self.ws = workspace(prob, device)
        self.aws = adjoint_workspace(prob, device)
        self.dts = torch.zeros(self.nsteps, dtype=torch.float64, device=device)
        nseg = (self.nsteps + self.k - 1) // self.k
        self.overlap = bool(overlap) and nseg > 1
        self.segs = [_Segment(prob, k, device) for _ in range(2 if self.overlap else 1)]
        seg = self.segs[0]
        self.seg_dt, self.seg_dec, self.seg_u, self.seg_ws, self.seg_cls = seg.dt, seg.dec, seg.u, seg.ws, seg.cls
        self.side = torch.cuda.Stream(device=device) if self.overlap else None   # default priority
        self.fa = torch.empty(shape, dtype=torch.float64, device=device)    # forward state at segment bounds
        self.fb = torch.empty(shape, dtype=torch.float64, device=device)
        self.ub = torch.empty(shape, dtype=torch.float64, device=device)    # adjoint state
        self.record_all = record_all
        self.all_dec = [Decisions(prob, device) for _ in range(self.nsteps)] if record_all else None
        self.verify = verify
        self.graphs = graphs
        self._fgraphs, self._bgraphs = {}, {}
        self.hashes = torch.zeros(self.nsteps, dtype=torch.int64, device=device) if verify else None
        self.checkpoints = []
        self.resident = None    # segment whose steps the first buffer set holds
        # optional int32 [nsteps, 16]: per-class item counts of each adjoint step
        # (entries (q1 - 1) P + (q2 - 1); the later entries of a row are not defined)
        self.class_log = None

    # ------------------------------------------------------------ segments
    def _fwd_body(self, m, decs):
        a, b = self.fa, self.fb
        for j in range(m):
            step_cfl(self.prob, a, self.cfl, self.seg_dt[j:j + 1], out=b, ws=self.ws, dec=decs[j])
            a, b = b, a
        if a is not self.fa:
            self.fa.copy_(a)

    def _rec_body(self, m, b=0):
        """The segment's m steps from u[0] of buffer set b, keeping every
        step's input state, decisions and class lists."""
        sg = self.segs[b]
        for j in range(m):
            out = sg.u[j + 1] if j + 1 < m else sg.tmp
            step_cfl(self.prob, sg.u[j], self.cfl, sg.dt[j:j + 1], out=out, ws=sg.ws[j], dec=sg.dec[j])

    def _adj_body(self, m, b=0):
        sg = self.segs[b]
        for j in reversed(range(m)):
            step_adjoint_lists(self.prob, sg.u[j], sg.dt[j:j + 1], sg.dec[j], self.ub, sg.ws[j],
                               ubar_in=self.ub, ws=self.aws)
            sg.cls[j].copy_(sg.ws[j][:64].view(torch.int32))

    def _bwd_body(self, m):
        self._rec_body(m)
        self._adj_body(m)

    def _run(self, cache, key, body):
        """Run body() once; with graphs, the first run of a key (segment kind,
        buffer set and length) is eager and is followed by a capture that
        later runs of that key replay (on the current stream)."""
        if not self.graphs:
            body()
        elif key in cache:
            cache[key].replay()
        else:
            body()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                body()
            cache[key] = g

    def forward(self, u0: torch.Tensor) -> torch.Tensor:
        self.fa.copy_(torch.as_tensor(u0, dtype=torch.float64, device=self.device))
        self.checkpoints = []
        self.resident = None
        last = (self.nsteps - 1) // self.k
        for s, n0 in enumerate(range(0, self.nsteps, self.k)):
            m = min(self.k, self.nsteps - n0)
            self.checkpoints.append(self.fa.clone())
            if self.record_all:       # every step's decisions kept: eager, into their own buffers
                self._fwd_body(m, self.all_dec[n0:n0 + m])
            elif s == last:           # into the recomputation buffers, kept for backward
                self.seg_u[0].copy_(self.fa)
                self._run(self._fgraphs, ("rec", 0, m), lambda: self._rec_body(m))
                self.fa.copy_(self.segs[0].tmp)
                self.resident = s
            else:
                decs = self.seg_dec if self.verify else [None] * m
                self._run(self._fgraphs, m, lambda: self._fwd_body(m, decs))
            self.dts[n0:n0 + m].copy_(self.seg_dt[:m])
            if self.verify:
                for j in range(m):
                    d = self.all_dec[n0 + j] if self.record_all else self.seg_dec[j]
                    self.hashes[n0 + j] = _order_hash(d)
        return self.fa.clone()

    def replay(self, u0: torch.Tensor) -> torch.Tensor:
        """The frozen forward map (decisions and time steps of the last
        forward run); needs record_all."""
        if not self.record_all:
            raise RuntimeError("replay needs record_all=True")
        u = torch.as_tensor(u0, dtype=torch.float64, device=self.device).contiguous().clone()
        nxt = torch.empty_like(u)
        for n in range(self.nsteps):
            step_replay(self.prob, u, self.dts[n:n + 1], self.all_dec[n], out=nxt, ws=self.ws)
            u, nxt = nxt, u
        return u

    def _record(self, s, b, dts, hashes):
        """Bookkeeping of segment s held in buffer set b (on the current stream)."""
        n0 = s * self.k
        m = min(self.k, self.nsteps - n0)
        sg = self.segs[b]
        dts[n0:n0 + m].copy_(sg.dt[:m])
        if self.class_log is not None:
            self.class_log[n0:n0 + m].copy_(sg.cls[:m])
        if self.verify:
            for j in range(m):
                hashes[n0 + j] = _order_hash(sg.dec[j])

    def _seg_len(self, s):
        return min(self.k, self.nsteps - s * self.k)

    def backward(self, ubar: torch.Tensor) -> torch.Tensor:
        if not self.checkpoints:
            raise RuntimeError("backward before forward")
        self.ub.copy_(torch.as_tensor(ubar, dtype=torch.float64, device=self.device))
        dts = torch.zeros(self.nsteps, dtype=torch.float64, device=self.device)
        hashes = torch.zeros_like(self.hashes) if self.verify else None
        if self.overlap:
            self._backward_overlapped(dts, hashes)
        else:
            for s in reversed(range(len(self.checkpoints))):
                m = self._seg_len(s)
                if s == self.resident:
                    self._run(self._bgraphs, ("adj", 0, m), lambda: self._adj_body(m))
                else:
                    self.seg_u[0].copy_(self.checkpoints[s])
                    self._run(self._bgraphs, m, lambda: self._bwd_body(m))
                    self.resident = s
                self._record(s, 0, dts, hashes)
        if self.verify:
            if not torch.equal(hashes, self.hashes) or not torch.equal(dts, self.dts):
                raise RuntimeError("recomputed decisions differ from the forward run")
        return self.ub.clone()

    def _backward_overlapped(self, dts, hashes):
        """Segments in reverse; segment s - 1 is recomputed on the side stream
        into the other buffer set while the adjoint steps of segment s run on
        the caller's stream.  Events order each buffer set's reuse: a
        recomputation waits for the adjoint steps that last read its set, the
        adjoint steps wait for the recomputation that filled theirs."""
        main, side = torch.cuda.current_stream(self.device), self.side
        nseg = len(self.checkpoints)
        rec_done = [torch.cuda.Event() for _ in range(2)]
        adj_done = [torch.cuda.Event() for _ in range(2)]
        for e in adj_done:
            e.record(main)
        side.wait_stream(main)        # the checkpoints and ubar are ready
        b = 0
        if self.resident != nseg - 1:  # the last segment recomputed first, on the caller's stream
            m = self._seg_len(nseg - 1)
            self.segs[0].u[0].copy_(self.checkpoints[nseg - 1])
            self._run(self._bgraphs, ("rec", 0, m), lambda: self._rec_body(m, 0))
        for s in reversed(range(nseg)):
            nb = 1 - b
            if s > 0:
                mp = self._seg_len(s - 1)
                side.wait_event(adj_done[nb])
                with torch.cuda.stream(side):
                    self.segs[nb].u[0].copy_(self.checkpoints[s - 1])
                    self._run(self._bgraphs, ("rec", nb, mp), lambda: self._rec_body(mp, nb))
                    rec_done[nb].record(side)
            m = self._seg_len(s)
            self._run(self._bgraphs, ("adj", b, m), lambda: self._adj_body(m, b))
            self._record(s, b, dts, hashes)
            adj_done[b].record(main)
            if s > 0:
                main.wait_event(rec_done[nb])
            b = nb
        self.resident = None      # the buffer sets now hold segments 0 and 1 in no fixed order


class ACATRun(torch.autograd.Function):
    """u_n = ACATRun.apply(u0, run): the n-step forward of an AdjointRun, with
    its checkpointed adjoint as the backward."""

    @staticmethod
    def forward(ctx, u0, run: AdjointRun):
        ctx.run = run
        return run.forward(u0.detach())

    @staticmethod
    def backward(ctx, grad_out):
        return ctx.run.backward(grad_out.contiguous()), None
