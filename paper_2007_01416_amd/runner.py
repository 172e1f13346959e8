"""Time loop around the ACAT step: device-side CFL time step, ping-pong state
buffers, and HIP-graph capture of several steps.

Each step is: acat_max_wave_speed -> acat_cfl_dt (dt and t stay on the
device) -> acat_step.  Nothing synchronises with the host, so a block of
steps can be captured once into a HIP graph (torch.cuda.CUDAGraph drives
hipStreamBeginCapture on its capture stream) and replayed.
"""
from __future__ import annotations

import torch

from . import (Batch, Decisions, Problem, cfl_dt, max_wave_speed, step, step_replay, workspace)


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
        max_wave_speed(p, self.u, self.smax)
        cfl_dt(p, self.smax, self.cfl, self.dt, self.t, self.t_final)
        out = self.buf[1 - self.cur]
        if replay:
            step_replay(p, self.u, self.dt, dec, out=out, ws=self.ws)
        else:
            step(p, self.u, self.dt, out=out, ws=self.ws, dec=dec)
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
    and one batched step; `capture(k)` records k steps into one HIP graph."""

    def __init__(self, batch: Batch, u0, cfl: float, device="cuda"):
        self.batch = batch
        self.cfl = float(cfl)
        u0 = torch.as_tensor(u0, dtype=torch.float64, device=device).contiguous()
        if tuple(u0.shape) != batch.shape:
            raise ValueError(f"initial state {tuple(u0.shape)} != {batch.shape}")
        self.buf = [u0.clone(), torch.empty_like(u0)]
        self.cur = 0
        self.dt = torch.zeros(batch.nprob, dtype=torch.float64, device=device)
        self.nsteps = 0
        self.graph = None
        self.graph_steps = 0

    @property
    def u(self) -> torch.Tensor:
        return self.buf[self.cur]

    def step(self):
        self.batch.cfl_dt(self.u, self.cfl, self.dt)
        self.batch.step(self.u, self.dt, out=self.buf[1 - self.cur])
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
