"""MI355X-native ACAT (arXiv:2007.01416): Python binding of libacat.so.

The binding only marshals arguments: every step of the method runs in the
HIP kernels behind the C ABI of ``include/acat.h``.  PyTorch provides device
memory and streams.  If the built library is missing, ``load()`` raises: there
is no CPU fallback.

Build first:  python -m paper_2007_01416_amd.build
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libacat.so")

FLUX = {"advection": 0, "burgers": 1, "euler": 2}
BC = {"periodic": 0, "transmissive": 1}
STATUS = {0: "ok", -1: "null", -2: "arg", -3: "alias", -4: "unsupported", -5: "device", -6: "workspace"}
DEV_NONFINITE, DEV_NONPHYSICAL = 1, 2


# variants (Problem.flags), as ACAT_FLAG_* in acat.h
FLAG_FLO_LF, FLAG_FLO_HLL, FLAG_PSI2_MODIFIED, FLAG_PSI1_ROE, FLAG_SQUARE_2D = 1, 2, 4, 8, 16


class AcatError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        super().__init__(f"{what}: acat status {code} ({STATUS.get(code, '?')})")


class _Problem(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("nvar", ctypes.c_int32),
                ("nx", ctypes.c_int64), ("ny", ctypes.c_int64),
                ("flux", ctypes.c_int32), ("P", ctypes.c_int32), ("bc", ctypes.c_int32),
                ("flags", ctypes.c_int32),
                ("gamma", ctypes.c_double), ("ax", ctypes.c_double), ("ay", ctypes.c_double),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double),
                ("eps", ctypes.c_double), ("theta", ctypes.c_double)]


class _Decisions(ctypes.Structure):
    _fields_ = [("order_x", ctypes.c_void_p), ("psi1_x", ctypes.c_void_p), ("alpha_x", ctypes.c_void_p),
                ("order_y", ctypes.c_void_p), ("psi1_y", ctypes.c_void_p), ("alpha_y", ctypes.c_void_p)]


_lib = None

_SIGS = {
    "acat_workspace_size": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)],
    "acat_step": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p,
                  ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p],
    "acat_step_noalloc": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p,
                          ctypes.c_void_p, ctypes.c_void_p],
    "acat_step_replay": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p,
                         ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p],
    "acat_step_cfl": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_double,
                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                      ctypes.c_void_p],
    "acat_adjoint_workspace_size": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)],
    "acat_step_adjoint": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p],
    "acat_step_adjoint_lists": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p,
                                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p],
    "acat_max_wave_speed": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
    "acat_cfl_dt": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_void_p,
                    ctypes.c_void_p, ctypes.c_void_p],
    "acat_device_status": [ctypes.POINTER(ctypes.c_int32), ctypes.c_void_p],
    "acat_status_string": [ctypes.c_int],
    "acat_coefficients": [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
    "acat_batch_workspace_size": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)],
    "acat_batch_init": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t],
    "acat_step_batched": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                          ctypes.c_size_t, ctypes.c_void_p],
    "acat_step_batched_cfl": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                              ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p],
    "acat_batched_cfl_dt": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
                            ctypes.c_size_t, ctypes.c_void_p],
    "acat_profile_enable": [ctypes.c_int32],
    "acat_fp64_fma_rate": [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p],
    "acat_profile_read": [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                          ctypes.POINTER(ctypes.c_int32)],
}


def load(path: str = LIB_PATH):
    """Load libacat.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"{path} not built: run `python -m paper_2007_01416_amd.build`")
        L = ctypes.CDLL(path)
        for name, args in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.acat_status_string.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(rc, what):
    if rc != 0:
        raise AcatError(rc, what)


@dataclass
class Problem:
    """Host-side problem description (mirrors acat_problem)."""
    dim: int
    nvar: int
    nx: int
    ny: int = 1
    flux: str = "euler"
    P: int = 2
    bc: str = "periodic"
    gamma: float = 1.4
    ax: float = 1.0
    ay: float = 1.0
    dx: float = 1.0
    dy: float = 1.0
    eps: float = 1e-12
    theta: float = 0.5
    flags: int = 0      # FLAG_* variants (0: the default method)
    _c: _Problem = field(default=None, init=False, repr=False)

    def c(self) -> _Problem:
        self._c = _Problem(self.dim, self.nvar, self.nx, self.ny if self.dim == 2 else 1, FLUX[self.flux],
                           self.P, BC[self.bc], self.flags, self.gamma, self.ax, self.ay, self.dx, self.dy, self.eps,
                           self.theta)
        return self._c

    @property
    def shape(self):
        return (self.nvar, self.nx) if self.dim == 1 else (self.nvar, self.ny, self.nx)

    @property
    def interfaces(self):
        ext = 0 if self.bc == "periodic" else 1
        if self.dim == 1:
            return (self.nx + ext,), None
        return (self.ny, self.nx + ext), (self.ny + ext, self.nx)

    @property
    def cells(self):
        return self.nx * (self.ny if self.dim == 2 else 1)


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def workspace_bytes(prob: Problem) -> int:
    n = ctypes.c_size_t(0)
    _check(load().acat_workspace_size(ctypes.byref(prob.c()), ctypes.byref(n)), "acat_workspace_size")
    return n.value


def workspace(prob: Problem, device="cuda") -> torch.Tensor:
    return torch.empty(workspace_bytes(prob), dtype=torch.uint8, device=device)


class Decisions:
    """Device buffers for one step's decisions (order, psi^1, alpha per interface)."""

    def __init__(self, prob: Problem, device="cuda"):
        sx, sy = prob.interfaces
        self.order_x = torch.zeros(sx, dtype=torch.int8, device=device)
        self.psi1_x = torch.zeros(sx, dtype=torch.float64, device=device)
        self.alpha_x = torch.zeros(sx, dtype=torch.float64, device=device)
        if sy is not None:
            self.order_y = torch.zeros(sy, dtype=torch.int8, device=device)
            self.psi1_y = torch.zeros(sy, dtype=torch.float64, device=device)
            self.alpha_y = torch.zeros(sy, dtype=torch.float64, device=device)
        else:
            self.order_y = self.psi1_y = self.alpha_y = None

    def c(self) -> _Decisions:
        self._c = _Decisions(*[t.data_ptr() if t is not None else None for t in
                               (self.order_x, self.psi1_x, self.alpha_x, self.order_y, self.psi1_y, self.alpha_y)])
        return self._c

    def tensors(self):
        return (self.order_x, self.psi1_x, self.alpha_x, self.order_y, self.psi1_y, self.alpha_y)

    def copy_(self, other: "Decisions"):
        for a, b in zip(self.tensors(), other.tensors()):
            if a is not None:
                a.copy_(b)
        return self


def _check_state(prob, t, name):
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != prob.shape:
        raise ValueError(f"{name}: expected contiguous cuda float64 {prob.shape}, got {t.dtype} {tuple(t.shape)}")


def step(prob: Problem, u: torch.Tensor, dt, out: torch.Tensor = None, ws: torch.Tensor = None,
         dec: Decisions = None, stream=None) -> torch.Tensor:
    """One ACAT step on the GPU.  dt: float or a 1-element cuda float64 tensor."""
    _check_state(prob, u, "u")
    out = torch.empty_like(u) if out is None else out
    ws = workspace(prob, u.device) if ws is None else ws
    dtv, dtp = (float(dt), None) if not torch.is_tensor(dt) else (0.0, _ptr(dt))
    dc = ctypes.byref(dec.c()) if dec is not None else None
    _check(load().acat_step(ctypes.byref(prob.c()), _ptr(u), _ptr(out), dtv, dtp, _ptr(ws), ws.numel(), dc,
                            _stream(stream)), "acat_step")
    return out


NOALLOC_SCRATCH_BYTES = 64 << 20   # ACAT_NOALLOC_SCRATCH_BYTES


def step_noalloc(prob: Problem, u: torch.Tensor, dt, out: torch.Tensor, dec: Decisions = None,
                 stream=None) -> torch.Tensor:
    """acat_step with the library's static per-device workspace: the call
    allocates nothing (out is the caller's).  Calls on one device share that
    workspace, so overlapping calls race."""
    _check_state(prob, u, "u")
    _check_state(prob, out, "out")
    dtv, dtp = (float(dt), None) if not torch.is_tensor(dt) else (0.0, _ptr(dt))
    dc = ctypes.byref(dec.c()) if dec is not None else None
    _check(load().acat_step_noalloc(ctypes.byref(prob.c()), _ptr(u), _ptr(out), dtv, dtp, dc, _stream(stream)),
           "acat_step_noalloc")
    return out


def step_cfl(prob: Problem, u: torch.Tensor, cfl: float, dt: torch.Tensor, t: torch.Tensor = None,
             t_final: float = float("inf"), out: torch.Tensor = None, ws: torch.Tensor = None,
             dec: Decisions = None, stream=None) -> torch.Tensor:
    """One ACAT step with its CFL time step computed inside the step (written
    to the 1-element cuda float64 tensor dt; t advanced when given)."""
    _check_state(prob, u, "u")
    out = torch.empty_like(u) if out is None else out
    ws = workspace(prob, u.device) if ws is None else ws
    dc = ctypes.byref(dec.c()) if dec is not None else None
    _check(load().acat_step_cfl(ctypes.byref(prob.c()), _ptr(u), _ptr(out), float(cfl), float(t_final), _ptr(t),
                                _ptr(dt), _ptr(ws), ws.numel(), dc, _stream(stream)), "acat_step_cfl")
    return out


def step_replay(prob: Problem, u: torch.Tensor, dt, dec: Decisions, out: torch.Tensor = None,
                ws: torch.Tensor = None, stream=None) -> torch.Tensor:
    """One ACAT step with frozen decisions."""
    _check_state(prob, u, "u")
    out = torch.empty_like(u) if out is None else out
    ws = workspace(prob, u.device) if ws is None else ws
    dtv, dtp = (float(dt), None) if not torch.is_tensor(dt) else (0.0, _ptr(dt))
    _check(load().acat_step_replay(ctypes.byref(prob.c()), _ptr(u), _ptr(out), dtv, dtp, _ptr(ws), ws.numel(),
                                   ctypes.byref(dec.c()), _stream(stream)), "acat_step_replay")
    return out


def adjoint_workspace_bytes(prob: Problem) -> int:
    n = ctypes.c_size_t(0)
    _check(load().acat_adjoint_workspace_size(ctypes.byref(prob.c()), ctypes.byref(n)),
           "acat_adjoint_workspace_size")
    return n.value


def adjoint_workspace(prob: Problem, device="cuda") -> torch.Tensor:
    return torch.empty(adjoint_workspace_bytes(prob), dtype=torch.uint8, device=device)


def step_adjoint(prob: Problem, u: torch.Tensor, dt, dec: Decisions, ubar_out: torch.Tensor,
                 ubar_in: torch.Tensor = None, ws: torch.Tensor = None, stream=None) -> torch.Tensor:
    """ubar_in = (d step_replay(u) / du)^T ubar_out for the decisions `dec`."""
    _check_state(prob, u, "u")
    _check_state(prob, ubar_out, "ubar_out")
    ubar_in = torch.empty_like(u) if ubar_in is None else ubar_in
    _check_state(prob, ubar_in, "ubar_in")
    ws = adjoint_workspace(prob, u.device) if ws is None else ws
    dtv, dtp = (float(dt), None) if not torch.is_tensor(dt) else (0.0, _ptr(dt))
    _check(load().acat_step_adjoint(ctypes.byref(prob.c()), _ptr(u), dtv, dtp, ctypes.byref(dec.c()),
                                    _ptr(ubar_out), _ptr(ubar_in), _ptr(ws), ws.numel(), _stream(stream)),
           "acat_step_adjoint")
    return ubar_in


def step_adjoint_lists(prob: Problem, u: torch.Tensor, dt, dec: Decisions, ubar_out: torch.Tensor,
                       step_ws: torch.Tensor, ubar_in: torch.Tensor = None, ws: torch.Tensor = None,
                       stream=None) -> torch.Tensor:
    """step_adjoint reusing the class lists that the forward step of u with
    decisions `dec` left in its workspace `step_ws`."""
    _check_state(prob, u, "u")
    _check_state(prob, ubar_out, "ubar_out")
    ubar_in = torch.empty_like(u) if ubar_in is None else ubar_in
    _check_state(prob, ubar_in, "ubar_in")
    ws = adjoint_workspace(prob, u.device) if ws is None else ws
    dtv, dtp = (float(dt), None) if not torch.is_tensor(dt) else (0.0, _ptr(dt))
    _check(load().acat_step_adjoint_lists(ctypes.byref(prob.c()), _ptr(u), dtv, dtp, ctypes.byref(dec.c()),
                                          _ptr(ubar_out), _ptr(ubar_in), _ptr(step_ws), step_ws.numel(),
                                          _ptr(ws), ws.numel(), _stream(stream)),
           "acat_step_adjoint_lists")
    return ubar_in


def max_wave_speed(prob: Problem, u: torch.Tensor, smax: torch.Tensor = None, stream=None) -> torch.Tensor:
    _check_state(prob, u, "u")
    smax = torch.empty(2, dtype=torch.float64, device=u.device) if smax is None else smax
    _check(load().acat_max_wave_speed(ctypes.byref(prob.c()), _ptr(u), _ptr(smax), _stream(stream)),
           "acat_max_wave_speed")
    return smax


def cfl_dt(prob: Problem, smax: torch.Tensor, cfl: float, dt: torch.Tensor, t: torch.Tensor = None,
           t_final: float = float("inf"), stream=None) -> torch.Tensor:
    _check(load().acat_cfl_dt(ctypes.byref(prob.c()), _ptr(smax), cfl, t_final, _ptr(t), _ptr(dt),
                              _stream(stream)), "acat_cfl_dt")
    return dt


def device_status(stream=None) -> int:
    v = ctypes.c_int32(0)
    _check(load().acat_device_status(ctypes.byref(v), _stream(stream)), "acat_device_status")
    return v.value


def coefficients(p: int):
    """The kernels' coefficient tables for half-width p (host numpy arrays)."""
    import numpy as np
    n = 2 * p
    g1 = np.zeros((n, n)); gt = np.zeros((n, n)); eta = np.zeros(n); tau = np.zeros(n)
    f = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    _check(load().acat_coefficients(p, f(g1), f(gt), f(eta), f(tau)), "acat_coefficients")
    return dict(g1=g1, gt=gt, eta=eta, tau=tau)


class _Batch(ctypes.Structure):
    _fields_ = [("nvar", ctypes.c_int32), ("flux", ctypes.c_int32),
                ("gamma", ctypes.c_double), ("ax", ctypes.c_double),
                ("eps", ctypes.c_double), ("theta", ctypes.c_double),
                ("nprob", ctypes.c_int32),
                ("n", ctypes.POINTER(ctypes.c_int64)), ("P", ctypes.POINTER(ctypes.c_int32)),
                ("bc", ctypes.POINTER(ctypes.c_int32)), ("dx", ctypes.POINTER(ctypes.c_double)),
                ("launch", ctypes.POINTER(ctypes.c_int32))]


class Batch:
    """A batch of independent 1D problems advanced together (acat_step_batched).

    States are SoA over the concatenated cells: shape (nvar, sum(n))."""

    def __init__(self, n, P, bc, dx, flux="euler", nvar=3, gamma=1.4, ax=1.0, eps=1e-12, theta=0.5,
                 device="cuda"):
        import numpy as np
        self.n = np.ascontiguousarray(n, dtype=np.int64)
        self.P = np.ascontiguousarray(P, dtype=np.int32)
        self.bc = np.ascontiguousarray([BC[b] if isinstance(b, str) else int(b) for b in bc], dtype=np.int32)
        self.dx = np.ascontiguousarray(dx, dtype=np.float64)
        self.nprob = len(self.n)
        self.nvar = nvar
        self.offsets = np.concatenate([[0], np.cumsum(self.n)])
        self.ncell = int(self.offsets[-1])
        self._c = _Batch(nvar, FLUX[flux], gamma, ax, eps, theta, self.nprob,
                         self.n.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                         self.P.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                         self.bc.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                         self.dx.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), None)
        self._launch = None
        self.launch_table = {}
        nb = ctypes.c_size_t(0)
        _check(load().acat_batch_workspace_size(ctypes.byref(self._c), ctypes.byref(nb)), "acat_batch_workspace_size")
        self.ws = torch.empty(nb.value, dtype=torch.uint8, device=device)
        torch.cuda.synchronize()
        _check(load().acat_batch_init(ctypes.byref(self._c), _ptr(self.ws), self.ws.numel()), "acat_batch_init")

    @property
    def shape(self):
        return (self.nvar, self.ncell)

    @property
    def orders(self):
        return sorted(set(range(1, int(self.P.max()) + 1)))

    def set_launch(self, table=None):
        """Launch shapes of the per-order flux kernels: {p: (waves_per_block,
        blocks_per_cu)} (missing p and None: the defaults 4 waves, occupancy
        limit).  Results do not depend on it."""
        import numpy as np
        if table is None:
            self._launch = None
            self._c.launch = None
        else:
            arr = np.zeros(8, dtype=np.int32)
            for p, (wv, pc) in table.items():
                arr[2 * (p - 1)] = wv
                arr[2 * (p - 1) + 1] = pc
            self._launch = arr
            self._c.launch = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        self.launch_table = dict(table) if table else {}
        nb = ctypes.c_size_t(0)
        _check(load().acat_batch_workspace_size(ctypes.byref(self._c), ctypes.byref(nb)), "acat_batch launch table")

    def split(self, u):
        """Per-problem views of a batched state."""
        return [u[:, self.offsets[b]:self.offsets[b + 1]] for b in range(self.nprob)]

    def step(self, u: torch.Tensor, dt: torch.Tensor, out: torch.Tensor = None, stream=None) -> torch.Tensor:
        out = torch.empty_like(u) if out is None else out
        _check(load().acat_step_batched(ctypes.byref(self._c), _ptr(u), _ptr(out), _ptr(dt), _ptr(self.ws),
                                        self.ws.numel(), _stream(stream)), "acat_step_batched")
        return out

    def step_cfl(self, u: torch.Tensor, dt: torch.Tensor, cfl: float, out: torch.Tensor = None,
                 stream=None) -> torch.Tensor:
        """One step with the time steps in `dt`, after which `dt` holds the CFL
        time steps of the result (as `cfl_dt(out, cfl, dt)` would give)."""
        out = torch.empty_like(u) if out is None else out
        _check(load().acat_step_batched_cfl(ctypes.byref(self._c), _ptr(u), _ptr(out), _ptr(dt), cfl,
                                            _ptr(self.ws), self.ws.numel(), _stream(stream)),
               "acat_step_batched_cfl")
        return out

    def cfl_dt(self, u: torch.Tensor, cfl: float, dt: torch.Tensor, stream=None) -> torch.Tensor:
        _check(load().acat_batched_cfl_dt(ctypes.byref(self._c), _ptr(u), cfl, _ptr(dt), _ptr(self.ws),
                                          self.ws.numel(), _stream(stream)), "acat_batched_cfl_dt")
        return dt


def profile(on: bool = True):
    """Start (clear) or stop the library's kernel timer."""
    _check(load().acat_profile_enable(1 if on else 0), "acat_profile_enable")


FMA_THREADS, FMA_CHAINS = 256, 16


def fp64_fma_rate(out: torch.Tensor, blocks: int, iters: int, stream=None) -> int:
    """Launch the FP64 FMA-chain kernel; returns the flops of the launch
    (the caller times it on the stream)."""
    if out.dtype != torch.float64 or not out.is_cuda or not out.is_contiguous():
        raise ValueError("out must be a contiguous float64 CUDA tensor")
    _check(load().acat_fp64_fma_rate(blocks, iters, out.data_ptr(), out.numel(), _stream(stream)),
           "acat_fp64_fma_rate")
    return 2 * blocks * FMA_THREADS * iters * FMA_CHAINS


def profile_read(max_kernels: int = 64) -> dict:
    """{kernel name: (launches, total ms)} of the launches timed since profile(True)."""
    names = ctypes.create_string_buffer(64 * max_kernels)
    ms = (ctypes.c_double * max_kernels)()
    cnt = (ctypes.c_int64 * max_kernels)()
    n = ctypes.c_int32(0)
    _check(load().acat_profile_read(max_kernels, names, ms, cnt, ctypes.byref(n)), "acat_profile_read")
    out = {}
    for k in range(min(n.value, max_kernels)):
        nm = names.raw[64 * k:64 * (k + 1)].split(b"\0")[0].decode()
        out[nm] = (int(cnt[k]), float(ms[k]))
    return out


from .runner import (ACATRun, AdjointRun, BatchSolver, Solver, auto_checkpoint,  # noqa: E402  (time loops, graphs)
                     resident_bytes_per_step)
