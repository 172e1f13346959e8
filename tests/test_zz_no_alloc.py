"""acat_step_noalloc (the allocation-free step: the library's static
per-device workspace) against acat_step with a caller workspace, through the
C ABI: the same kernels, so states and decisions agree bit for bit.  Two
calls in a row, the second on a smaller problem, so the second call runs on
the array the first one left behind."""
import sys

import numpy as np
import pytest

import workloads
from gpu_helpers import from_workload

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def T(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def N(t):
    return t.detach().cpu().numpy()


def _compare(acat, pg, u0, dt, label):
    import torch
    u = T(u0)
    dec_a, dec_b = acat.Decisions(pg), acat.Decisions(pg)
    ref = acat.step(pg, u, dt, dec=dec_a)
    out = torch.full_like(u, float("nan"))
    acat.step_noalloc(pg, u, dt, out, dec=dec_b)
    torch.cuda.synchronize()
    same = torch.equal(ref, out)
    same_dec = all(torch.equal(a, b) for a, b in zip(dec_a.tensors(), dec_b.tensors()) if a is not None)
    say(f"[noalloc {label}] state bitwise={same} decisions bitwise={same_dec}")
    assert same, label
    assert same_dec, label


@pytest.mark.parametrize("dim", [1, 2])
def test_noalloc_matches_step_twice_second_smaller(acat, dim):
    import oracle
    if dim == 1:
        cases = [(workloads.euler_1d(n=4096, P=4), {}), (workloads.euler_1d(n=1000, P=2), dict(bc="periodic"))]
    else:
        cases = [(workloads.euler_2d(n=256, P=3), {}), (workloads.euler_2d(n=96, P=2), dict(bc="transmissive"))]
    for w, over in cases:
        po, pg = from_workload(w, **over)
        dt = oracle.dt_cfl(po, w["u"], w["cfl"])
        _compare(acat, pg, w["u"], dt, f"{dim}D {w['u'].shape} {over}")


def test_noalloc_device_dt_and_size_limit(acat):
    import torch
    w = workloads.euler_2d(n=128, P=3)
    po, pg = from_workload(w)
    sm = acat.max_wave_speed(pg, T(w["u"]))
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    acat.cfl_dt(pg, sm, w["cfl"], dt)
    _compare(acat, pg, w["u"], dt, "2D 128^2 device dt")
    # a problem whose workspace exceeds the static array is rejected before any launch
    big = acat.Problem(dim=2, nvar=4, nx=2048, ny=2048, flux="euler", P=3, bc="periodic", dx=0.01, dy=0.01)
    assert acat.workspace_bytes(big) > acat.NOALLOC_SCRATCH_BYTES
    u = torch.zeros(big.shape, dtype=torch.float64, device="cuda")
    with pytest.raises(acat.AcatError) as e:
        acat.step_noalloc(big, u, 1e-3, torch.empty_like(u))
    assert e.value.code == -6
