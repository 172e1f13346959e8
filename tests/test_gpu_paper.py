"""The paper's experiments (Sec. 5) on the GPU: full runs to the paper's
final times, bit for bit against the oracle."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_helpers import from_workload

pytestmark = pytest.mark.gpu


def run_both(acat, w, nthreads=8, **over):
    po, pg = from_workload(w, **over)
    uo, t, n = oracle.run(po, w["u"], w["cfl"], t_final=w["t_final"], nthreads=nthreads)
    s = acat.Solver(pg, w["u"], w["cfl"], t_final=w["t_final"])
    s.run_to_end(check_every=16)
    ug = s.u.cpu().numpy()
    print(f"[paper] {w.get('name', '')} steps oracle={n} t={s.time()} bitwise={np.array_equal(ug, uo)}", flush=True)
    return ug, uo, s.time(), t


@pytest.mark.parametrize("name", list(workloads.RIEMANN_1D))
@pytest.mark.parametrize("P", [1, 2, 3])
def test_shock_tubes_bitwise(acat, name, P):
    w = workloads.paper_riemann_1d(name, P=P)
    ug, uo, tg, to = run_both(acat, w)
    assert tg == to and np.array_equal(ug, uo)


@pytest.mark.parametrize("name", ["transport_sine", "transport_square", "burgers_sine"])
def test_scalar_problems_bitwise(acat, name):
    w = workloads.paper_scalar_1d(name, P=3)
    ug, uo, tg, to = run_both(acat, w, ax=1.0)
    assert tg == to and np.array_equal(ug, uo)


@pytest.mark.parametrize("config", [4, 6, 8])
def test_lax_liu_bitwise(acat, config):
    w = workloads.paper_lax_liu(config, n=100, P=2)
    ug, uo, tg, to = run_both(acat, w, nthreads=16)
    assert tg == to and np.array_equal(ug, uo)


def test_transport_2d_bitwise(acat):
    w = workloads.paper_transport_2d(n=100, P=2)
    ug, uo, tg, to = run_both(acat, w, nthreads=16, ax=1.0, ay=1.0)
    assert tg == to and np.array_equal(ug, uo)
