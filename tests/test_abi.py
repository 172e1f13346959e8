"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/acat.h declares, rejects invalid arguments before
any launch, and its compile-time coefficient tables equal the oracle's
(independently derived) tables bit for bit."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2007_01416_amd", "libacat.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libacat.so not built")


@pytest.fixture(scope="module")
def lib():
    import paper_2007_01416_amd as acat
    return acat.load()


def declared_functions():
    src = open(os.path.join(ROOT, "include", "acat.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(acat_[a-z_0-9]+)\s*\(", src)))


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 8
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings(lib):
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert lib.acat_status_string(code)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_kernel_tables_equal_oracle_tables(p):
    import paper_2007_01416_amd as acat
    a = acat.coefficients(p)
    o = oracle.coeffs(p)
    for k in ("g1", "gt", "eta", "tau"):
        assert np.array_equal(a[k], o[k]), k


def _prob(**kw):
    import paper_2007_01416_amd as acat
    base = dict(dim=1, nvar=3, nx=64, flux="euler", P=2, bc="periodic", dx=0.1)
    base.update(kw)
    return acat.Problem(**base)


@pytest.mark.parametrize("kw,code", [
    (dict(dim=3), -2), (dict(P=0), -2), (dict(P=7), -2), (dict(nvar=2), -2), (dict(dx=0.0), -2),
    (dict(nx=3), -2), (dict(theta=0.0), -2), (dict(theta=1.5), -2), (dict(eps=-1.0), -2),
    (dict(flux="burgers", nvar=1, dim=2, ny=16, dy=0.1), -2),
    (dict(flux="advection", nvar=2), -4), (dict(dim=2, nvar=4, ny=64, dy=0.1, P=5), -4),
    (dict(gamma=1.0), -2),
    (dict(flags=16), -2),    # the square-stencil variant is 2D only
    # empty grids
    (dict(nx=0), -2), (dict(dim=2, nvar=4, nx=64, ny=0, dy=0.1), -2), (dict(nx=-5), -2),
    # smallest grid: 2 max(P, 2) cells per direction
    (dict(nx=7, P=4), -2), (dict(nx=11, P=6), -2), (dict(dim=2, nvar=4, nx=64, ny=5, dy=0.1, P=3), -2),
    # largest: item indices are 32-bit
    (dict(nx=(1 << 31) + 1), -2), (dict(nx=1 << 31), -4),
    (dict(dim=2, nvar=4, nx=1 << 16, ny=1 << 16, dy=0.1), -4),
])
def test_workspace_size_rejects_invalid_problems(lib, kw, code):
    n = ctypes.c_size_t(0)
    assert lib.acat_workspace_size(ctypes.byref(_prob(**kw).c()), ctypes.byref(n)) == code


def test_step_argument_errors_before_launch(lib):
    p = _prob()
    pc = p.c()
    ws = ctypes.create_string_buffer(16)
    buf = (ctypes.c_double * (3 * 64))()
    buf2 = (ctypes.c_double * (3 * 64))()
    a, b = ctypes.cast(buf, ctypes.c_void_p), ctypes.cast(buf2, ctypes.c_void_p)
    # null state
    assert lib.acat_step(ctypes.byref(pc), None, b, 0.1, None, ws, 16, None, None) == -1
    # aliasing input and output
    assert lib.acat_step(ctypes.byref(pc), a, a, 0.1, None, ws, 16, None, None) == -3
    # negative dt
    assert lib.acat_step(ctypes.byref(pc), a, b, -1.0, None, ws, 16, None, None) == -2
    # workspace too small
    assert lib.acat_step(ctypes.byref(pc), a, b, 0.1, None, ws, 16, None, None) == -6
    # replay needs decision maps
    need = ctypes.c_size_t(0)
    lib.acat_workspace_size(ctypes.byref(pc), ctypes.byref(need))
    big = ctypes.create_string_buffer(need.value)
    assert lib.acat_step_replay(ctypes.byref(pc), a, b, 0.1, None, big, need.value, None, None) == -1
    # cfl: non-positive cfl
    assert lib.acat_cfl_dt(ctypes.byref(pc), a, 0.0, 1.0, None, b, None) == -2
    assert lib.acat_max_wave_speed(ctypes.byref(pc), None, b, None) == -1


@pytest.mark.parametrize("P", [1, 2, 3, 4, 5, 6])
def test_smallest_grid_is_accepted(lib, P):
    n = ctypes.c_size_t(0)
    g = 2 * max(P, 2)
    assert lib.acat_workspace_size(ctypes.byref(_prob(nx=g, P=P).c()), ctypes.byref(n)) == 0 and n.value > 0
    if P <= 4:
        p2 = _prob(dim=2, nvar=4, nx=g, ny=g, dy=0.1, P=P)
        assert lib.acat_workspace_size(ctypes.byref(p2.c()), ctypes.byref(n)) == 0 and n.value > 0


def test_workspace_grows_with_problem(lib):
    import paper_2007_01416_amd as acat
    small = acat.workspace_bytes(_prob(nx=64))
    large = acat.workspace_bytes(_prob(nx=4096, P=4))
    assert large > small > 0
    w2 = acat.workspace_bytes(_prob(dim=2, nvar=4, nx=64, ny=32, dy=0.1, P=3))
    assert w2 > 9 * 4 * 64 * 32


def test_auto_checkpoint_spacing(lib):
    """AdjointRun(checkpoint_every="auto"): the segment is the longest whose
    resident steps (state, step workspace, decisions) fit the budget."""
    import paper_2007_01416_amd as acat
    p2 = _prob(dim=2, nvar=4, nx=64, ny=32, dy=0.1, P=3)
    per = acat.resident_bytes_per_step(p2)
    # state 4 x 64 x 32 doubles, the step workspace, and per interface an
    # order (1 byte), psi^1 and alpha (8 bytes each) in both directions
    assert per == 8 * 4 * 64 * 32 + acat.workspace_bytes(p2) + (32 * 64 + 32 * 64) * 17
    assert acat.auto_checkpoint(200, per, 10 ** 15) == 200
    assert acat.auto_checkpoint(200, per, 7 * per + per - 1) == 7
    assert acat.auto_checkpoint(200, per, 0) == 1
    with pytest.raises(ValueError):
        acat.auto_checkpoint(0, per, 10 ** 9)


def _batch_struct(n, P, bc, dx, flux=2, nvar=3):
    import paper_2007_01416_amd as acat
    n = np.ascontiguousarray(n, np.int64); P = np.ascontiguousarray(P, np.int32)
    bc = np.ascontiguousarray(bc, np.int32); dx = np.ascontiguousarray(dx, np.float64)
    b = acat._Batch(nvar, flux, 1.4, 1.0, 1e-12, 0.5, len(n), n.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                    P.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), bc.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                    dx.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return b, (n, P, bc, dx)


@pytest.mark.parametrize("n,P,bc,dx,code", [
    ([64, 32], [2, 3], [0, 1], [0.1, 0.1], 0),
    ([64, 4], [2, 1], [0, 1], [0.1, 0.1], -2),      # too few cells
    ([64, 32], [2, 5], [0, 1], [0.1, 0.1], -2),     # P out of range
    ([64, 32], [2, 3], [0, 7], [0.1, 0.1], -2),     # bad boundary
    ([64, 32], [2, 3], [0, 1], [0.1, 0.0], -2),     # dx <= 0
])
def test_batch_validation(lib, n, P, bc, dx, code):
    b, keep = _batch_struct(n, P, bc, dx)
    nb = ctypes.c_size_t(0)
    assert lib.acat_batch_workspace_size(ctypes.byref(b), ctypes.byref(nb)) == code
    if code == 0:
        assert nb.value > 0
        # a step needs its state and time-step pointers, and a large enough workspace
        ws = ctypes.create_string_buffer(nb.value)
        assert lib.acat_step_batched(ctypes.byref(b), None, None, None, ws, nb.value, None) == -1
        assert lib.acat_step_batched(ctypes.byref(b), ws, ws, ws, ws, 16, None) == -6
        # the fused-CFL step also needs cfl > 0
        assert lib.acat_step_batched_cfl(ctypes.byref(b), None, None, None, 0.5, ws, nb.value, None) == -1
        assert lib.acat_step_batched_cfl(ctypes.byref(b), ws, ws, ws, 0.0, ws, nb.value, None) == -2
        assert lib.acat_step_batched_cfl(ctypes.byref(b), ws, ws, ws, float("nan"), ws, nb.value, None) == -2
        assert lib.acat_step_batched_cfl(ctypes.byref(b), ws, ws, ws, 0.5, ws, 16, None) == -6


@pytest.mark.parametrize("table,code", [
    ([0] * 8, 0), ([1, 0, 2, 4, 4, 32, 0, 1], 0),
    ([3, 0, 0, 0, 0, 0, 0, 0], -2),                 # 3 waves per block
    ([0, 0, 0, 0, 0, 0, 8, 0], -2),                 # 8 waves per block
    ([0, 33, 0, 0, 0, 0, 0, 0], -2),                # too many blocks per CU
    ([0, 0, 0, -1, 0, 0, 0, 0], -2),
])
def test_batch_launch_table_validation(lib, table, code):
    b, keep = _batch_struct([64, 32], [2, 3], [0, 1], [0.1, 0.1])
    t = np.ascontiguousarray(table, np.int32)
    b.launch = t.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    nb = ctypes.c_size_t(0)
    assert lib.acat_batch_workspace_size(ctypes.byref(b), ctypes.byref(nb)) == code


def test_adjoint_argument_errors_before_launch(lib):
    import paper_2007_01416_amd as acat
    p = _prob()
    pc = p.c()
    n = ctypes.c_size_t(0)
    assert lib.acat_adjoint_workspace_size(ctypes.byref(pc), ctypes.byref(n)) == 0
    # the contribution buffer dominates: nvar * interfaces * 2P doubles
    assert n.value >= 8 * 3 * 64 * 4
    # every order and boundary of the forward step has an adjoint; the HLL variant has none
    p2 = _prob(dim=2, nvar=4, ny=32, dy=0.1, bc="transmissive", P=4)
    assert lib.acat_adjoint_workspace_size(ctypes.byref(p2.c()), ctypes.byref(n)) == 0
    assert lib.acat_adjoint_workspace_size(ctypes.byref(_prob(P=6, bc="transmissive").c()), ctypes.byref(n)) == 0
    assert lib.acat_adjoint_workspace_size(ctypes.byref(_prob(flags=2).c()), ctypes.byref(n)) == -4
    psq = _prob(dim=2, nvar=4, ny=32, dy=0.1, P=3, flags=16)
    assert lib.acat_workspace_size(ctypes.byref(psq.c()), ctypes.byref(n)) == 0
    assert lib.acat_adjoint_workspace_size(ctypes.byref(psq.c()), ctypes.byref(n)) == -4
    assert lib.acat_adjoint_workspace_size(ctypes.byref(_prob(P=7).c()), ctypes.byref(n)) == -2
    p5 = _prob(dim=2, nvar=4, ny=32, dy=0.1, P=5)
    assert lib.acat_adjoint_workspace_size(ctypes.byref(p5.c()), ctypes.byref(n)) == -4
    ub = (ctypes.c_double * (3 * 64))()
    ub2 = (ctypes.c_double * (3 * 64))()
    u = (ctypes.c_double * (3 * 64))()
    a, b, c = (ctypes.cast(x, ctypes.c_void_p) for x in (u, ub, ub2))
    o = (ctypes.c_int8 * 64)()
    d = (ctypes.c_double * 64)()
    dec = acat._Decisions(ctypes.cast(o, ctypes.c_void_p), ctypes.cast(d, ctypes.c_void_p),
                          ctypes.cast(d, ctypes.c_void_p), None, None, None)
    ws = ctypes.create_string_buffer(16)
    adj = lib.acat_step_adjoint
    assert adj(ctypes.byref(pc), a, 0.1, None, None, b, c, ws, 16, None) == -1            # no decisions
    nodec = acat._Decisions(None, None, None, None, None, None)
    assert adj(ctypes.byref(pc), a, 0.1, None, ctypes.byref(nodec), b, c, ws, 16, None) == -1
    assert adj(ctypes.byref(pc), a, 0.1, None, ctypes.byref(dec), None, c, ws, 16, None) == -1
    assert adj(ctypes.byref(pc), a, -1.0, None, ctypes.byref(dec), b, c, ws, 16, None) == -2
    assert adj(ctypes.byref(pc), a, 0.1, None, ctypes.byref(dec), b, a, ws, 16, None) == -3   # ubar_in over u
    half = ctypes.c_void_p(ctypes.addressof(ub) + 8 * 10)
    assert adj(ctypes.byref(pc), a, 0.1, None, ctypes.byref(dec), b, half, ws, 16, None) == -3
    assert adj(ctypes.byref(pc), a, 0.1, None, ctypes.byref(dec), b, c, ws, 16, None) == -6   # workspace
    # 2D needs the y decisions too
    p2 = _prob(dim=2, nvar=4, nx=16, ny=16, dy=0.1)
    assert adj(ctypes.byref(p2.c()), a, 0.1, None, ctypes.byref(dec), b, c, ws, 16, None) == -1
    # the list-reusing form: the same checks, then the step workspace's presence and size
    adl = lib.acat_step_adjoint_lists
    need = ctypes.c_size_t(0)
    assert lib.acat_adjoint_workspace_size(ctypes.byref(pc), ctypes.byref(need)) == 0
    big = ctypes.create_string_buffer(need.value)
    swn = ctypes.c_size_t(0)
    assert lib.acat_workspace_size(ctypes.byref(pc), ctypes.byref(swn)) == 0
    assert adl(ctypes.byref(pc), a, 0.1, None, ctypes.byref(dec), b, c, None, swn.value, big, need.value,
               None) == -1
    assert adl(ctypes.byref(pc), a, 0.1, None, ctypes.byref(dec), b, a, ws, swn.value, big, need.value,
               None) == -3
    assert adl(ctypes.byref(pc), a, 0.1, None, ctypes.byref(dec), b, c, ws, swn.value, ws, 16, None) == -6
    assert adl(ctypes.byref(pc), a, 0.1, None, ctypes.byref(dec), b, c, ws, swn.value - 1, big, need.value,
               None) == -6
    assert adl(ctypes.byref(_prob(flags=2).c()), a, 0.1, None, ctypes.byref(dec), b, c, ws, swn.value, big,
               need.value, None) == -4


def test_step_cfl_argument_errors_before_launch(lib):
    p = _prob()
    pc = p.c()
    buf = (ctypes.c_double * (3 * 64))()
    buf2 = (ctypes.c_double * (3 * 64))()
    a, b = ctypes.cast(buf, ctypes.c_void_p), ctypes.cast(buf2, ctypes.c_void_p)
    ws = ctypes.create_string_buffer(16)
    f = lib.acat_step_cfl
    assert f(ctypes.byref(pc), a, b, 0.5, 1.0, None, None, ws, 16, None, None) == -1     # dt_dev required
    assert f(ctypes.byref(pc), a, b, 0.0, 1.0, None, b, ws, 16, None, None) == -2      # cfl > 0
    assert f(ctypes.byref(pc), a, a, 0.5, 1.0, None, b, ws, 16, None, None) == -3      # aliasing
    assert f(ctypes.byref(pc), a, b, 0.5, 1.0, None, b, ws, 16, None, None) == -6      # workspace


@pytest.mark.parametrize("flags,code,adj", [
    (1, 0, 0), (2, 0, -4), (4, 0, 0), (1 | 4, 0, 0), (1 | 2, -2, -2), (16, -2, -2), (8, -4, -4),
])
def test_flags_validation(lib, flags, code, adj):
    """Variants: Lax-Friedrichs and HLL exclusive, Roe-speed limiter for
    scalar laws only (Euler here), unknown bits rejected; no HLL adjoint."""
    n = ctypes.c_size_t(0)
    pc = _prob(flags=flags).c()
    assert lib.acat_workspace_size(ctypes.byref(pc), ctypes.byref(n)) == code
    assert lib.acat_adjoint_workspace_size(ctypes.byref(pc), ctypes.byref(n)) == adj
    # the Roe-speed limiter is accepted for a scalar law
    pb = _prob(flux="burgers", nvar=1, flags=8).c()
    assert lib.acat_workspace_size(ctypes.byref(pb), ctypes.byref(n)) == 0


def test_fma_rate_argument_errors(lib):
    buf = (ctypes.c_double * 256)()
    p = ctypes.cast(buf, ctypes.c_void_p)
    assert lib.acat_fp64_fma_rate(1, 1, None, 256, None) == -1
    assert lib.acat_fp64_fma_rate(0, 1, p, 256, None) == -2
    assert lib.acat_fp64_fma_rate(1, 0, p, 256, None) == -2
    assert lib.acat_fp64_fma_rate(2, 1, p, 256, None) == -2


def test_empty_batch_is_rejected(lib):
    import paper_2007_01416_amd as acat
    n = np.zeros(0, np.int64); P = np.zeros(0, np.int32); bc = np.zeros(0, np.int32); dx = np.zeros(0)
    b = acat._Batch(3, 2, 1.4, 1.0, 1e-12, 0.5, 0, n.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                    P.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), bc.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                    dx.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    nb = ctypes.c_size_t(0)
    assert lib.acat_batch_workspace_size(ctypes.byref(b), ctypes.byref(nb)) == -2


def test_noalloc_rejects_problems_beyond_its_static_workspace(lib):
    """acat_step_noalloc refuses, before any launch, a problem whose
    workspace exceeds the static array (2048^2 2D Euler: 262 MB)."""
    big = _prob(dim=2, nvar=4, nx=2048, ny=2048, dy=0.01, P=3)
    n = ctypes.c_size_t(0)
    assert lib.acat_workspace_size(ctypes.byref(big.c()), ctypes.byref(n)) == 0
    assert n.value > 64 << 20
    assert lib.acat_step_noalloc(ctypes.byref(big.c()), None, None, 1e-3, None, None, None) == -6
    assert lib.acat_step_noalloc(ctypes.byref(_prob(P=0).c()), None, None, 1e-3, None, None, None) == -2
