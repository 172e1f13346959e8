"""The library's 2D adjoint kernel templates run on the CPU under the address,
undefined-behaviour sanitizers (tests/host_kernels: the kernels of
acat_adjoint.hip compiled by g++ with a host execution model of the HIP
constructs they use, one thread per lane).  The corner classes whose
one-kernel form gave wrong values on the GPU, (2,4), (4,2), (3,4) and (4,3),
and two controls are run in the one-kernel form (both recursions in one
launch) and in the split form the library uses (two launches), on both
boundaries, and compared with the oracle's tangent of the same frozen step
through <J^T w, v> = <w, J v> on two random directions v (the GPU tests
compare element by element with the dense adjoint).  A clean run means the template itself is free of out-of-bounds
accesses, undefined behaviour and source-level errors in every form; the
GPU's wrong values in the one-kernel form then come from its device build.
The mirror-pair kernel (classes (qa, qb) and (qb, qa) in one launch) is run
the same way on a grid mixing the two classes and must equal the two
one-class kernels bit for bit; this includes the (1, 4) pair, whose device
build gave wrong values on the GPU and which the library therefore launches
one class at a time."""
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2007_01416_amd", "csrc")
NX, NY, P, NV = 10, 9, 4, 4
CASES = [(bc, q1, q2) for bc in (0, 1) for (q1, q2) in ((2, 4), (4, 2), (3, 4), (4, 3), (3, 3), (1, 4))]
# mirror pairs (qa, qb) + (qb, qa) in one launch, transmissive
PAIRS = [(1, 1, 2), (1, 1, 3), (1, 2, 3), (1, 1, 4)]


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    d = tmp_path_factory.mktemp("host_kernels")
    src = open(os.path.join(CSRC, "acat_adjoint.hip")).read()
    marker = "#define ACAT_CHECK_LAUNCH()"
    assert marker in src
    with open(d / "adjoint_kernels.inc", "w") as f:
        f.write(src[:src.index(marker)] + "\n}  // namespace\n}  // namespace acat\n")
    exe = str(d / "adjoint2d_host")
    cmd = ["g++", "-std=c++20", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-ffp-contract=off", "-fconstexpr-ops-limit=4000000000", "-I", str(d),
           "-I", os.path.join(HERE, "host_kernels"), "-I", CSRC, "-I", os.path.join(ROOT, "include"),
           os.path.join(HERE, "host_kernels", "adjoint2d_host.cpp"), "-o", exe, "-pthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    out = str(d / "adj.bin")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, out] + [f"{bc}:{q1}:{q2}" for bc, q1, q2 in CASES]
                       + [f"pair:{bc}:{qa}:{qb}" for bc, qa, qb in PAIRS], capture_output=True, text=True, env=env)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    return np.fromfile(out)


def smooth_state():
    x = (np.arange(NX) + 0.5) / NX
    y = (np.arange(NY) + 0.5) / NY
    X, Y = np.meshgrid(x, y, indexing="xy")
    rho = 1 + 0.1 * np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y)
    v, w = 0.3 + 0.05 * np.sin(2 * np.pi * Y), -0.2 + 0.05 * np.cos(2 * np.pi * X)
    p = 1 + 0.05 * np.sin(2 * np.pi * (X + Y))
    return np.stack([rho, rho * v, rho * w, p / 0.4 + 0.5 * rho * (v * v + w * w)])


@pytest.mark.parametrize("case", range(len(CASES)))
def test_adjoint_template_on_host_matches_dense_oracle(harness, case):
    bc, q1, q2 = CASES[case]
    n = NV * NX * NY
    base = 3 * n * case
    one, split, ub = (harness[base + k * n:base + (k + 1) * n].reshape(NV, NY, NX) for k in range(3))
    po = oracle.Problem(dim=2, nvar=4, nx=NX, ny=NY, P=P, bc=bc, dx=1.0 / NX, dy=1.0 / NY)
    nIx, nIy = po.n_interfaces
    maps = (np.full((NY, nIx), q1, np.int8), np.full((nIy, NX), q2, np.int8), np.full((NY, nIx), 0.6),
            np.full((nIy, NX), 0.6), np.full((NY, nIx), 2.0), np.full((nIy, NX), 2.0))
    u = smooth_state()
    assert np.abs(one - split).max() <= 1e-13 * np.abs(split).max()
    rng = np.random.default_rng(case)
    for _ in range(2):
        v = rng.standard_normal(u.shape)
        rhs = float(np.vdot(ub, oracle.jvp(po, u, v, 0.002, maps)[1]))
        for name, got in (("one-kernel", one), ("split", split)):
            lhs = float(np.vdot(got, v))
            print(f"bc={bc} ({q1},{q2}) {name}: <J^T w, v> {lhs:.15e} <w, J v> {rhs:.15e}", file=sys.stderr)
            assert abs(lhs - rhs) <= 1e-12 * abs(rhs), name


@pytest.mark.parametrize("case", range(len(PAIRS)))
def test_mirror_pair_kernel_on_host_equals_one_class_kernels(harness, case):
    """The pair kernel (corners of (qa, qb) and (qb, qa) mixed on one grid,
    blocks split between the two class lists) gives the same gathered adjoint,
    bit for bit, as the two one-class kernels run one after the other."""
    n = NV * NX * NY
    base = 3 * n * len(CASES) + 2 * n * case
    pair, sep = (harness[base + k * n:base + (k + 1) * n] for k in range(2))
    assert np.abs(sep).max() > 0
    assert np.array_equal(pair, sep)
