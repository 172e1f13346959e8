"""Pins of the oracle's coefficient tables (differentiation formulas of
Sec. 2.1/2.2 and the interface weights defined by the telescoping relation
between centred and interpolatory formulas, Sec. 2.1)."""
from fractions import Fraction as Fr
from math import factorial

import numpy as np
import pytest

import oracle
from oracle import rational as R


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_tables_match_independent_rational_derivation(p):
    # C++ tables: expanded Lagrange basis; rational.py: moment-condition solve.
    c = oracle.coeffs(p)
    J = R.stencil(p)
    g1 = np.array([[float(x) for x in R.weights(J, Fr(j), 1)] for j in J])
    gt = np.array([[float(x) for x in R.weights(J, Fr(0), k)] for k in range(2 * p)])
    tau = np.array([float(x) for x in R.weights(J, Fr(1, 2), 2 * p - 1)])
    eta = np.array([float(x) for x in R.eta(p)])
    assert np.array_equal(g1, c["g1"])
    assert np.array_equal(gt, c["gt"])
    assert np.array_equal(tau, c["tau"])
    assert np.array_equal(eta, c["eta"])


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_moment_identities(p):
    # sum_j gamma^{k,q}_j (j - q)^m = k! delta_{mk} for m < 2p (exactness on polynomials)
    c = oracle.coeffs(p)
    J = np.arange(-p + 1, p + 1, dtype=float)
    for a, q in enumerate(J):
        for m in range(2 * p):
            terms = c["g1"][a] * (J - q) ** m
            assert abs(terms.sum() - (1.0 if m == 1 else 0.0)) < 1e-14 * max(1.0, np.abs(terms).sum())
    for k in range(2 * p):
        for m in range(2 * p):
            terms = c["gt"][k] * J ** m
            assert abs(terms.sum() - (factorial(k) if m == k else 0.0)) < 1e-14 * max(1.0, np.abs(terms).sum())


def test_textbook_tables():
    c1, c2 = oracle.coeffs(1), oracle.coeffs(2)
    assert np.array_equal(c1["d1"], [-0.5, 0.0, 0.5])
    assert np.array_equal(c1["eta"], [0.5, 0.5])
    assert np.array_equal(c1["g1"], [[-1, 1], [-1, 1]])
    # 4-point one-sided first derivative at node 0 of {-1,0,1,2}
    assert np.allclose(c2["g1"][1], [-1 / 3, -1 / 2, 1, -1 / 6], rtol=0, atol=1e-16)
    # centred 5-point first derivative and the 4th-order interface weights
    assert np.allclose(c2["d1"], np.array([1, -8, 0, 8, -1]) / 12, rtol=0, atol=1e-16)
    assert np.allclose(c2["eta"], np.array([-1, 7, 7, -1]) / 12, rtol=0, atol=1e-16)
    # (2p-1)-th derivative weights are the signed binomials (undivided difference)
    assert np.array_equal(oracle.coeffs(2)["tau"], [-1, 3, -3, 1])
    assert np.array_equal(oracle.coeffs(4)["tau"], [-1, 7, -21, 35, -35, 21, -7, 1])


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_eta_telescopes_to_centred_derivative(p):
    # A_i - A_{i-1} with weights eta reproduces the centred (2p+1)-point D^1
    c = oracle.coeffs(p)
    eta = np.concatenate([[0.0], c["eta"], [0.0]])   # eta_{-p} .. eta_{p+1}
    d = eta[:-1] - eta[1:]                           # delta_m = eta_m - eta_{m+1}, m = -p..p
    assert np.allclose(d, c["d1"], rtol=0, atol=1e-15)


@pytest.mark.parametrize("p", [2, 3])
def test_lagrange_interpolation_weights_are_not_eta(p):
    # The point value interpolant at x_{i+1/2} differs from the weights the
    # telescoping relation defines (the reading that makes CAT reduce to
    # Lax-Wendroff): guard against swapping them.
    lag = np.array([float(x) for x in R.weights(R.stencil(p), Fr(1, 2), 0)])
    assert not np.allclose(lag, oracle.coeffs(p)["eta"])
