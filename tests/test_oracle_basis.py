"""Pins of the oracle's trajectory parametrisation (eq. (param), Sec. III-B).

Each check is a closed form or invariant of the Bernstein basis, not a re-typing
of the oracle's formula: partition of unity, the end-point rows, exact
reproduction of monomials through their Bernstein coefficients, and agreement
of the derivative matrices with finite differences of P.
"""
from math import comb

import numpy as np
import pytest

from oracle.basis import basis_matrices, sample_times

CASES = [(11, 50, 5.0), (11, 100, 10.0), (8, 37, 3.0), (6, 7, 1.0)]


@pytest.mark.parametrize("n_coef,T,tf", CASES)
def test_partition_of_unity(n_coef, T, tf):
    P, Pd, Pdd = basis_matrices(n_coef, T, tf)
    assert P.shape == (T, n_coef)
    np.testing.assert_allclose(P.sum(axis=1), 1.0, atol=1e-13)
    scale = (n_coef - 1) / tf
    np.testing.assert_allclose(Pd.sum(axis=1), 0.0, atol=1e-12 * scale)
    np.testing.assert_allclose(Pdd.sum(axis=1), 0.0, atol=1e-11 * scale ** 2)
    assert np.all(P >= 0.0)


@pytest.mark.parametrize("n_coef,T,tf", CASES)
def test_endpoint_rows(n_coef, T, tf):
    P, Pd, Pdd = basis_matrices(n_coef, T, tf)
    N = n_coef - 1
    e0 = np.zeros(n_coef); e0[0] = 1
    eN = np.zeros(n_coef); eN[-1] = 1
    np.testing.assert_allclose(P[0], e0, atol=1e-15)
    np.testing.assert_allclose(P[-1], eN, atol=1e-15)
    v0 = np.zeros(n_coef); v0[:2] = [-1, 1]
    vN = np.zeros(n_coef); vN[-2:] = [-1, 1]
    np.testing.assert_allclose(Pd[0], N / tf * v0, atol=1e-13)
    np.testing.assert_allclose(Pd[-1], N / tf * vN, atol=1e-13)
    a0 = np.zeros(n_coef); a0[:3] = [1, -2, 1]
    aN = np.zeros(n_coef); aN[-3:] = [1, -2, 1]
    np.testing.assert_allclose(Pdd[0], N * (N - 1) / tf ** 2 * a0, atol=1e-12)
    np.testing.assert_allclose(Pdd[-1], N * (N - 1) / tf ** 2 * aN, atol=1e-12)


@pytest.mark.parametrize("n_coef,T,tf", CASES)
def test_monomial_reproduction(n_coef, T, tf):
    """tau^q has Bernstein coefficients C(j, q) / C(N, q); P, P-dot and P-ddot must
    return tau^q and its first two time derivatives exactly."""
    P, Pd, Pdd = basis_matrices(n_coef, T, tf)
    N = n_coef - 1
    tau, _ = sample_times(T, tf)
    for q in range(N + 1):
        c = np.array([comb(j, q) / comb(N, q) for j in range(n_coef)])
        np.testing.assert_allclose(P @ c, tau ** q, atol=1e-13)
        d1 = q * tau ** max(q - 1, 0) / tf if q >= 1 else np.zeros(T)
        d2 = q * (q - 1) * tau ** max(q - 2, 0) / tf ** 2 if q >= 2 else np.zeros(T)
        np.testing.assert_allclose(Pd @ c, d1, atol=1e-11)
        np.testing.assert_allclose(Pdd @ c, d2, atol=1e-10)


def test_finite_differences():
    """Central differences of P (and of P-dot) in physical time converge to P-dot (P-ddot) at O(h^2)."""
    errs = []
    for T in (201, 401):
        P, Pd, Pdd = basis_matrices(11, T, 10.0)
        h = 10.0 / (T - 1)
        fd1 = (P[2:] - P[:-2]) / (2 * h)
        fd2 = (Pd[2:] - Pd[:-2]) / (2 * h)
        errs.append((np.max(np.abs(fd1 - Pd[1:-1])), np.max(np.abs(fd2 - Pdd[1:-1]))))
    for k in range(2):
        assert errs[1][k] < errs[0][k] / 3.5          # second-order convergence
        assert errs[1][k] < 1e-3
