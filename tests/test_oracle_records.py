"""Pins of the oracle's per-iteration records against values fixed by hand.

* Smoothness cost J = sum over agents, axes and instants of the squared acceleration,
  eq. (cost_proposed).  Bernstein coefficients C(j, q) / C(N, q) reproduce tau^q exactly
  (degree elevation), so a trajectory built from them has a known acceleration at every
  sample: for x(t) = s (t / t_f)^2 it is 2 s / t_f^2 at all T instants, for
  x(t) = s (t / t_f)^3 it is 6 s tau_k / t_f^2.  J is then a closed-form sum.  An affine
  part (zero acceleration) must not change it.
* Residual records of Algorithm 1's stopping rule and of the residual trend of Sec. IV-B:
  r_max is the largest Euclidean norm of f_c over pairs and instants, and r_rms the root
  mean square of those norms over all n(n-1)/2 * T pair-instants.  Both are checked on a
  hand-built f_c whose row norms are Pythagorean quadruples, so every expected value is a
  small exact number.
"""
from math import comb

import numpy as np
import pytest

from oracle import am


def _power_coeffs(N, q):
    """Bernstein coefficients of tau^q in degree N: C(j, q) / C(N, q)."""
    return np.array([comb(j, q) / comb(N, q) for j in range(N + 1)])


@pytest.mark.parametrize("T,tf", [(50, 5.0), (100, 10.0), (23, 3.0)])
def test_cost_of_quadratic_trajectories(T, tf):
    n = 3
    plan = am.make_plan(n, T, 11, tf, 0.3, 0.6, 1.0)
    N = 10
    quad = _power_coeffs(N, 2)
    lin = _power_coeffs(N, 1)
    one = _power_coeffs(N, 0)
    scale = np.array([[1.0, -2.0, 0.5], [3.0, 0.0, -1.5], [0.25, 2.0, -4.0]])
    c = np.zeros((n, 3, 11))
    for i in range(n):
        for a in range(3):
            # s tau^2 plus an affine part, which has no acceleration
            c[i, a] = scale[i, a] * quad + (1.0 + i) * one - (2.0 * a - 1.0) * lin
    expected = float(np.sum(scale ** 2)) * T * (2.0 / tf ** 2) ** 2
    assert am.smoothness_cost(plan, c) == pytest.approx(expected, rel=1e-12)


@pytest.mark.parametrize("T,tf", [(50, 5.0), (100, 10.0)])
def test_cost_of_cubic_trajectories(T, tf):
    n = 2
    plan = am.make_plan(n, T, 11, tf, 0.3, 0.6, 1.0)
    cub = _power_coeffs(10, 3)
    scale = np.array([[2.0, -1.0, 0.0], [0.5, 1.5, -3.0]])
    c = scale[:, :, None] * cub[None, None, :]
    # sum_k (6 s tau_k / t_f^2)^2 with tau_k = k / (T - 1): sum_k k^2 = (T-1) T (2T-1) / 6
    sum_tau2 = (T - 1) * T * (2 * T - 1) / 6.0 / (T - 1) ** 2
    expected = float(np.sum(scale ** 2)) * 36.0 / tf ** 4 * sum_tau2
    assert am.smoothness_cost(plan, c) == pytest.approx(expected, rel=1e-12)


def test_cost_is_recorded_per_iteration():
    """The cost entry of the iteration record is J of that iteration's coefficients."""
    plan = am.make_plan(3, 12, 11, 2.0, 0.3, 0.6, 1.0)
    cub = _power_coeffs(10, 3)
    c = np.stack([np.stack([k * cub for k in (1.0, 2.0, 3.0)]) for _ in range(3)])
    nu = np.zeros((3, 3, 6))
    g = np.zeros((3, 3, 11))
    beq = np.zeros((3, 3, 6))
    f_c = np.zeros((plan.n_rows, plan.T, 3))
    rec = am.records(plan, c, nu, g, beq, f_c)
    sum_tau2 = 11 * 12 * 23 / 6.0 / 11 ** 2
    assert rec["cost"] == pytest.approx(3 * (1 + 4 + 9) * 36.0 / 2.0 ** 4 * sum_tau2, rel=1e-12)


def _records_of(f_c):
    plan = am.make_plan(3, 12, 11, 2.0, 0.3, 0.6, 1.0)
    c = np.zeros((3, 3, 11))
    return am.records(plan, c, np.zeros((3, 3, 6)), np.zeros((3, 3, 11)), np.zeros((3, 3, 6)), f_c)


def test_residual_records_hand_built():
    # 3 agents -> 3 pairs, 12 instants: 36 pair-instants; four nonzero rows
    f_c = np.zeros((3, 12, 3))
    f_c[0, 0] = (3.0, 4.0, 0.0)      # norm 5
    f_c[1, 7] = (0.0, 0.0, -2.0)     # norm 2
    f_c[2, 3] = (1.0, -2.0, 2.0)     # norm 3
    f_c[2, 11] = (-2.0, 3.0, 6.0)    # norm 7
    rec = _records_of(f_c)
    assert rec["r_max"] == pytest.approx(7.0, rel=1e-15)
    # sum of squared norms 25 + 4 + 9 + 49 = 87 over 36 pair-instants
    assert rec["r_rms"] == pytest.approx(np.sqrt(87.0 / 36.0), rel=1e-15)


def test_residual_records_two_entries():
    """Norms 3 and 4 and 34 zeros: r_max = 4, r_rms = 5 / 6 (sqrt(25 / 36)); the mean of the
    norms (7 / 36) or the RMS over the nonzero entries only (sqrt(12.5)) would differ."""
    f_c = np.zeros((3, 12, 3))
    f_c[1, 2] = (0.0, 3.0, 0.0)
    f_c[0, 9] = (0.0, 0.0, 4.0)
    rec = _records_of(f_c)
    assert rec["r_max"] == pytest.approx(4.0, rel=1e-15)
    assert rec["r_rms"] == pytest.approx(5.0 / 6.0, rel=1e-15)


def test_residual_records_uniform_field():
    """The same f_c at every pair-instant: r_rms equals r_max equals that norm."""
    f_c = np.broadcast_to(np.array([2.0, -6.0, 9.0]), (3, 12, 3)).copy()    # norm 11
    rec = _records_of(f_c)
    assert rec["r_max"] == pytest.approx(11.0, rel=1e-15)
    assert rec["r_rms"] == pytest.approx(11.0, rel=1e-15)
