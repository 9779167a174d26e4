"""Trajectory parametrisation, eq. (param), Sec. III-B ("Steps (step_x_3d)-(step_z_3d)").

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper writes each position component as a linear map of basis
coefficients, x_i = P c_{x_i}, with velocity P-dot c and acceleration
P-ddot c, and leaves the basis open (polynomials are one example).  The reading used
here: a Bernstein basis of degree n_coef-1 on normalised time tau in [0, 1],
sampled at T uniformly spaced instants that include both end points
(tau_k = k/(T-1), t_k = t_final * tau_k).  Derivatives are taken in physical
time, so one factor 1/t_final per derivative.
"""
from math import comb

import numpy as np


def sample_times(T, t_final):
    """Normalised and physical sample instants (tau_k, t_k), k = 0..T-1."""
    tau = np.arange(T, dtype=np.float64) / (T - 1)
    return tau, t_final * tau


def bernstein(deg, j, tau):
    """B_{j,deg}(tau) = C(deg, j) tau^j (1 - tau)^(deg - j); zero outside 0 <= j <= deg."""
    tau = np.asarray(tau, dtype=np.float64)
    if j < 0 or j > deg:
        return np.zeros_like(tau)
    return comb(deg, j) * tau ** j * (1.0 - tau) ** (deg - j)


def basis_matrices(n_coef, T, t_final):
    """Return (P, Pdot, Pddot), each T x n_coef, FP64.

    P[k, j]     = B_{j,N}(tau_k)                                   N = n_coef - 1
    Pdot[k, j]  = N/t_f      * (B_{j-1,N-1} - B_{j,N-1})(tau_k)
    Pddot[k, j] = N(N-1)/t_f^2 * (B_{j-2,N-2} - 2 B_{j-1,N-2} + B_{j,N-2})(tau_k)
    """
    N = n_coef - 1
    tau, _ = sample_times(T, t_final)
    P = np.stack([bernstein(N, j, tau) for j in range(n_coef)], axis=1)
    Pd = np.stack([N * (bernstein(N - 1, j - 1, tau) - bernstein(N - 1, j, tau))
                   for j in range(n_coef)], axis=1) / t_final
    Pdd = np.stack([N * (N - 1) * (bernstein(N - 2, j - 2, tau)
                                   - 2.0 * bernstein(N - 2, j - 1, tau)
                                   + bernstein(N - 2, j, tau))
                    for j in range(n_coef)], axis=1) / t_final ** 2
    return P, Pd, Pdd
