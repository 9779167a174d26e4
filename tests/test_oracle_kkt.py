"""Pins of the oracle's x/y/z QP step (eqs. (cost_step_x)-(kkt_step_x), Remarks 1-2).

* The literal A_fc of eq. (A_f), the pair-by-pair Gram matrix and the closed form
  (n I - 1 1^T) (x) P^T P agree.
* The inverse-based step agrees with an independent null-space solution of the
  equality-constrained QP whose objective is written out as sums over agents,
  pairs and instants (not through A_fc or K).
* K^{-1} agrees with the two-block closed form obtained from the spectral
  decomposition of n I - 1 1^T.
* The boundary coefficients come out exactly: for rest-to-rest boundary data the
  first three Bernstein coefficients equal the start and the last three the goal.
* K does not depend on the agent dimensions or on the boundary data (Remark 2).
"""
import numpy as np
import pytest
import scipy.linalg

from oracle import am, kkt
from oracle.basis import basis_matrices


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


@pytest.mark.parametrize("n", [2, 3, 5])
def test_collision_gram_forms(n):
    P, _, _ = basis_matrices(11, 20, 4.0)
    Afc = kkt.collision_matrix(P, n)
    assert Afc.shape == (20 * n * (n - 1) // 2, 11 * n)
    closed = np.kron(n * np.eye(n) - np.ones((n, n)), P.T @ P)
    np.testing.assert_allclose(Afc.T @ Afc, closed, atol=1e-12)
    np.testing.assert_allclose(kkt.collision_gram(P, n), closed, atol=1e-12)
    b = _rng(n).standard_normal((n * (n - 1) // 2, 20))
    np.testing.assert_allclose(kkt.collision_transpose_apply(P, n, b).ravel(),
                               Afc.T @ b.ravel(), atol=1e-12)


def test_collision_rows_are_pair_differences():
    """Row (p, t) of A_fc applied to c gives x_i(t) - x_j(t) for the p-th pair (i < j)."""
    n, T = 4, 9
    P, _, _ = basis_matrices(7, T, 2.0)
    Afc = kkt.collision_matrix(P, n)
    c = _rng(1).standard_normal((n, 7))
    x = c @ P.T
    I, J = kkt.pair_index(n)
    want = np.concatenate([x[i] - x[j] for i, j in zip(I, J)])
    np.testing.assert_allclose(Afc @ c.ravel(), want, atol=1e-13)
    assert list(zip(I, J))[:3] == [(0, 1), (0, 2), (0, 3)]


def _objective_by_sums(P, Pdd, rho, c, bfc, I, J):
    """1/2 sum_i sum_t xdd_i(t)^2 + rho/2 sum_{p,t} (x_i - x_j - b_p(t))^2.

    The smoothness weight 1/2 is the reading that matches Q_x as printed in eq. (kkt_step_x).
    """
    x = c @ P.T
    xdd = c @ Pdd.T
    val = 0.5 * np.sum(xdd ** 2)
    for p, (i, j) in enumerate(zip(I, J)):
        val += 0.5 * rho * np.sum((x[i] - x[j] - bfc[p]) ** 2)
    return val


@pytest.mark.parametrize("n,rho", [(2, 1.0), (3, 1.0), (4, 2.5)])
def test_step_matches_null_space_solution(n, rho):
    """Minimise the sum-form objective over {c : A c_i = b_eq,i} with a null-space
    basis (SVD) and a dense least-squares particular solution; compare with K^{-1} q."""
    T, nv = 24, 11
    plan = am.make_plan(n, T, nv, 3.0, 0.5, 0.7, rho)
    rng = _rng(7 + n)
    starts, goals = rng.uniform(-2, 2, (n, 3)), rng.uniform(-2, 2, (n, 3))
    beq = am.boundary_rhs_all(starts, goals)
    bfc = rng.standard_normal((n * (n - 1) // 2, T, 3))
    c, nu, g = am.step_xyz(plan, bfc, beq)
    Aeq = np.kron(np.eye(n), plan.A)
    Z = scipy.linalg.null_space(Aeq)
    for ax in range(3):
        c_p = np.linalg.lstsq(Aeq, beq[:, ax, :].ravel(), rcond=None)[0]
        f = lambda y: _objective_by_sums(plan.P, plan.Pdd, rho, (c_p + Z @ y).reshape(n, nv),
                                         bfc[:, :, ax], plan.I, plan.J)
        # the objective is quadratic in y: recover its Hessian and gradient by exact
        # polarisation, then solve the reduced normal equations
        m = Z.shape[1]
        f0 = f(np.zeros(m))
        E = np.eye(m)
        fe = np.array([f(E[k]) for k in range(m)])
        fm = np.array([f(-E[k]) for k in range(m)])
        grad = (fe - fm) / 2
        diag = fe + fm - 2 * f0
        Hr = np.diag(diag)
        for k in range(m):
            for l in range(k + 1, m):
                v = f(E[k] + E[l]) - fe[k] - fe[l] + f0
                Hr[k, l] = Hr[l, k] = v
        y = np.linalg.solve(Hr, -grad)
        c_ref = (c_p + Z @ y).reshape(n, nv)
        np.testing.assert_allclose(c[:, ax, :], c_ref, atol=1e-7 * max(1, np.abs(c_ref).max()))


@pytest.mark.parametrize("n", [2, 5, 16])
def test_inverse_two_block_closed_form(n):
    """In per-agent ordering K = (11^T/n) (x) K(0) + (I - 11^T/n) (x) K(n), where
    K(s) = [[Pdd^T Pdd + s rho P^T P, A^T], [A, 0]]; hence K^{-1} has the same form with
    K(0)^{-1} and K(n)^{-1}."""
    T, nv, rho = 40, 11, 1.3
    plan = am.make_plan(n, T, nv, 6.0, 0.3, 0.6, rho)
    nb = plan.A.shape[0]

    def Ks(s):
        M = np.zeros((nv + nb, nv + nb))
        M[:nv, :nv] = plan.Pdd.T @ plan.Pdd + s * rho * plan.P.T @ plan.P
        M[:nv, nv:] = plan.A.T
        M[nv:, :nv] = plan.A
        return M

    Pi1 = np.ones((n, n)) / n
    closed = np.kron(Pi1, np.linalg.inv(Ks(0.0))) + np.kron(np.eye(n) - Pi1, np.linalg.inv(Ks(float(n))))
    # permutation from per-agent ordering [c_0, nu_0, c_1, nu_1, ...] to [c (all); nu (all)]
    perm = np.concatenate([np.concatenate([np.arange(i * nv, (i + 1) * nv),
                                           n * nv + np.arange(i * nb, (i + 1) * nb)])
                           for i in range(n)])
    Kinv_agent = plan.Kinv[np.ix_(perm, perm)]
    err = np.max(np.abs(Kinv_agent - closed)) / np.max(np.abs(closed))
    assert err < 1e-10


def test_kkt_symmetric_and_independent_of_dimensions_and_boundary():
    p1 = am.make_plan(4, 30, 11, 5.0, 0.4, 0.8, 1.0)
    p2 = am.make_plan(4, 30, 11, 5.0, 1.7, 0.2, 1.0)
    np.testing.assert_array_equal(p1.K, p2.K)
    np.testing.assert_allclose(p1.K, p1.K.T, atol=0)
    lit = kkt.kkt_matrix(p1.P, p1.Pdd, p1.A, 4, 1.0, literal=True)
    np.testing.assert_allclose(lit, p1.K, atol=1e-12)


@pytest.mark.parametrize("n,T,tf", [(4, 50, 5.0), (16, 100, 10.0)])
def test_exact_boundary_coefficients(n, T, tf):
    """Rest-to-rest data fixes c_0 = c_1 = c_2 = start and c_8 = c_9 = c_10 = goal
    (Bernstein end-point derivatives), whatever the collision term."""
    plan = am.make_plan(n, T, 11, tf, 0.3, 0.6, 1.0)
    rng = _rng(n)
    starts, goals = rng.uniform(-5, 5, (n, 3)), rng.uniform(-5, 5, (n, 3))
    beq = am.boundary_rhs_all(starts, goals)
    bfc = rng.standard_normal((n * (n - 1) // 2, T, 3)) * 3
    c, nu, g = am.step_xyz(plan, bfc, beq)
    for k in range(3):
        np.testing.assert_allclose(c[:, :, k], starts, atol=1e-9)
        np.testing.assert_allclose(c[:, :, 10 - k], goals, atol=1e-9)


def test_boundary_only_initialisation_is_minimum_acceleration():
    """c^0 satisfies A c = b_eq and has zero projected gradient of sum xdd^2 on null(A)."""
    plan = am.make_plan(3, 30, 11, 5.0, 0.4, 0.8, 1.0)
    rng = _rng(3)
    starts, goals = rng.uniform(-3, 3, (3, 3)), rng.uniform(-3, 3, (3, 3))
    st = am.initial_state(plan, starts, goals)
    Z = scipy.linalg.null_space(plan.A)
    for i in range(3):
        for ax in range(3):
            c = st.c[i, ax]
            np.testing.assert_allclose(plan.A @ c, st.beq[i, ax], atol=1e-12)
            grad = 2 * plan.Pdd.T @ (plan.Pdd @ c)
            assert np.max(np.abs(Z.T @ grad)) < 1e-9
    np.testing.assert_allclose(st.lam, 0.0)
