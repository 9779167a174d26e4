"""Whole-loop pins of the oracle's Algorithm 1.

* Far-apart fixed point: if every pair is collision-free along the boundary-only
  trajectories, then with zero multipliers nothing ever moves (c^k = c^0,
  lambda^k = 0, f_c = 0).
* The x/y/z step minimises the augmented Lagrangian (eq. (aug_lagrange), written
  here as plain sums over pairs and instants) over the boundary-feasible set.
* Symmetries of the problem carried through 15 iterations: translation, rotation
  about z, mirror in z, relabelling of agents, and time reversal (swap starts and goals).
* Residual-decay envelope (the trend of Fig. "residual", Sec. IV-B): the mean of
  the RMS residual over successive iteration windows does not increase, and falls
  by at least 10x from the first to the last window.
* Boundary equalities and KKT stationarity hold to FP64 rounding at every iteration.
"""
import numpy as np
import pytest
import scipy.linalg

from oracle import am
from paper_2011_04240_amd import scenarios as sc


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def test_far_apart_fixed_point():
    plan = am.make_plan(4, 30, 11, 5.0, 0.4, 0.8, 1.0)
    starts = np.array([[10.0 * i, 0.0, 0.0] for i in range(4)])
    goals = starts + np.array([0.0, 5.0, 1.0])
    st0 = am.initial_state(plan, starts, goals)
    st = am.solve(plan, starts, goals, 20)
    np.testing.assert_allclose(st.c, st0.c, atol=1e-9)
    np.testing.assert_allclose(st.lam, 0.0, atol=1e-9)
    assert max(st.history["r_max"]) < 1e-9


def _lagrangian_x_by_sums(plan, c_axis, d, e_axis, lam_axis):
    """1/2 sum_i sum_t xdd^2 + sum_{i<j} sum_t rho/2 (x_i - x_j - d e + lam/rho)^2 for one axis."""
    x = c_axis @ plan.P.T
    xdd = c_axis @ plan.Pdd.T
    val = 0.5 * np.sum(xdd ** 2)
    p = 0
    for i in range(plan.n):
        for j in range(i + 1, plan.n):
            val += 0.5 * plan.rho * np.sum((x[i] - x[j] - d[p] * e_axis[p] + lam_axis[p] / plan.rho) ** 2)
            p += 1
    return val


def test_xyz_step_minimises_lagrangian():
    plan = am.make_plan(5, 40, 11, 5.0, 0.5, 0.9, 1.5)
    starts, goals = sc.swap_circle(5, radius=1.5, seed=3)
    st = am.initial_state(plan, starts, goals)
    for _ in range(4):
        st = am.iterate(plan, st)
    e = am.spheroid_direction(plan, st.alpha, st.beta)
    nxt = am.iterate(plan, st)
    Z = scipy.linalg.null_space(np.kron(np.eye(plan.n), plan.A))
    rng = _rng(11)
    for ax in range(3):
        c1 = nxt.c[:, ax, :].ravel()
        L = lambda v: _lagrangian_x_by_sums(plan, v.reshape(plan.n, -1), st.d, e[..., ax], st.lam[..., ax])
        L0 = L(c1)
        for _ in range(6):
            z = Z @ rng.standard_normal(Z.shape[1])
            z /= np.linalg.norm(z)
            eps = 1e-3
            lp, lm = L(c1 + eps * z), L(c1 - eps * z)
            assert abs(lp - lm) / (2 * eps) < 1e-6 * max(1.0, abs(L0))   # stationary
            assert lp > L0 and lm > L0                                  # a minimum
        np.testing.assert_allclose(np.kron(np.eye(plan.n), plan.A) @ c1, nxt.beq[:, ax, :].ravel(), atol=1e-10)


def _run(plan, starts, goals, k=15):
    return am.solve(plan, starts, goals, k)


@pytest.fixture(scope="module")
def base():
    plan = am.make_plan(5, 40, 11, 5.0, 0.4, 0.8, 1.0)
    starts, goals = sc.swap_circle(5, radius=1.5, seed=9)
    return plan, starts, goals, _run(plan, starts, goals)


def test_translation_invariance(base):
    plan, s, g, ref = base
    v = np.array([3.0, -7.0, 2.5])
    st = _run(plan, s + v, g + v)
    np.testing.assert_allclose(st.lam, ref.lam, atol=1e-8)
    np.testing.assert_allclose(st.d, ref.d, atol=1e-8)
    np.testing.assert_allclose(st.X, ref.X + v[None, :, None], atol=1e-8)


def test_rotation_about_z(base):
    plan, s, g, ref = base
    th = 0.7
    R = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1]])
    st = _run(plan, s @ R.T, g @ R.T)
    np.testing.assert_allclose(st.lam, ref.lam @ R.T, atol=1e-8)
    np.testing.assert_allclose(st.d, ref.d, atol=1e-8)
    np.testing.assert_allclose(st.c, np.einsum('ab,ibk->iak', R, ref.c), atol=1e-8)


def test_mirror_in_z(base):
    plan, s, g, ref = base
    M = np.diag([1.0, 1.0, -1.0])
    st = _run(plan, s @ M, g @ M)
    np.testing.assert_allclose(st.lam, ref.lam @ M, atol=1e-8)
    np.testing.assert_allclose(st.d, ref.d, atol=1e-8)
    np.testing.assert_allclose(st.beta, np.pi - ref.beta, atol=1e-8)


def test_agent_relabelling(base):
    plan, s, g, ref = base
    perm = np.array([3, 0, 4, 2, 1])          # new agent k is old agent perm[k]
    st = _run(plan, s[perm], g[perm])
    np.testing.assert_allclose(st.c, ref.c[perm], atol=1e-8)
    old_index = {(i, j): p for p, (i, j) in enumerate(zip(plan.I, plan.J))}
    for p, (k, l) in enumerate(zip(plan.I, plan.J)):
        i, j = perm[k], perm[l]
        sign = 1.0 if i < j else -1.0
        q = old_index[(min(i, j), max(i, j))]
        np.testing.assert_allclose(st.lam[p], sign * ref.lam[q], atol=1e-8)
        np.testing.assert_allclose(st.d[p], ref.d[q], atol=1e-8)


def test_time_reversal(base):
    plan, s, g, ref = base
    st = _run(plan, g, s)
    np.testing.assert_allclose(st.c, ref.c[:, :, ::-1], atol=1e-8)
    np.testing.assert_allclose(st.X, ref.X[:, :, ::-1], atol=1e-8)
    np.testing.assert_allclose(st.lam, ref.lam[:, ::-1, :], atol=1e-8)
    np.testing.assert_allclose(st.d, ref.d[:, ::-1], atol=1e-8)


def _windows_non_increasing(r, edges):
    means = [np.mean(r[a:b]) for a, b in zip(edges[:-1], edges[1:])]
    return means, all(m1 <= m0 for m0, m1 in zip(means[:-1], means[1:]))


@pytest.mark.parametrize("seed", range(4))
def test_residual_decay_swap_circle(seed):
    plan = am.make_plan(4, 50, 11, 5.0, 0.4, 0.8, 1.0)
    s, g = sc.swap_circle(4, seed=seed)
    st = am.solve(plan, s, g, 200)
    r = np.asarray(st.history["r_rms"])
    means, ok = _windows_non_increasing(r, [0, 25, 50, 100, 150, 200])
    assert ok, means
    assert means[-1] < means[0] / 10
    assert max(st.history["bnd_res"]) < 1e-10
    assert max(st.history["kkt_res"]) < 1e-9


def test_residual_decay_swap_sphere():
    plan = am.make_plan(16, 100, 11, 10.0, 0.3, 0.6, 1.0)
    s, g = sc.swap_sphere(16, seed=0)
    st = am.solve(plan, s, g, 300)
    r = np.asarray(st.history["r_rms"])
    means, ok = _windows_non_increasing(r, [0, 50, 100, 200, 300])
    assert ok, means
    assert means[-1] < means[0] / 10
    assert max(st.history["bnd_res"]) < 1e-9


def test_stop_on_tolerance():
    plan = am.make_plan(4, 50, 11, 5.0, 0.4, 0.8, 1.0)
    s, g = sc.swap_circle(4, seed=0)
    st = am.solve(plan, s, g, 500, tol=0.05)
    r = st.history["r_max"]
    assert r[-1] < 0.05 and all(x >= 0.05 for x in r[:-1])


def test_schedule_with_constant_rho_is_plain_solve():
    plan = am.make_plan(4, 50, 11, 5.0, 0.4, 0.8, 1.0)
    s, g = sc.swap_circle(4, seed=2)
    ref = am.solve(plan, s, g, 60)
    st = am.solve_schedule([plan, plan, plan], [0, 10, 35], s, g, 60)
    np.testing.assert_array_equal(st.c, ref.c)
    np.testing.assert_array_equal(st.lam, ref.lam)


def test_schedule_switch_uses_new_rho_in_the_step():
    """At a switch the x-step objective is the augmented Lagrangian with the new rho:
    c^{k+1} is stationary for (rho_new/2) sum ||x_i - x_j - d e + lambda/rho_new||^2."""
    p1 = am.make_plan(5, 40, 11, 5.0, 0.5, 0.9, 1.0)
    p2 = am.make_plan(5, 40, 11, 5.0, 0.5, 0.9, 3.0)
    s, g = sc.swap_circle(5, radius=1.5, seed=4)
    st = am.solve_schedule([p1], [0], s, g, 6)
    e = am.spheroid_direction(p2, st.alpha, st.beta)
    nxt = am.iterate(p2, st)
    Z = scipy.linalg.null_space(np.kron(np.eye(5), p2.A))
    rng = _rng(12)
    for ax in range(3):
        c1 = nxt.c[:, ax, :].ravel()
        L = lambda v: _lagrangian_x_by_sums(p2, v.reshape(5, -1), st.d, e[..., ax], st.lam[..., ax])
        for _ in range(4):
            z = Z @ rng.standard_normal(Z.shape[1])
            z /= np.linalg.norm(z)
            lp, lm = L(c1 + 1e-3 * z), L(c1 - 1e-3 * z)
            assert abs(lp - lm) / 2e-3 < 1e-6 * max(1.0, abs(L(c1)))


@pytest.mark.parametrize("seed", range(3))
def test_increasing_rho_schedule_decays(seed):
    """Doubling rho every 30 iterations (the schedule used by the library's serving
    defaults) keeps the residual-decay envelope and ends far below the start."""
    n = 16
    s, g = sc.random_density_box(n, seed=seed)
    plans = [am.make_plan(n, 60, 11, 6.0, 0.3, 0.6, 2.0 ** j) for j in range(6)]
    st = am.solve_schedule(plans, [30 * j for j in range(6)], s, g, 180)
    r = np.asarray(st.history["r_rms"])
    means = [np.mean(r[a:b]) for a, b in ((0, 30), (30, 60), (60, 120), (120, 180)) if a < len(r)]
    assert all(m1 <= m0 * 1.05 for m0, m1 in zip(means[:-1], means[1:])), means
    assert r[-1] < r[0] / 10 or st.history["r_max"][-1] < 1e-6
