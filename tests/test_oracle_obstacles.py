"""Pins of the oracle's static obstacles (Sec. IV-A: circumscribing spheres; their cost
enters only through A_fc^T b, Sec. IV-B).

* The literal A_fc with agent-obstacle rows: A_fc^T A_fc equals the pair-by-pair Gram and
  the closed form ((n + n_obs) I - 1 1^T) (x) P^T P; A_fc^T b by blocks equals the literal product.
* The x-step minimises the augmented Lagrangian written as plain sums over agent pairs
  and agent-obstacle pairs (a dropped or mis-signed obstacle centre fails stationarity).
* Far-apart fixed point with obstacles; translation of agents and obstacles together;
  rotation about z; relabelling of obstacles and of agents.
* Residual-decay envelope with obstacles; the constraint residual of every obstacle row
  is recorded in r_max.
"""
import numpy as np
import pytest
import scipy.linalg

from oracle import am, basis, kkt
from paper_2011_04240_amd import scenarios as sc


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


@pytest.mark.parametrize("n,n_obs", [(2, 1), (3, 2), (4, 3)])
def test_literal_gram_with_obstacles(n, n_obs):
    P, Pd, Pdd = basis.basis_matrices(11, 12, 3.0)
    Afc = kkt.collision_matrix(P, n, n_obs)
    T = P.shape[0]
    assert Afc.shape == (T * (n * (n - 1) // 2 + n * n_obs), n * 11)
    G = Afc.T @ Afc
    np.testing.assert_allclose(G, kkt.collision_gram(P, n, n_obs), atol=1e-12)
    L = (n + n_obs) * np.eye(n) - np.ones((n, n))
    np.testing.assert_allclose(G, np.kron(L, P.T @ P), atol=1e-12)
    b = _rng(n).standard_normal((n * (n - 1) // 2 + n * n_obs, T))
    np.testing.assert_allclose(kkt.collision_transpose_apply(P, n, b, n_obs),
                               (Afc.T @ b.ravel()).reshape(n, 11), atol=1e-12)


def _lagrangian_axis(plan, obs, c_axis, d, e_axis, lam_axis, ax):
    """1/2 sum xdd^2 + sum over agent pairs and agent-obstacle pairs of
    rho/2 (x_i - x_j - d e + lam/rho)^2, x_j = the obstacle centre for obstacle rows."""
    x = c_axis @ plan.P.T
    xdd = c_axis @ plan.Pdd.T
    val = 0.5 * np.sum(xdd ** 2)
    p = 0
    for i in range(plan.n):
        for j in range(i + 1, plan.n):
            val += 0.5 * plan.rho * np.sum((x[i] - x[j] - d[p] * e_axis[p] + lam_axis[p] / plan.rho) ** 2)
            p += 1
    for i in range(plan.n):
        for o in range(plan.n_obs):
            val += 0.5 * plan.rho * np.sum((x[i] - obs[o, ax] - d[p] * e_axis[p] + lam_axis[p] / plan.rho) ** 2)
            p += 1
    return val


def test_xyz_step_minimises_lagrangian_with_obstacles():
    s, g, obs = sc.obstacle_box(4, 3, seed=2)
    plan = am.make_plan(4, 30, 11, 4.0, 0.3, 0.6, 1.3, n_obs=3)
    st = am.initial_state(plan, s, g, obs)
    for _ in range(3):
        st = am.iterate(plan, st)
    e = am.spheroid_direction(plan, st.alpha, st.beta, am.row_dims(plan, obs))
    nxt = am.iterate(plan, st)
    Z = scipy.linalg.null_space(np.kron(np.eye(plan.n), plan.A))
    rng = _rng(21)
    for ax in range(3):
        c1 = nxt.c[:, ax, :].ravel()
        L = lambda v: _lagrangian_axis(plan, obs, v.reshape(plan.n, -1), st.d, e[..., ax], st.lam[..., ax], ax)
        L0 = L(c1)
        for _ in range(5):
            z = Z @ rng.standard_normal(Z.shape[1])
            z /= np.linalg.norm(z)
            lp, lm = L(c1 + 1e-3 * z), L(c1 - 1e-3 * z)
            assert abs(lp - lm) / 2e-3 < 1e-6 * max(1.0, abs(L0))
            assert lp > L0 and lm > L0


def test_far_apart_fixed_point_with_obstacles():
    plan = am.make_plan(3, 30, 11, 5.0, 0.4, 0.8, 1.0, n_obs=2)
    starts = np.array([[10.0 * i, 0.0, 0.0] for i in range(3)])
    goals = starts + np.array([0.0, 5.0, 1.0])
    obs = np.array([[5.0, 40.0, 0.0, 0.5, 0.7], [-30.0, 2.0, 1.0, 0.6, 0.6]])
    st0 = am.initial_state(plan, starts, goals, obs)
    st = am.solve(plan, starts, goals, 20, obs=obs)
    np.testing.assert_allclose(st.c, st0.c, atol=1e-9)
    np.testing.assert_allclose(st.lam, 0.0, atol=1e-9)
    assert max(st.history["r_max"]) < 1e-9


# agents swapping across a circle of radius 2 m, obstacles on and near the crossing paths
CROSSING_OBS = np.array([[0.0, 0.0, 0.0, 0.75, 0.9], [1.0, 0.5, 0.0, 0.5, 0.6],
                         [-0.8, 0.9, 0.1, 0.45, 0.6], [0.3, -1.1, -0.1, 0.5, 0.65]])


@pytest.fixture(scope="module")
def base():
    s, g = sc.swap_circle(5, radius=2.0, seed=11)
    plan = am.make_plan(5, 40, 11, 5.0, 0.3, 0.6, 1.0, n_obs=4)
    return plan, s, g, CROSSING_OBS, am.solve(plan, s, g, 15, obs=CROSSING_OBS)


def test_obstacles_are_active(base):
    plan, s, g, obs, ref = base
    st0 = am.initial_state(plan, s, g, obs)
    s_obs = np.sqrt(np.sum((st0.delta[plan.n_pairs:] / np.concatenate(am.row_dims(plan, obs), 1)[plan.n_pairs:,
                                                                                                   None, [0, 0, 1]]) ** 2, -1))
    assert s_obs.min() < 0.5                      # straight lines pass through obstacles
    free = am.solve(am.make_plan(5, 40, 11, 5.0, 0.3, 0.6, 1.0), s, g, 15)
    assert np.max(np.abs(free.c - ref.c)) > 1e-2
    fo = np.sqrt(np.sum(ref.f_c[plan.n_pairs:] ** 2, -1))
    assert fo.max() > 1e-3


def test_translation_with_obstacles(base):
    plan, s, g, obs, ref = base
    v = np.array([3.0, -7.0, 2.5])
    o2 = obs.copy()
    o2[:, :3] += v
    st = am.solve(plan, s + v, g + v, 15, obs=o2)
    np.testing.assert_allclose(st.lam, ref.lam, atol=1e-8)
    np.testing.assert_allclose(st.d, ref.d, atol=1e-8)
    np.testing.assert_allclose(st.X, ref.X + v[None, :, None], atol=1e-8)


def test_rotation_about_z_with_obstacles(base):
    plan, s, g, obs, ref = base
    th = -1.1
    R = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1]])
    o2 = obs.copy()
    o2[:, :3] = obs[:, :3] @ R.T
    st = am.solve(plan, s @ R.T, g @ R.T, 15, obs=o2)
    np.testing.assert_allclose(st.lam, ref.lam @ R.T, atol=1e-8)
    np.testing.assert_allclose(st.c, np.einsum('ab,ibk->iak', R, ref.c), atol=1e-8)


def test_obstacle_relabelling(base):
    plan, s, g, obs, ref = base
    perm = np.array([2, 0, 3, 1])           # new obstacle k is old obstacle perm[k]
    st = am.solve(plan, s, g, 15, obs=obs[perm])
    np.testing.assert_allclose(st.c, ref.c, atol=1e-8)
    npairs, no = plan.n_pairs, plan.n_obs
    for i in range(plan.n):
        for k in range(no):
            np.testing.assert_allclose(st.lam[npairs + i * no + k], ref.lam[npairs + i * no + perm[k]], atol=1e-8)
            np.testing.assert_allclose(st.d[npairs + i * no + k], ref.d[npairs + i * no + perm[k]], atol=1e-8)


def test_agent_relabelling_with_obstacles(base):
    plan, s, g, obs, ref = base
    perm = np.array([3, 0, 4, 2, 1])
    st = am.solve(plan, s[perm], g[perm], 15, obs=obs)
    np.testing.assert_allclose(st.c, ref.c[perm], atol=1e-8)
    npairs, no = plan.n_pairs, plan.n_obs
    for k in range(plan.n):
        np.testing.assert_allclose(st.lam[npairs + k * no: npairs + (k + 1) * no],
                                   ref.lam[npairs + perm[k] * no: npairs + (perm[k] + 1) * no], atol=1e-8)


def test_residual_decay_with_obstacles():
    s, g = sc.swap_circle(5, radius=2.0, seed=4)
    plan = am.make_plan(5, 50, 11, 6.0, 0.3, 0.6, 1.0, n_obs=4)
    st = am.solve(plan, s, g, 250, obs=CROSSING_OBS)
    r = np.asarray(st.history["r_rms"])
    means = [np.mean(r[a:b]) for a, b in ((0, 25), (25, 50), (50, 100), (100, 175), (175, 250))]
    assert all(m1 <= m0 for m0, m1 in zip(means[:-1], means[1:])), means
    assert means[-1] < means[0] / 10
    assert max(st.history["bnd_res"]) < 1e-10
    assert max(st.history["kkt_res"]) < 1e-9
    # every obstacle row is in the record: its residual never exceeds r_max
    fo = np.sqrt(np.sum(st.f_c[plan.n_pairs:] ** 2, axis=-1))
    assert fo.max() <= st.history["r_max"][-1] + 1e-15


def test_obstacle_rows_use_their_own_axes():
    """At lambda = 0 the d step is d = max(1, s) with s the scaled distance in each
    row's own clearance spheroid (obstacles have l_xy != l_z and differ from the pairs')."""
    s, g = sc.swap_circle(5, radius=2.0, seed=3)
    plan = am.make_plan(5, 40, 11, 5.0, 0.3, 0.6, 1.0, n_obs=4)
    st = am.initial_state(plan, s, g, CROSSING_OBS)
    X = st.X
    for i in range(plan.n):
        for o in range(plan.n_obs):
            dl = X[i].T - CROSSING_OBS[o, :3]                       # (T, 3)
            lxy, lz = CROSSING_OBS[o, 3], CROSSING_OBS[o, 4]
            sd = np.sqrt((dl[:, 0] ** 2 + dl[:, 1] ** 2) / lxy ** 2 + dl[:, 2] ** 2 / lz ** 2)
            np.testing.assert_allclose(st.d[plan.n_pairs + i * plan.n_obs + o], np.maximum(1.0, sd), rtol=1e-12)
