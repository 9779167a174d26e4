"""Pins of the oracle's element-wise steps: (sphere_project), (step_d), (lag_update).

* d: brute-force 1-D grid over d >= 1 of the step-(step_d) objective.
* alpha, beta: brute-force 2-D grid over the angles of the step-(step_alpha)
  objective (sign convention of f_c) for spheres with zero multipliers, where the
  radial projection is the exact minimiser; e is compared, never raw alpha.
* identities: delta = s e with s the scaled distance; non-colliding pairs with
  zero multipliers give d = s and f_c = 0; an unclipped d leaves e^T lambda^{k+1} = 0;
  alpha in [-pi, pi], beta in [0, pi], d >= 1 (eq. (alpha_beta_constr)); delta = 0 gives e = (0, 0, l_z).
"""
import numpy as np
import pytest

from oracle import am


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _plan(a, b, rho=1.0):
    return am.make_plan(2, 8, 11, 2.0, a, b, rho)


def _scaled_distance(plan, delta):
    return np.sqrt((delta[..., 0] / plan.a) ** 2 + (delta[..., 1] / plan.a) ** 2
                   + (delta[..., 2] / plan.b) ** 2)


@pytest.mark.parametrize("a,b,rho", [(0.3, 0.6, 1.0), (0.4, 0.8, 2.0), (1.0, 1.0, 0.5)])
def test_delta_equals_s_times_e(a, b, rho):
    plan = _plan(a, b, rho)
    delta = _rng(1).standard_normal((500, 1, 3))
    delta[:7, 0, :2] = 0.0                     # purely vertical pairs (cos alpha undefined)
    delta[7:12, 0, 0] = 0.0                    # dx = 0
    al, be = am.step_alpha_beta(plan, delta)
    e = am.spheroid_direction(plan, al, be)
    s = _scaled_distance(plan, delta)
    np.testing.assert_allclose(s[..., None] * e, delta, atol=1e-14)
    assert np.all(al >= -np.pi) and np.all(al <= np.pi)
    assert np.all(be >= 0.0) and np.all(be <= np.pi)


def test_zero_difference_direction():
    plan = _plan(0.3, 0.6)
    al, be = am.step_alpha_beta(plan, np.zeros((1, 1, 3)))
    np.testing.assert_array_equal(am.spheroid_direction(plan, al, be)[0, 0], [0.0, 0.0, 0.6])


@pytest.mark.parametrize("seed", range(6))
def test_d_step_brute_force(seed):
    rng = _rng(100 + seed)
    plan = _plan(rng.uniform(0.2, 1.0), rng.uniform(0.2, 1.0), rng.uniform(0.5, 3.0))
    delta = rng.standard_normal((1, 1, 3)) * rng.uniform(0.05, 2.0)
    lam = rng.standard_normal((1, 1, 3)) * 2.0
    al = rng.uniform(-np.pi, np.pi, (1, 1))
    be = rng.uniform(0, np.pi, (1, 1))
    d = am.step_d(plan, delta, al, be, lam)[0, 0]
    e = am.spheroid_direction(plan, al, be)[0, 0]
    grid = np.linspace(1.0, 30.0, 290001)
    obj = np.sum((delta[0, 0][None, :] - grid[:, None] * e[None, :] + lam[0, 0] / plan.rho) ** 2, axis=1)
    assert abs(grid[np.argmin(obj)] - d) <= 2e-4 + 1e-9
    assert d >= 1.0


def _angle_grid_argmin(plan, delta, d, lam, na=1441, nb=721):
    al = np.linspace(-np.pi, np.pi, na)
    be = np.linspace(0.0, np.pi, nb)
    A, B = np.meshgrid(al, be, indexing="ij")
    e = am.spheroid_direction(plan, A, B)
    r = delta[None, None, :] - d * e + lam[None, None, :] / plan.rho
    obj = np.sum(r * r, axis=-1)
    k = np.unravel_index(np.argmin(obj), obj.shape)
    return e[k], obj[k]


@pytest.mark.parametrize("seed", range(5))
def test_alpha_beta_brute_force_spheres(seed):
    rng = _rng(200 + seed)
    r0 = rng.uniform(0.3, 1.5)
    plan = _plan(r0, r0)
    delta = rng.standard_normal(3)
    d = rng.uniform(1.0, 3.0)
    al, be = am.step_alpha_beta(plan, delta[None, None, :])
    e_cf = am.spheroid_direction(plan, al, be)[0, 0]
    e_grid, _ = _angle_grid_argmin(plan, delta, d, np.zeros(3))
    # grid spacing pi/720 in both angles: directions agree to a few spacings (times the radius)
    assert np.max(np.abs(e_cf - e_grid)) < 3 * np.pi / 720 * r0


@pytest.mark.parametrize("seed", range(3))
def test_alpha_beta_spheroid_gap_is_nonnegative(seed):
    """For spheroids the closed form is the paper's approximate step: its objective is
    never below the grid optimum by more than the grid resolution allows."""
    rng = _rng(300 + seed)
    plan = _plan(0.3, 0.6)
    delta = rng.standard_normal(3) * 0.5
    lam = rng.standard_normal(3) * 0.2
    d = rng.uniform(1.0, 2.0)
    al, be = am.step_alpha_beta(plan, delta[None, None, :])
    e_cf = am.spheroid_direction(plan, al, be)[0, 0]
    obj_cf = np.sum((delta - d * e_cf + lam / plan.rho) ** 2)
    _, obj_grid = _angle_grid_argmin(plan, delta, d, lam)
    assert obj_cf >= obj_grid - 1e-4


def test_noncolliding_pairs_are_fixed():
    plan = _plan(0.3, 0.6)
    rng = _rng(5)
    delta = rng.standard_normal((400, 1, 3))
    s = _scaled_distance(plan, delta)
    delta = delta[s >= 1.0][:, None, :]
    lam = np.zeros_like(delta)
    al, be = am.step_alpha_beta(plan, delta)
    d = am.step_d(plan, delta, al, be, lam)
    np.testing.assert_allclose(d, _scaled_distance(plan, delta), rtol=1e-14)
    f = am.constraint_residual(plan, delta, al, be, d)
    np.testing.assert_allclose(f, 0.0, atol=1e-14)


def test_unclipped_multiplier_orthogonality():
    """For d > 1 the d-step is the unconstrained minimiser, so e^T (lambda + rho f_c) = 0."""
    plan = _plan(0.4, 0.8, 1.7)
    rng = _rng(6)
    delta = rng.standard_normal((2000, 1, 3))
    lam = rng.standard_normal((2000, 1, 3))
    al, be = am.step_alpha_beta(plan, delta)
    d = am.step_d(plan, delta, al, be, lam)
    f = am.constraint_residual(plan, delta, al, be, d)
    lam1 = am.step_lambda(plan, lam, f)
    e = am.spheroid_direction(plan, al, be)
    dot = np.sum(e * lam1, axis=-1)
    free = d > 1.0
    assert free.sum() > 100 and (~free).sum() > 100
    np.testing.assert_allclose(dot[free], 0.0, atol=1e-12)
    assert np.all(d >= 1.0)


@pytest.mark.parametrize("seed", range(5))
def test_shifted_projection_is_exact_for_spheres(seed):
    """Projecting delta + lambda/rho: for spheres the closed form is the exact minimiser
    of the step-(step_alpha) objective at any multipliers (2-D grid search)."""
    rng = _rng(500 + seed)
    r0 = rng.uniform(0.3, 1.5)
    plan = _plan(r0, r0, rng.uniform(0.5, 2.0))
    delta = rng.standard_normal(3)
    lam = rng.standard_normal(3) * 0.7
    d = rng.uniform(1.0, 3.0)
    al, be = am.step_alpha_beta(plan, delta[None, None, :], lam[None, None, :], shifted=True)
    e_cf = am.spheroid_direction(plan, al, be)[0, 0]
    e_grid, _ = _angle_grid_argmin(plan, delta, d, lam)
    assert np.max(np.abs(e_cf - e_grid)) < 3 * np.pi / 720 * r0


def test_shifted_projection_reduces_to_plain_at_zero_multipliers():
    plan = _plan(0.3, 0.6)
    delta = _rng(8).standard_normal((50, 4, 3))
    lam = np.zeros_like(delta)
    a1, b1 = am.step_alpha_beta(plan, delta)
    a2, b2 = am.step_alpha_beta(plan, delta, lam, shifted=True)
    np.testing.assert_array_equal(a1, a2)
    np.testing.assert_array_equal(b1, b2)
