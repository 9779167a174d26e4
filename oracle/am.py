"""Algorithm 1 (alternating minimisation), Sec. III-A/III-B, step by step in FP64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Array conventions (shared with the library's exposed layouts, not with its code):
  c      (n, 3, n_coef)   coefficients, [agent][axis][coef], axis order x, y, z
  X      (n, 3, T)        positions P c
  lam, delta, e, f_c      (n_rows, T, 3)  row p = pair (i, j), i < j, in A_fc row order,
                          then (with obstacles) row n_pairs + i n_obs + o = agent i, obstacle o
  d, alpha, beta          (n_rows, T)
  obs                     (n_obs, 5)  static obstacle: centre x, y, z and the combined
                          agent-obstacle semi-axes l_xy, l_z of its clearance spheroid

Readings of points the paper leaves open (each used below):
  * pairs are unordered, i < j, and delta = X_i - X_j (eq. (A_f) stacks n-r copies);
  * the linear term of the x-step is rho A_fc^T b (the rho follows from expanding
    the penalty of eq. (step_x_3d)); Q_x = Pddot^T Pddot as printed in eq. (kkt_step_x);
  * beta = atan2(hypot(dx, dy)/l_xy, dz/l_z), equal to eq. (sphere_project) wherever
    cos(alpha) != 0 and defined where it is 0; delta = 0 exactly gives alpha = beta = 0;
  * a variant (shifted=True) projects delta + lambda/rho instead of delta;
  * the direction convention of e follows f_c, eq. (sphere_proposed):
    e = (l_xy sin b cos a, l_xy sin b sin a, l_z cos b);
  * d is clipped to d >= 1 as eq. (alpha_beta_constr) states;
  * initialisation: lambda = 0, c from the boundary-only minimum-acceleration
    problem, then alpha, beta, d from steps (sphere_project)/(step_d) at those positions;
  * static obstacles (Sec. IV-A: circumscribing spheres) are rows of the same form
    with delta = X_i - x_o and the obstacle's own semi-axes; their b carries x_o;
  * stop after `iters` iterations or once max ||f_c|| falls below `tol`.
"""
from dataclasses import dataclass, field

import numpy as np

from . import basis as _basis
from . import kkt as _kkt


@dataclass
class Plan:
    n: int
    T: int
    n_coef: int
    t_final: float
    a: float          # l_xy
    b: float          # l_z
    rho: float
    P: np.ndarray
    Pd: np.ndarray
    Pdd: np.ndarray
    A: np.ndarray
    K: np.ndarray
    Kinv: np.ndarray
    K0inv: np.ndarray
    I: np.ndarray
    J: np.ndarray
    n_obs: int = 0

    @property
    def n_pairs(self):
        return self.n * (self.n - 1) // 2

    @property
    def n_rows(self):
        return self.n_pairs + self.n * self.n_obs


def make_plan(n, T, n_coef=11, t_final=10.0, a=0.3, b=0.6, rho=1.0, literal=None, n_obs=0):
    """Offline part: basis, K of eq. (kkt_step_x) and its FP64 inverse (Remarks 1-2).
    K depends on the number of static obstacles, not on where they are."""
    if literal is None:
        literal = n <= 8
    P, Pd, Pdd = _basis.basis_matrices(n_coef, T, t_final)
    A = _kkt.boundary_matrix(P, Pd, Pdd)
    K = _kkt.kkt_matrix(P, Pdd, A, n, rho, literal=literal, n_obs=n_obs)
    Kinv = _kkt.invert(K)
    K0inv = _kkt.invert(_kkt.boundary_only_kkt(Pdd, A))
    I, J = _kkt.pair_index(n)
    return Plan(n, T, n_coef, float(t_final), float(a), float(b), float(rho),
                P, Pd, Pdd, A, K, Kinv, K0inv, I, J, int(n_obs))


def _obstacles(plan, obs):
    obs = np.zeros((0, 5)) if obs is None else np.asarray(obs, dtype=np.float64).reshape(-1, 5)
    assert obs.shape[0] == plan.n_obs, "the plan was made for %d obstacles" % plan.n_obs
    return obs


def row_dims(plan, obs=None):
    """Semi-axes (l_xy, l_z) of every row, each of shape (n_rows, 1): the agent pair's
    (a, b), then each agent-obstacle row's own."""
    obs = _obstacles(plan, obs)
    lxy = np.concatenate([np.full(plan.n_pairs, plan.a), np.tile(obs[:, 3], plan.n)])
    lz = np.concatenate([np.full(plan.n_pairs, plan.b), np.tile(obs[:, 4], plan.n)])
    return lxy[:, None], lz[:, None]


def boundary_rhs_all(starts, goals):
    """b_eq for every agent and axis, shape (n, 3, 6)."""
    starts = np.asarray(starts, dtype=np.float64)
    goals = np.asarray(goals, dtype=np.float64)
    n = starts.shape[0]
    beq = np.zeros((n, 3, 6))
    for i in range(n):
        for ax in range(3):
            beq[i, ax] = _kkt.boundary_rhs(starts[i, ax], goals[i, ax])
    return beq


def spheroid_direction(plan, alpha, beta, dims=None):
    """e(alpha, beta) = (l_xy sin b cos a, l_xy sin b sin a, l_z cos b), eq. (sphere_proposed).
    dims = (l_xy, l_z) broadcastable to alpha (default: the plan's a, b)."""
    lxy, lz = (plan.a, plan.b) if dims is None else dims
    return np.stack([lxy * np.sin(beta) * np.cos(alpha),
                     lxy * np.sin(beta) * np.sin(alpha),
                     lz * np.cos(beta)], axis=-1)


def collision_rhs(plan, d, alpha, beta, lam, obs=None):
    """b_fc of eq. (b_f) for the three axes: d e - lambda / rho, shape (n_rows, T, 3);
    an obstacle row's target also carries the obstacle's centre."""
    b = d[..., None] * spheroid_direction(plan, alpha, beta, row_dims(plan, obs)) - lam / plan.rho
    if plan.n_obs:
        obs = _obstacles(plan, obs)
        b[plan.n_pairs:] += np.tile(obs[:, :3], (plan.n, 1))[:, None, :]
    return b


def linear_term(plan, b_fc):
    """rho A_fc^T b_fc per axis, shape (n, 3, n_coef)."""
    g = np.zeros((plan.n, 3, plan.n_coef))
    for ax in range(3):
        g[:, ax, :] = plan.rho * _kkt.collision_transpose_apply(plan.P, plan.n, b_fc[:, :, ax], plan.n_obs)
    return g


def step_xyz(plan, b_fc, beq):
    """Steps (step_x_3d)-(step_z_3d) through eq. (kkt_step_x): [c; nu] = K^{-1} [rho A_fc^T b; b_eq].

    The three axes share K (only the right-hand side differs).  Returns (c, nu, g).
    """
    n, nv = plan.n, plan.n_coef
    g = linear_term(plan, b_fc)
    c = np.zeros((n, 3, nv))
    nu = np.zeros((n, 3, plan.A.shape[0]))
    for ax in range(3):
        q = np.concatenate([g[:, ax, :].ravel(), beq[:, ax, :].ravel()])
        sol = plan.Kinv @ q
        c[:, ax, :] = sol[:n * nv].reshape(n, nv)
        nu[:, ax, :] = sol[n * nv:].reshape(n, -1)
    return c, nu, g


def positions(plan, c):
    """X = P c for every agent and axis, eq. (param); shape (n, 3, T)."""
    return c @ plan.P.T


def pair_differences(plan, X, obs=None):
    """delta_p(t) = X_i(t) - X_j(t) for p = (i, j), i < j, then X_i(t) - x_o for every
    agent i and obstacle o; shape (n_rows, T, 3)."""
    d = np.transpose(X[plan.I] - X[plan.J], (0, 2, 1))
    if not plan.n_obs:
        return d
    obs = _obstacles(plan, obs)
    do = np.transpose(X, (0, 2, 1))[:, None, :, :] - obs[None, :, None, :3]      # (n, n_obs, T, 3)
    return np.concatenate([d, do.reshape(-1, X.shape[2], 3)])


def step_alpha_beta(plan, delta, lam=None, shifted=False, dims=None):
    """Closed-form alpha, beta of eq. (sphere_project) (projection onto the spheroid).

    shifted=True is the variant that projects delta + lambda/rho, the point the
    objective of eq. (step_alpha) actually measures against (exact for spheres)."""
    lxy, lz = (plan.a, plan.b) if dims is None else dims
    if shifted:
        delta = delta + lam / plan.rho
    dx, dy, dz = delta[..., 0], delta[..., 1], delta[..., 2]
    alpha = np.arctan2(dy, dx)
    beta = np.arctan2(np.hypot(dx, dy) / lxy, dz / lz)
    zero = (dx == 0) & (dy == 0) & (dz == 0)
    alpha = np.where(zero, 0.0, alpha)
    beta = np.where(zero, 0.0, beta)
    return alpha, beta


def step_d(plan, delta, alpha, beta, lam, dims=None):
    """Eq. (step_d): the scalar QP per pair and instant, solved in closed form, clipped to d >= 1."""
    e = spheroid_direction(plan, alpha, beta, dims)
    dstar = np.sum(e * (delta + lam / plan.rho), axis=-1) / np.sum(e * e, axis=-1)
    return np.maximum(1.0, dstar)


def constraint_residual(plan, delta, alpha, beta, d, dims=None):
    """f_c of eq. (sphere_proposed): delta - d e, shape (n_rows, T, 3)."""
    return delta - d[..., None] * spheroid_direction(plan, alpha, beta, dims)


def step_lambda(plan, lam, f_c):
    """Eq. (lag_update): lambda <- lambda + rho f_c."""
    return lam + plan.rho * f_c


@dataclass
class State:
    c: np.ndarray
    lam: np.ndarray
    d: np.ndarray
    alpha: np.ndarray
    beta: np.ndarray
    beq: np.ndarray
    nu: np.ndarray = None
    g: np.ndarray = None
    X: np.ndarray = None
    delta: np.ndarray = None
    f_c: np.ndarray = None
    history: dict = field(default_factory=lambda: {k: [] for k in
                          ("r_max", "r_rms", "cost", "bnd_res", "kkt_res")})
    obs: np.ndarray = None

    def proj(self, plan):
        """d e, the point on the spheroid the multipliers are measured against."""
        return self.d[..., None] * spheroid_direction(plan, self.alpha, self.beta, row_dims(plan, self.obs))


def initial_state(plan, starts, goals, obs=None):
    """Initialisation of Algorithm 1 (its first statement): lambda = 0, boundary-only c,
    then alpha, beta and d = max(1, d*) at the resulting positions."""
    obs = _obstacles(plan, obs)
    dims = row_dims(plan, obs)
    beq = boundary_rhs_all(starts, goals)
    n, nv = plan.n, plan.n_coef
    c = np.zeros((n, 3, nv))
    for i in range(n):
        for ax in range(3):
            sol = plan.K0inv @ np.concatenate([np.zeros(nv), beq[i, ax]])
            c[i, ax] = sol[:nv]
    X = positions(plan, c)
    delta = pair_differences(plan, X, obs)
    lam = np.zeros((plan.n_rows, plan.T, 3))
    alpha, beta = step_alpha_beta(plan, delta, dims=dims)
    d = step_d(plan, delta, alpha, beta, lam, dims)
    return State(c=c, lam=lam, d=d, alpha=alpha, beta=beta, beq=beq, X=X, delta=delta, obs=obs)


def smoothness_cost(plan, c):
    """Sum over agents, axes and instants of the squared acceleration, eq. (cost_proposed)."""
    return float(np.sum((c @ plan.Pdd.T) ** 2))


def iterate_rhs(plan, b_fc, lam, beq, shifted=False, obs=None):
    """One pass of the while-loop of Algorithm 1 given b_fc (eq. (b_f)) and lambda^k.

    Returns a dict with every intermediate: g, c, nu, X, delta, alpha, beta, d, e,
    proj = d e, f_c, lam (= lambda^{k+1}) and the residual records.
    shifted selects the projection variant of step_alpha_beta.
    """
    dims = row_dims(plan, obs)
    c, nu, g = step_xyz(plan, b_fc, beq)
    X = positions(plan, c)
    delta = pair_differences(plan, X, obs)
    alpha, beta = step_alpha_beta(plan, delta, lam, shifted, dims)
    d = step_d(plan, delta, alpha, beta, lam, dims)
    f_c = constraint_residual(plan, delta, alpha, beta, d, dims)
    lam_next = step_lambda(plan, lam, f_c)
    e = spheroid_direction(plan, alpha, beta, dims)
    out = dict(g=g, c=c, nu=nu, X=X, delta=delta, alpha=alpha, beta=beta, d=d, e=e,
               proj=d[..., None] * e, f_c=f_c, lam=lam_next)
    out.update(records(plan, c, nu, g, beq, f_c))
    return out


def records(plan, c, nu, g, beq, f_c):
    """Residual bookkeeping of one iteration: max and RMS of ||f_c||_2 (m), the
    smoothness cost, the boundary residual ||A c - b_eq||_inf and the KKT
    stationarity residual ||H c + A^T nu - rho A_fc^T b||_inf."""
    n, nv = plan.n, plan.n_coef
    norms = np.sqrt(np.sum(f_c * f_c, axis=-1))
    bnd = float(np.max(np.abs(np.einsum('bk,iak->iab', plan.A, c) - beq)))
    kkt = 0.0
    for ax in range(3):
        sol = np.concatenate([c[:, ax, :].ravel(), nu[:, ax, :].ravel()])
        r = plan.K[:n * nv] @ sol - g[:, ax, :].ravel()
        kkt = max(kkt, float(np.max(np.abs(r))))
    return dict(r_max=float(norms.max()) if norms.size else 0.0,
                r_rms=float(np.sqrt(np.mean(norms ** 2))) if norms.size else 0.0,
                cost=smoothness_cost(plan, c), bnd_res=bnd, kkt_res=kkt)


def iterate(plan, st, shifted=False):
    """One iteration of Algorithm 1 from State ^k to State ^{k+1}."""
    b_fc = collision_rhs(plan, st.d, st.alpha, st.beta, st.lam, st.obs)
    out = iterate_rhs(plan, b_fc, st.lam, st.beq, shifted, st.obs)
    nxt = State(c=out["c"], lam=out["lam"], d=out["d"], alpha=out["alpha"], beta=out["beta"],
                beq=st.beq, nu=out["nu"], g=out["g"], X=out["X"], delta=out["delta"],
                f_c=out["f_c"], history=st.history, obs=st.obs)
    for k in nxt.history:
        nxt.history[k].append(out[k])
    return nxt


def solve(plan, starts, goals, iters, tol=0.0, shifted=False, obs=None):
    """Algorithm 1: initialise, then iterate until `iters` passes or max ||f_c|| < tol."""
    st = initial_state(plan, starts, goals, obs)
    for _ in range(iters):
        st = iterate(plan, st, shifted)
        if st.history["r_max"][-1] < tol:
            break
    return st


def solve_schedule(plans, start_iters, starts, goals, iters, tol=0.0, shifted=False, obs=None):
    """Algorithm 1 with the penalty parameter increased in stages (Sec. IV-A: inverses
    cached for several increasing rho, the larger ones used in later iterations).

    plans[j] (same n, T, basis; its own rho and K^{-1}) is used from iteration
    start_iters[j] on (start_iters[0] = 0, increasing).  Iteration k of stage j uses
    rho_j throughout: b_fc = d e - lambda/rho_j in the x-step, lambda/rho_j in the d
    step, lambda += rho_j f_c.
    """
    assert start_iters[0] == 0 and all(b > a for a, b in zip(start_iters[:-1], start_iters[1:]))
    st = initial_state(plans[0], starts, goals, obs)
    j = 0
    for k in range(iters):
        while j + 1 < len(plans) and k >= start_iters[j + 1]:
            j += 1
        st = iterate(plans[j], st, shifted)
        if st.history["r_max"][-1] < tol:
            break
    return st
