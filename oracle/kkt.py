"""Matrices of the x/y/z QP step and their offline inverse, Sec. III-B.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Everything here follows the matrix form of step (step_x_3d):
  * A      -- boundary rows [P_1; Pdot_1; Pddot_1; P_m; Pdot_m; Pddot_m] (the A of
              A_eq = diag(A, ..., A)), with b_eq = [x0, v0, a0, xf, vf, af].
  * A_fc   -- the stacked collision blocks A_r of eq. (A_f): for agent r the rows
              of every pair (r, j > r), P in the columns of agent r and -P in the
              columns of agent j.  Row order: pair (r, j) major, time minor.
              With static obstacles (Sec. IV-A, circumscribing spheres) each agent r
              also has one row block per obstacle o, P in the columns of agent r only
              (the obstacle's position is data and moves to b); these blocks follow
              all agent pairs, agent major, obstacle minor.
  * K      -- the KKT matrix of eq. (kkt_step_x),
              [[Q_x + rho A_fc^T A_fc, A_eq^T], [A_eq, 0]],  Q_x = diag(Pddot^T Pddot)
              exactly as printed there.
  * K^{-1} -- computed once (Remarks 1-2): it depends on n, rho and P only.
"""
import numpy as np


def boundary_matrix(P, Pd, Pdd):
    """A (6 x n_coef): first and last rows of P, P-dot, P-ddot."""
    return np.vstack([P[0], Pd[0], Pdd[0], P[-1], Pd[-1], Pdd[-1]])


def boundary_rhs(start, goal):
    """b_eq for one agent and one axis: rest-to-rest, zero velocity and acceleration."""
    return np.array([start, 0.0, 0.0, goal, 0.0, 0.0], dtype=np.float64)


def pair_index(n):
    """Unordered pairs (i, j), i < j, in the row order of A_fc: i major, j minor."""
    I, J = np.triu_indices(n, k=1)
    return I.astype(np.int64), J.astype(np.int64)


def collision_matrix(P, n, n_obs=0):
    """Literal A_fc of eq. (A_f): vertical stack of the blocks A_r, r = 0..n-2.

    A_r holds n-1-r copies of P stacked in the columns of agent r and a block
    diagonal of -P over the columns of agents r+1..n-1.  Size (T*n(n-1)/2) x (n*n_coef),
    plus T*n*n_obs obstacle rows.  Only meant for small n (it is dense).
    """
    T, nv = P.shape
    blocks = []
    for r in range(n - 1):
        k = n - 1 - r
        Ar = np.zeros((k * T, n * nv))
        for q in range(k):
            j = r + 1 + q
            Ar[q * T:(q + 1) * T, r * nv:(r + 1) * nv] = P
            Ar[q * T:(q + 1) * T, j * nv:(j + 1) * nv] = -P
        blocks.append(Ar)
    for r in range(n):
        for o in range(n_obs):
            Ao = np.zeros((T, n * nv))
            Ao[:, r * nv:(r + 1) * nv] = P
            blocks.append(Ao)
    return np.vstack(blocks)


def collision_gram(P, n, n_obs=0):
    """A_fc^T A_fc accumulated pair by pair: each pair (i, j) adds P^T P to the
    (i,i) and (j,j) blocks and -P^T P to the (i,j) and (j,i) blocks; each
    agent-obstacle pair (i, o) adds P^T P to the (i,i) block."""
    nv = P.shape[1]
    PtP = P.T @ P
    G = np.zeros((n * nv, n * nv))
    for i, j in zip(*pair_index(n)):
        si, sj = slice(i * nv, (i + 1) * nv), slice(j * nv, (j + 1) * nv)
        G[si, si] += PtP
        G[sj, sj] += PtP
        G[si, sj] -= PtP
        G[sj, si] -= PtP
    for i in range(n):
        si = slice(i * nv, (i + 1) * nv)
        for _ in range(n_obs):
            G[si, si] += PtP
    return G


def collision_transpose_apply(P, n, b, n_obs=0):
    """A_fc^T b for b of shape (n_pairs + n n_obs, T) (rows in A_fc order), returned
    as (n, n_coef).

    Uses the block structure of A_fc: pair (i, j) contributes +P^T b_p to agent i
    and -P^T b_p to agent j; agent-obstacle row (i, o) contributes +P^T b to agent i.
    """
    I, J = pair_index(n)
    npairs = len(I)
    PtB = b @ P                              # row p holds (P^T b_p)^T
    out = np.zeros((n, P.shape[1]))
    np.add.at(out, I, PtB[:npairs])
    np.add.at(out, J, -PtB[:npairs])
    if n_obs:
        np.add.at(out, np.repeat(np.arange(n), n_obs), PtB[npairs:])
    return out


def kkt_matrix(P, Pdd, A, n, rho, literal=False, n_obs=0):
    """K of eq. (kkt_step_x) for n agents (and n_obs static obstacles), unknowns
    ordered [c (agent-major); nu (agent-major)]."""
    nv, nb = P.shape[1], A.shape[0]
    if literal:
        Afc = collision_matrix(P, n, n_obs)
        gram = Afc.T @ Afc
    else:
        gram = collision_gram(P, n, n_obs)
    H = np.kron(np.eye(n), Pdd.T @ Pdd) + rho * gram
    Aeq = np.kron(np.eye(n), A)
    K = np.zeros((n * (nv + nb), n * (nv + nb)))
    K[:n * nv, :n * nv] = H
    K[:n * nv, n * nv:] = Aeq.T
    K[n * nv:, :n * nv] = Aeq
    return K


def boundary_only_kkt(Pdd, A):
    """Per-agent KKT matrix of min 1/2 c^T Pddot^T Pddot c s.t. A c = b_eq (no collision term)."""
    nv, nb = Pdd.shape[1], A.shape[0]
    K0 = np.zeros((nv + nb, nv + nb))
    K0[:nv, :nv] = Pdd.T @ Pdd
    K0[:nv, nv:] = A.T
    K0[nv:, :nv] = A
    return K0


def invert(K):
    """Offline FP64 inverse (Remark 1)."""
    return np.linalg.inv(K)
