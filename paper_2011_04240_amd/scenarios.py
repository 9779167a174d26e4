"""Seeded synthetic start/goal generators (inputs only, none of the method's arithmetic).

These stand in for the paper's benchmarks of Sec. IV-B: agents on a circle or
sphere swapping to antipodal positions (Fig. "square_benchmark"), and random
start/goal positions in a box (Fig. "random_benchmark").  The paper's own
dataset is not available; every instance here is generated from a seed with
NumPy's PCG64 generator.  This module is the one piece shared by the oracle
tests and the GPU path: it only produces positions, counts and arrival times.
"""
import numpy as np


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def swap_circle(n, radius=3.0, jitter=0.05, seed=0):
    """Starts evenly on a horizontal circle (z = 0), goals antipodal; uniform +-jitter
    drawn independently for every coordinate of starts and goals."""
    rng = _rng(seed)
    ang = 2.0 * np.pi * np.arange(n) / n
    base = np.stack([radius * np.cos(ang), radius * np.sin(ang), np.zeros(n)], axis=1)
    starts = base + rng.uniform(-jitter, jitter, size=(n, 3))
    goals = -base + rng.uniform(-jitter, jitter, size=(n, 3))
    return starts, goals


def swap_sphere(n, radius=4.0, jitter=0.05, seed=0):
    """Starts on a sphere by a Fibonacci (golden-angle) lattice, goals antipodal, +-jitter."""
    rng = _rng(seed)
    k = np.arange(n) + 0.5
    z = 1.0 - 2.0 * k / n
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = np.pi * (3.0 - np.sqrt(5.0)) * np.arange(n)
    base = radius * np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)
    starts = base + rng.uniform(-jitter, jitter, size=(n, 3))
    goals = -base + rng.uniform(-jitter, jitter, size=(n, 3))
    return starts, goals


def _poisson_disk(rng, n, box, min_sep, max_tries=200000):
    pts = np.zeros((0, 3))
    tries = 0
    while pts.shape[0] < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("rejection sampling did not place %d points in box %s" % (n, box))
        p = rng.uniform(0.0, 1.0, size=3) * np.asarray(box)
        if pts.shape[0] == 0 or np.min(np.linalg.norm(pts - p, axis=1)) >= min_sep:
            pts = np.vstack([pts, p])
    return pts


def random_box(n, box=(10.0, 10.0, 5.0), min_sep=1.0, seed=0):
    """Starts and goals drawn independently and uniformly in the box by rejection
    sampling: a point is kept when it is at least min_sep from every point already
    kept in the same set."""
    rng = _rng(seed)
    starts = _poisson_disk(rng, n, box, min_sep)
    goals = _poisson_disk(rng, n, box, min_sep)
    return starts, goals


def density_box(n, ref_n=64, ref_box=(10.0, 10.0, 5.0)):
    """Box with the 2:2:1 aspect of ref_box whose volume scales with n (same agent density)."""
    vol = np.prod(ref_box) * n / ref_n
    s = (vol / 4.0) ** (1.0 / 3.0)
    return (2.0 * s, 2.0 * s, s)


def random_density_box(n, min_sep=1.0, seed=0):
    return random_box(n, box=density_box(n), min_sep=min_sep, seed=seed)


def packed_cube(n, side=0.2, seed=0):
    """Starts and goals drawn independently and uniformly in a cube of the given side,
    no separation: with side 0.2 m every pair of agents of semi-axes (0.3, 0.6) m
    overlaps at both ends of the horizon (a stress case in which every pair carries a
    multiplier, not a feasible plan)."""
    rng = _rng(seed)
    return rng.uniform(0.0, side, size=(n, 3)), rng.uniform(0.0, side, size=(n, 3))


def agent_counts(count, choices, seed=0):
    """Seeded uniform draw of agent counts from `choices`."""
    rng = _rng(seed)
    return [int(x) for x in rng.choice(np.asarray(choices), size=count)]


def poisson_arrivals(rate, count, seed=0):
    """Arrival times (s) of a Poisson process: cumulative exponential gaps of mean 1/rate."""
    rng = _rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


def obstacle_box(n, n_obs, r_range=(0.2, 0.5), agent=(0.15, 0.3), clearance=1.2, min_sep=1.0, seed=0):
    """Random-box starts and goals at the n = 64 density plus n_obs static spherical
    obstacles (radius uniform in r_range) placed uniformly in the same box, each kept
    away from every start and goal (scaled distance >= clearance in its own clearance
    spheroid).  Returns starts, goals and obstacles [n_obs][x, y, z, l_xy, l_z] where
    (l_xy, l_z) = agent semi-axes + obstacle radius."""
    starts, goals = random_density_box(n, min_sep=min_sep, seed=seed)
    box = np.asarray(density_box(n))
    rng = _rng(seed + 7919)
    pts = np.concatenate([starts, goals])
    obs = []
    tries = 0
    while len(obs) < n_obs:
        tries += 1
        if tries > 200000:
            raise RuntimeError("could not place %d obstacles" % n_obs)
        r = rng.uniform(*r_range)
        c = rng.uniform(0.0, 1.0, 3) * box
        lxy, lz = agent[0] + r, agent[1] + r
        d = pts - c
        s2 = (d[:, 0] ** 2 + d[:, 1] ** 2) / lxy ** 2 + d[:, 2] ** 2 / lz ** 2
        if np.all(s2 >= clearance ** 2):
            obs.append([c[0], c[1], c[2], lxy, lz])
    return starts, goals, np.asarray(obs, dtype=np.float64).reshape(-1, 5)
