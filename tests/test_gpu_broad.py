"""The FP32 pairwise kernel's broad phase against the all-general pass, bit for bit.

Per work item the kernel bounds every agent's positions over the item's instants by a box;
a row whose boxes keep s^2 above the shortcut threshold at every instant and whose
multipliers are flagged all +0 is skipped, and when at most half the rows are kept only
they are worked through (the row list).  With the parity outputs on, every row takes the
general branch in the streaming order instead.  Both must give the same iterates: sparse
random-box problems (n = 64, T = 100, the row list) at two tile shapes, and problems with
static obstacles (the obstacle rows of the broad phase), over 40 iterations each.
"""
import numpy as np
import pytest

from paper_2011_04240_amd import mato
from paper_2011_04240_amd import scenarios as sc

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def _compare(plans, starts, goals, tiles, obstacles=None, chunks=4, per=10):
    kw = {} if obstacles is None else {"obstacles_list": obstacles}
    fast = mato.Batch(plans, starts, goals, **kw)
    general = mato.Batch(plans, starts, goals, **kw)
    if tiles is not None:
        fast.set_tiles(*tiles)
        general.set_tiles(*tiles)
    general.debug(True)
    for _ in range(chunks):
        fast.step(per, use_graph=False)
        general.step(per, use_graph=False)
    nz = 0
    for q in range(len(plans)):
        a, b = fast.get_state(q), general.get_state(q)
        np.testing.assert_array_equal(a["lam"], b["lam"])
        np.testing.assert_array_equal(a["c"], b["c"])
        np.testing.assert_array_equal(fast.residuals(q)[0], general.residuals(q)[0])
        np.testing.assert_array_equal(fast.residuals(q)[2], general.residuals(q)[2])
        nz += np.count_nonzero(a["lam"])
    return nz


@pytest.mark.parametrize("tiles", [(16384, 256), (32768, 512)])
def test_broad_phase_random_box_bitwise(tiles):
    say("broad phase, random box n=64 T=100, tiles", tiles)
    scen = [sc.random_box(64, seed=300 + k) for k in range(4)]
    plan = mato.Plan(64, 100, 11, 10.0, 0.3, 0.6, 1.0, "fp32")
    nz = _compare([plan] * 4, [s for s, _ in scen], [g for _, g in scen], tiles)
    assert nz > 0                                   # some pairs collide: the general branch is exercised


def test_broad_phase_obstacles_bitwise():
    say("broad phase with obstacles")
    cases = [(12, 6, 1), (20, 3, 2)]
    scen = [sc.obstacle_box(n, k, seed=sd) for n, k, sd in cases]
    plans = [mato.Plan(n, 60, 11, 6.0, 0.3, 0.6, 1.0, "fp32", n_obs=k) for n, k, _ in cases]
    for q in range(2):
        _compare([plans[q]], [scen[q][0]], [scen[q][1]], (1024, 256), obstacles=[scen[q][2]])
