"""GPU edge cases and batching through the C ABI, against the FP64 oracle.

* smallest problem (n = 2, one pair) at the smallest horizon (T = n_coef);
* largest problem (n = MATO_MAX_AGENTS, one instant of all pairs fills the LDS);
* coincident agents (delta = 0 exactly, the alpha = beta = 0 branch);
* uneven-size problems in one batch give bitwise the same iterates as alone;
* error paths: non-finite input, invalid problem index, NOT_CONVERGED warning.
"""
import numpy as np
import pytest

from oracle import am
from paper_2011_04240_amd import mato
from paper_2011_04240_amd import scenarios as sc

pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / (den if den > 0 else 1.0))


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-8), ("fp32", 1e-3)])
def test_two_agents_minimum_horizon(precision, tol):
    say("n=2 T=11", precision)
    s = np.array([[0.0, 0.0, 0.0], [0.3, 0.05, 0.0]])
    g = np.array([[0.3, 0.0, 0.0], [0.0, 0.05, 0.0]])
    op = am.make_plan(2, 11, 11, 2.0, 0.4, 0.8, 1.0)
    st = am.solve(op, s, g, 40)
    b = mato.Batch([mato.Plan(2, 11, 11, 2.0, 0.4, 0.8, 1.0, precision)], [s], [g])
    b.run(40, 0.0, 10)
    r_max, _, cost = b.residuals(0)
    assert rel(b.coeffs(0), st.c) < tol
    assert rel(r_max, st.history["r_max"]) < tol
    assert rel(cost, st.history["cost"]) < tol


def test_largest_problem_single_step():
    n, T = mato.MATO_MAX_AGENTS, 24
    say("n=%d T=%d single step" % (n, T))
    s, g = sc.random_density_box(n, seed=5)
    op = am.make_plan(n, T, 11, 3.0, 0.3, 0.6, 1.0)
    st = am.initial_state(op, s, g)
    st = am.iterate(op, st)
    lam = st.lam.astype(np.float32)
    proj = st.proj(op).astype(np.float32)
    ref = am.iterate_rhs(op, proj.astype(np.float64) - lam.astype(np.float64), lam.astype(np.float64), st.beq)
    b = mato.Batch([mato.Plan(n, T, 11, 3.0, 0.3, 0.6, 1.0, "fp32")], [s], [g])
    b.set_state(0, st.c, lam, proj)
    b.step(1, use_graph=False)
    out = b.get_state(0)
    assert rel(out["c"], ref["c"]) < 1e-5
    assert rel(out["lam"], ref["lam"]) < 1e-5


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-8), ("fp32", 1e-5)])
def test_coincident_agents(precision, tol):
    """Agents 0 and 1 share start and goal: delta is exactly 0 along the boundary-only
    trajectories, so the initial projection takes e = (0, 0, l_z)."""
    say("coincident agents", precision)
    s = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 0.0], [3.0, 0.0, 1.0], [-2.0, 1.0, 0.5]])
    g = np.array([[2.0, 1.0, 0.0], [2.0, 1.0, 0.0], [0.0, 0.0, 1.0], [1.0, -1.0, 0.5]])
    op = am.make_plan(4, 30, 11, 4.0, 0.4, 0.8, 1.0)
    st0 = am.initial_state(op, s, g)
    assert np.all(st0.delta[0] == 0.0)
    b = mato.Batch([mato.Plan(4, 30, 11, 4.0, 0.4, 0.8, 1.0, precision)], [s], [g])
    g_ref = am.linear_term(op, am.collision_rhs(op, st0.d, st0.alpha, st0.beta, st0.lam))
    assert rel(b.linear_term(0), g_ref) < tol
    st = am.solve(op, s, g, 5)
    b.step(5, use_graph=False)
    assert rel(b.coeffs(0), st.c) < (tol if precision == "fp64" else 1e-4)


def test_uneven_batch_matches_alone_bitwise():
    say("uneven batch vs alone")
    ns = [5, 13, 8, 21, 13, 37, 5]
    plans = {n: mato.Plan(n, 40, 11, 5.0, 0.3, 0.6, 1.0, "fp32") for n in set(ns)}
    scen = [sc.random_density_box(n, seed=10 + q) for q, n in enumerate(ns)]
    mix = mato.Batch([plans[n] for n in ns], [x[0] for x in scen], [x[1] for x in scen])
    mix.step(25, use_graph=True)
    mix.sync()
    for q, n in enumerate(ns):
        alone = mato.Batch([plans[n]], [scen[q][0]], [scen[q][1]])
        alone.step(25, use_graph=False)
        a, m = alone.get_state(0), mix.get_state(q)
        np.testing.assert_array_equal(a["c"], m["c"])
        np.testing.assert_array_equal(a["lam"], m["lam"])
        np.testing.assert_array_equal(alone.residuals(0)[0], mix.residuals(q)[0])


def test_large_batch_uploads_match_alone_bitwise():
    """A batch whose creation uploads several MB of boundary data (the engine's pinned staging
    ring wraps many times, and its work list and descriptors take the large-copy path) gives every
    problem exactly the iterates it has alone."""
    say("large batch uploads vs alone")
    n, count = 48, 384      # 30 KB of boundary data per problem; 38 400 work items (614 KB)
    plan = mato.Plan(n, 100, 11, 10.0, 0.3, 0.6, 1.0, "fp32", solve="structured")
    scen = [sc.random_density_box(n, seed=700 + q) for q in range(count)]
    mix = mato.Batch([plan] * count, [x[0] for x in scen], [x[1] for x in scen])
    mix.step(12, use_graph=False)
    mix.sync()
    for q in (0, 17, 200, count - 1):
        alone = mato.Batch([plan], [scen[q][0]], [scen[q][1]])
        alone.step(12, use_graph=False)
        np.testing.assert_array_equal(alone.coeffs(0), mix.coeffs(q))
        np.testing.assert_array_equal(alone.residuals(0)[0], mix.residuals(q)[0])


@pytest.mark.parametrize("precision,count", [("fp32", 2560), ("fp32", 4096), ("bf16", 2560), ("bf16", 4096)])
def test_product_tile_widths_agree_bitwise(precision, count):
    """The FP32 and the BF16 inverse products give the same coefficients bit for bit whatever
    the tile form: 2560 problems of n = 8 take 64-column tiles with two groups of wavefronts
    (240 tiles, fewer than compute units), 4096 take 48-column tiles with one group (512
    tiles), and one problem alone takes 48-column tiles with two groups."""
    say("product tile widths", precision, count)
    n = 8
    plan = mato.Plan(n, 20, 11, 5.0, 0.3, 0.6, 1.0, precision)
    scen = [sc.random_density_box(n, seed=900 + q) for q in range(count)]
    big = mato.Batch([plan] * count, [x[0] for x in scen], [x[1] for x in scen])
    big.step(6, use_graph=False)
    big.sync()
    for q in (0, 1111, count - 1):
        alone = mato.Batch([plan], [scen[q][0]], [scen[q][1]])
        alone.step(6, use_graph=False)
        np.testing.assert_array_equal(alone.coeffs(0), big.coeffs(q))
        np.testing.assert_array_equal(alone.get_state(0)["lam"], big.get_state(q)["lam"])


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_far_pair_shortcut_matches_general_branch_bitwise(precision):
    """A pair with no multiplier that clears the collision set by a margin takes a shortcut in
    the pairwise kernel (d e = delta), and an iteration stores only the multipliers whose bits
    change.  With the debug outputs on, every pair takes the general branch.  Both give the same
    iterates bit for bit on a crowded scene where pairs enter and leave the collision set."""
    say("far-pair shortcut", precision)
    n = 24
    plan = mato.Plan(n, 60, 11, 6.0, 0.3, 0.6, 1.0, precision)
    s, g = sc.swap_circle(n, radius=3.0, seed=5)
    fast, general = mato.Batch([plan], [s], [g]), mato.Batch([plan], [s], [g])
    general.debug(True)
    for _ in range(4):
        fast.step(10, use_graph=False)
        general.step(10, use_graph=False)
        a, b = fast.get_state(0), general.get_state(0)
        np.testing.assert_array_equal(a["lam"], b["lam"])
        np.testing.assert_array_equal(a["c"], b["c"])
    np.testing.assert_array_equal(fast.residuals(0)[0], general.residuals(0)[0])
    lam = fast.get_state(0)["lam"]
    assert 0 < np.count_nonzero(lam) < lam.size // 2      # both branches taken


def test_batch_matches_oracle_per_problem():
    say("uneven batch vs oracle")
    ns = [6, 11, 17]
    scen = [sc.random_density_box(n, seed=40 + q) for q, n in enumerate(ns)]
    b = mato.Batch([mato.Plan(n, 30, 11, 4.0, 0.3, 0.6, 1.0, "fp64") for n in ns],
                   [x[0] for x in scen], [x[1] for x in scen])
    b.run(30, 0.0, 10)
    for q, n in enumerate(ns):
        st = am.solve(am.make_plan(n, 30, 11, 4.0, 0.3, 0.6, 1.0), scen[q][0], scen[q][1], 30)
        assert rel(b.coeffs(q), st.c) < 1e-8
        assert rel(b.residuals(q)[0], st.history["r_max"]) < 1e-8


def test_convergence_stop_and_warning():
    say("tolerance stop")
    s, g = sc.swap_circle(4, seed=0)
    b = mato.Batch([mato.Plan(4, 50, 11, 5.0, 0.4, 0.8, 1.0, "fp64")], [s], [g])
    assert b.run(500, 0.05, 7) == mato.MATO_OK
    it, conv = b.status(0)
    r_max, _, _ = b.residuals(0)
    assert conv and r_max[-1] < 0.05 and np.all(r_max[:-1] >= 0.05) and it == len(r_max)
    ref = am.solve(am.make_plan(4, 50, 11, 5.0, 0.4, 0.8, 1.0), s, g, 500, tol=0.05)
    assert it == len(ref.history["r_max"])
    b2 = mato.Batch([mato.Plan(4, 50, 11, 5.0, 0.4, 0.8, 1.0, "fp32")], [s], [g])
    assert b2.run(5, 1e-9, 5) == mato.MATO_WARN_NOT_CONVERGED


def test_error_paths():
    say("error paths")
    p = mato.Plan(4, 20, 11, 3.0, 0.4, 0.8, 1.0, "fp32")
    s, g = sc.swap_circle(4, seed=1)
    bad = s.copy()
    bad[2, 1] = np.nan
    with pytest.raises(mato.MatoError) as e:
        mato.Batch([p], [bad], [g])
    assert e.value.status == mato.MATO_ERR_NONFINITE
    b = mato.Batch([p], [s], [g])
    with pytest.raises(mato.MatoError) as e:
        mato.mato_batch_coeffs(b.handle, 1, np.empty((4, 3, 11)))
    assert e.value.status == mato.MATO_ERR_INVALID_ARG
    p64 = mato.Plan(4, 20, 11, 3.0, 0.4, 0.8, 1.0, "fp64")
    with pytest.raises(mato.MatoError):
        mato.Batch([p, p64], [s, s], [g, g])          # mixed precisions


def test_autotune_keeps_results():
    say("autotune")
    ns = [8, 24]
    scen = [sc.random_density_box(n, seed=70 + q) for q, n in enumerate(ns)]
    plans = [mato.Plan(n, 50, 11, 5.0, 0.3, 0.6, 1.0, "fp32") for n in ns]
    ref = mato.Batch(plans, [x[0] for x in scen], [x[1] for x in scen])
    ref.step(10)
    tuned = mato.Batch(plans, [x[0] for x in scen], [x[1] for x in scen])
    ipw, thr = tuned.autotune()
    assert thr in (256, 512, 1024) and ipw >= 1
    tuned.step(10)
    for q in range(2):
        np.testing.assert_array_equal(ref.get_state(q)["lam"], tuned.get_state(q)["lam"])


def test_fp64_lds_limit():
    """FP64 keeps 3 (n + n(n-1)/2) doubles per instant in LDS: n = 116 does not fit."""
    say("fp64 lds limit")
    s, g = sc.random_density_box(116, seed=5)
    p = mato.Plan(116, 12, 11, 2.0, 0.3, 0.6, 1.0, "fp64", solve="structured")
    with pytest.raises(mato.MatoError) as e:
        mato.Batch([p], [s], [g])
    assert e.value.status == mato.MATO_ERR_UNSUPPORTED


def test_fp64_largest_n_matches_oracle():
    say("fp64 n115")
    n, T = 115, 12
    s, g = sc.random_density_box(n, seed=6)
    ref = am.solve(am.make_plan(n, T, 11, 2.0, 0.3, 0.6, 1.0), s, g, 3)
    b = mato.Batch([mato.Plan(n, T, 11, 2.0, 0.3, 0.6, 1.0, "fp64", solve="structured")], [s], [g])
    b.step(3, use_graph=False)
    r_max, _, _ = b.residuals(0)
    assert rel(b.coeffs(0), ref.c) < 1e-9
    assert rel(r_max, ref.history["r_max"]) < 1e-8


def test_mixed_solve_kinds_rejected():
    say("mixed solve kinds")
    s, g = sc.swap_circle(4, seed=1)
    pd = mato.Plan(4, 20, 11, 3.0, 0.4, 0.8, 1.0, "fp32")
    ps = mato.Plan(4, 20, 11, 3.0, 0.4, 0.8, 1.0, "fp32", solve="structured")
    with pytest.raises(mato.MatoError) as e:
        mato.Batch([pd, ps], [s, s], [g, g])
    assert e.value.status == mato.MATO_ERR_INVALID_ARG
    b = mato.Batch([pd], [s], [g])
    with pytest.raises(mato.MatoError) as e:
        b.set_rho_schedule([[pd], [ps]], [0, 10])
    assert e.value.status == mato.MATO_ERR_INVALID_ARG


def test_single_problem_api():
    """mato_solve_run / mato_step / state hooks give what a batch of one gives."""
    say("single-problem api")
    s, g = sc.swap_circle(4, seed=2)
    p = mato.Plan(4, 50, 11, 5.0, 0.4, 0.8, 1.0, "fp32")
    h, status = mato.mato_solve_run(p.handle, np.ascontiguousarray(s), np.ascontiguousarray(g), 20, 0.0, 5)
    assert status in (mato.MATO_OK, mato.MATO_WARN_NOT_CONVERGED)
    mato.mato_step(h, 7)
    mato.mato_solve_sync(h)
    b = mato.Batch([p], [s], [g])
    b.step(27)
    c = np.empty((4, 3, 11))
    mato.mato_solve_coeffs(h, c)
    np.testing.assert_array_equal(c, b.coeffs(0))
    r_max = np.empty(27)
    assert mato.mato_residuals(h, r_max, None, None, 27) == 27
    np.testing.assert_array_equal(r_max, b.residuals(0)[0])
    lam = np.empty((6, 50, 3), np.float32)
    mato.mato_get_state(h, c, lam)
    np.testing.assert_array_equal(lam, b.get_state(0)["lam"])
    # resume a second solve from the first one's state: same next iterate
    mato.lib().mato_batch_debug(h, 1)
    mato.mato_step(h, 1)
    proj = np.empty((6, 50, 3), np.float32)
    c1, lam1 = np.empty((4, 3, 11)), np.empty((6, 50, 3), np.float32)
    mato.mato_get_state(h, c1, lam1, proj)
    h2, _ = mato.mato_solve_run(p.handle, np.ascontiguousarray(s), np.ascontiguousarray(g), 0, 0.0, 1)
    mato.mato_set_state(h2, c1, lam1, proj)
    mato.mato_step(h, 3)
    mato.mato_step(h2, 3)
    c2, c3 = np.empty((4, 3, 11)), np.empty((4, 3, 11))
    mato.mato_solve_coeffs(h, c2)
    mato.mato_solve_coeffs(h2, c3)
    np.testing.assert_array_equal(c2, c3)
    mato.mato_solve_destroy(h)
    mato.mato_solve_destroy(h2)


def test_stream_copy_probe():
    say("stream copy probe")
    ms = mato.mato_stream_copy(1 << 24, 256, 3)
    assert ms > 0
    with pytest.raises(mato.MatoError) as e:
        mato.mato_stream_copy(15, 256, 1)
    assert e.value.status == mato.MATO_ERR_INVALID_ARG
    ms = mato.mato_stream_update(1 << 24, 256, 3)
    assert ms > 0
    with pytest.raises(mato.MatoError) as e:
        mato.mato_stream_update(1 << 24, 0, 1)
    assert e.value.status == mato.MATO_ERR_INVALID_ARG
    ms = mato.mato_stream_read(1 << 24, 256, 3)          # checks the sum of what it read
    assert ms > 0
    assert mato.mato_stream_read(1 << 24, 1, 1) > 0      # 2^22 floats on one workgroup: exact
    with pytest.raises(mato.MatoError) as e:
        mato.mato_stream_read(1 << 30, 1, 1)              # 2^28 floats on one workgroup: refused
    assert e.value.status == mato.MATO_ERR_INVALID_ARG


def test_batches_on_library_streams():
    """Two batches on their own library streams, stepped together, give exactly the
    iterates of the same problems in one batch on the default stream."""
    say("library streams")
    ns = [7, 12, 9]
    scen = [sc.random_density_box(n, seed=90 + k) for k, n in enumerate(ns)]
    plans = [mato.Plan(n, 40, 11, 4.0, 0.3, 0.6, 1.0, "fp32") for n in ns]
    ref = mato.Batch(plans, [x[0] for x in scen], [x[1] for x in scen])
    ref.step(25)
    s1, s2 = mato.Stream(), mato.Stream()
    b1 = mato.Batch(plans[:2], [x[0] for x in scen[:2]], [x[1] for x in scen[:2]], stream=s1)
    b2 = mato.Batch(plans[2:], [x[0] for x in scen[2:]], [x[1] for x in scen[2:]], stream=s2)
    b1.step(25)
    b2.step(25)
    b1.sync()
    b2.sync()
    for q in range(2):
        np.testing.assert_array_equal(b1.coeffs(q), ref.coeffs(q))
    np.testing.assert_array_equal(b2.coeffs(0), ref.coeffs(2))
    b1.close()
    b2.close()
    s1.close()
    s2.close()


def test_history_keeps_latest_beyond_capacity():
    """Past MATO_HISTORY_CAP iterations the history keeps its first entries and its last
    entry follows the latest iteration: equal to the first entry of a fresh problem
    resumed from the state one iteration earlier and stepped once."""
    say("history beyond capacity")
    cap = mato.MATO_HISTORY_CAP
    s, g = sc.swap_circle(4, seed=5)
    p = mato.Plan(4, 20, 11, 5.0, 0.4, 0.8, 1.0, "fp32")
    b = mato.Batch([p], [s], [g])
    b.step(cap - 1)
    head = [np.copy(x) for x in b.residuals(0)]
    assert len(head[0]) == cap - 1
    b.step(4)                            # iterations cap .. cap + 3 overwrite the last entry
    b.debug(True)
    b.step(1)                            # iteration cap + 4 leaves proj for the resume
    st = b.get_state(0, proj=True)
    b.step(1)                            # iteration cap + 5: the latest
    r = b.residuals(0)
    assert b.status(0)[0] == cap + 5 and len(r[0]) == cap
    for x, y in zip(r, head):
        np.testing.assert_array_equal(x[:cap - 1], y)
    fresh = mato.Batch([p], [s], [g])
    fresh.set_state(0, st["c"], st["lam"], st["proj"])
    fresh.step(1)
    one = fresh.residuals(0)
    for x, y in zip(r, one):
        assert x[cap - 1] == y[-1]
