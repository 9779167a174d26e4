"""Static obstacles (agent-obstacle rows of A_fc) on the GPU against the FP64 oracle.

Tolerances as in test_gpu_parity: 1e-5 relative per step for FP32, 1e-8 for FP64, whole
runs 1e-8 (FP64) and 1e-3 on the final cost and r_max (FP32); the plan inverse 1e-10."""
import numpy as np
import pytest

from oracle import am
from paper_2011_04240_amd import mato
from paper_2011_04240_amd import scenarios as sc

pytestmark = pytest.mark.gpu

# five agents swapping across a 2 m circle; obstacles on and near the crossing paths
CROSSING_OBS = np.array([[0.0, 0.0, 0.0, 0.75, 0.9], [1.0, 0.5, 0.0, 0.5, 0.6],
                         [-0.8, 0.9, 0.1, 0.45, 0.6], [0.3, -1.1, -0.1, 0.5, 0.65]])


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / (den if den > 0 else 1.0))


def say(*x):
    print(*x, flush=True)


def _scene():
    s, g = sc.swap_circle(5, radius=2.0, seed=11)
    return s, g, CROSSING_OBS


def _oplan(n_obs=4, n=5, T=40, tf=5.0):
    return am.make_plan(n, T, 11, tf, 0.3, 0.6, 1.0, n_obs=n_obs)


def _gplan(precision, solve, n_obs=4, n=5, T=40, tf=5.0):
    return mato.Plan(n, T, 11, tf, 0.3, 0.6, 1.0, precision, solve=solve, n_obs=n_obs)


@pytest.mark.parametrize("solve", ["dense", "structured"])
def test_inverse_with_obstacles(solve):
    say("inverse with obstacles", solve)
    assert rel(_gplan("fp64", solve).inverse(), _oplan().Kinv) < 1e-10


@pytest.mark.parametrize("solve", ["dense", "structured"])
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_single_step_with_obstacles(precision, solve):
    say("single step with obstacles", precision, solve)
    s, g, obs = _scene()
    op = _oplan()
    st = am.initial_state(op, s, g, obs)
    for _ in range(4):
        st = am.iterate(op, st)
    S = np.float64 if precision == "fp64" else np.float32
    lam = st.lam.astype(S)
    proj = st.proj(op).astype(S)
    b_fc = proj.astype(np.float64) - lam.astype(np.float64) / op.rho
    b_fc[op.n_pairs:] += np.tile(obs[:, :3], (op.n, 1))[:, None, :]
    ref = am.iterate_rhs(op, b_fc, lam.astype(np.float64), st.beq, obs=obs)
    b_next = ref["proj"] - ref["lam"] / op.rho
    b_next[op.n_pairs:] += np.tile(obs[:, :3], (op.n, 1))[:, None, :]
    g_next = am.linear_term(op, b_next)

    bt = mato.Batch([_gplan(precision, solve)], [s], [g], obstacles_list=[obs])
    bt.set_state(0, st.c, lam, proj)
    tol = 1e-8 if precision == "fp64" else 1e-5
    assert rel(bt.linear_term(0), ref["g"]) < tol
    bt.debug(True)
    bt.step(1, use_graph=False)
    out = bt.get_state(0, proj=True, d=True, X=True)
    r_max, r_rms, cost = bt.residuals(0)
    errs = dict(c=rel(out["c"], ref["c"]), X=rel(out["X"], ref["X"]), proj=rel(out["proj"], ref["proj"]),
                d=rel(out["d"], ref["d"]), lam=rel(out["lam"], ref["lam"]), g=rel(bt.linear_term(0), g_next),
                r_max=abs(r_max[-1] - ref["r_max"]) / ref["r_max"],
                r_rms=abs(r_rms[-1] - ref["r_rms"]) / ref["r_rms"],
                cost=abs(cost[-1] - ref["cost"]) / ref["cost"])
    say("  errors", {k: "%.2e" % v for k, v in errs.items()})
    for k, v in errs.items():
        assert v < tol, (k, v, errs)


@pytest.mark.parametrize("solve", ["dense", "structured"])
def test_full_run_fp64_with_obstacles(solve):
    say("full run fp64 with obstacles", solve)
    s, g, obs = _scene()
    ref = am.solve(_oplan(), s, g, 120, obs=obs)
    bt = mato.Batch([_gplan("fp64", solve)], [s], [g], obstacles_list=[obs])
    bt.run(120, 0.0, 40)
    r_max, _, cost = bt.residuals(0)
    assert rel(r_max, ref.history["r_max"]) < 1e-8
    assert rel(cost, ref.history["cost"]) < 1e-10
    assert rel(bt.coeffs(0), ref.c) < 1e-9
    assert rel(bt.get_state(0)["lam"], ref.lam) < 1e-8


def test_obstacle_box_fp32_structured():
    """n = 16 agents, 32 obstacles at the n = 64 density, T = 100, 200 iterations."""
    say("obstacle box n16 x 32")
    s, g, obs = sc.obstacle_box(16, 32, seed=3)
    ref = am.solve(_oplan(32, 16, 100, 10.0), s, g, 200, obs=obs)
    bt = mato.Batch([_gplan("fp32", "structured", 32, 16, 100, 10.0)], [s], [g], obstacles_list=[obs])
    bt.run(200, 0.0, 50)
    r_max, _, cost = bt.residuals(0)
    say("  cost %.6e vs %.6e, r_max %.4e vs %.4e" % (cost[-1], ref.history["cost"][-1], r_max[-1],
                                                     ref.history["r_max"][-1]))
    assert abs(cost[-1] - ref.history["cost"][-1]) / ref.history["cost"][-1] < 1e-3
    assert abs(r_max[-1] - ref.history["r_max"][-1]) <= 1e-3 * max(ref.history["r_max"][-1], 1e-3)


def test_mixed_obstacle_counts_bitwise_vs_alone():
    say("mixed obstacle counts")
    cases = [(6, 0, 1), (9, 3, 2), (5, 7, 3)]
    scen = [sc.obstacle_box(n, k, seed=sd) for n, k, sd in cases]
    plans = [_gplan("fp32", "structured", k, n, 50, 5.0) for n, k, _ in cases]
    b = mato.Batch(plans, [x[0] for x in scen], [x[1] for x in scen], obstacles_list=[x[2] for x in scen])
    b.step(30)
    for q, (n, k, _) in enumerate(cases):
        solo = mato.Batch([plans[q]], [scen[q][0]], [scen[q][1]], obstacles_list=[scen[q][2]])
        solo.step(30)
        np.testing.assert_array_equal(b.coeffs(q), solo.coeffs(0))
        np.testing.assert_array_equal(b.get_state(q)["lam"], solo.get_state(0)["lam"])


def test_obstacle_errors():
    say("obstacle errors")
    s, g, obs = _scene()
    p = _gplan("fp32", "structured")
    with pytest.raises(mato.MatoError) as e:
        mato.Batch([p], [s], [g])                                   # obstacles missing
    assert e.value.status == mato.MATO_ERR_INVALID_ARG
    bad = obs.copy()
    bad[1, 2] = np.inf
    with pytest.raises(mato.MatoError) as e:
        mato.Batch([p], [s], [g], obstacles_list=[bad])
    assert e.value.status == mato.MATO_ERR_NONFINITE
    bad = obs.copy()
    bad[0, 3] = 0.0
    with pytest.raises(mato.MatoError) as e:
        mato.Batch([p], [s], [g], obstacles_list=[bad])
    assert e.value.status == mato.MATO_ERR_INVALID_ARG


def test_server_with_obstacles_alone_vs_mix():
    """Requests with different obstacle counts (plans per agent and obstacle count) served
    together finish exactly as each problem alone."""
    say("server with obstacles")
    cases = [(6, 4, 1), (9, 0, 2), (5, 7, 3), (9, 4, 4)]
    scen = [sc.obstacle_box(n, k, seed=sd) for n, k, sd in cases]
    srv = mato.Server(T=50, t_final=5.0, a=0.3, b=0.6, precision="fp32", max_slots=2, chunk=5, max_iters=300,
                      tol=1e-3, solve="structured")
    ids = [srv.submit(s, g, o) for s, g, o in scen]
    out = {}
    for _ in range(100000):
        srv.step()
        for k, i in enumerate(ids):
            if k not in out and srv.poll(i)[0] == 2:
                st, it, conv, _ = srv.poll(i)
                out[k] = (srv.result(i, cases[k][0]), it, conv)
        if len(out) == len(ids):
            break
    assert len(out) == len(ids)
    for k, (n, n_obs, _) in enumerate(cases):
        p = _gplan("fp32", "structured", n_obs, n, 50, 5.0)
        b = mato.Batch([p], [scen[k][0]], [scen[k][1]], obstacles_list=[scen[k][2]])
        b.run(300, 1e-3, 5)
        it, conv = b.status(0)
        c, its, convs = out[k]
        assert its == it and convs == conv
        np.testing.assert_array_equal(c, b.coeffs(0))


def test_most_obstacles_fp64():
    """MATO_MAX_OBSTACLES static obstacles around 3 agents (3 075 collision rows): the
    inverse and 5 FP64 iterations against the oracle."""
    say("maximum obstacle count")
    n, k, T_ = 3, mato.MATO_MAX_OBSTACLES, 20
    rng = np.random.Generator(np.random.PCG64(77))
    s = np.array([[0.0, 0.0, 0.0], [2.0, 0.0, 0.0], [0.0, 2.0, 0.0]])
    g = -s
    obs = np.concatenate([rng.uniform(-20.0, 20.0, size=(k, 3)), rng.uniform(0.5, 1.0, size=(k, 2))], axis=1)
    plan = mato.Plan(n, T_, 11, 5.0, 0.3, 0.6, 1.0, "fp64", n_obs=k)
    ref_plan = am.make_plan(n, T_, 11, 5.0, 0.3, 0.6, 1.0, n_obs=k)
    assert rel(plan.inverse(), ref_plan.Kinv) < 1e-10
    ref = am.solve(ref_plan, s, g, 5, obs=obs)
    bt = mato.Batch([plan], [s], [g], obstacles_list=[obs])
    bt.run(5, 0.0, 5)
    assert rel(bt.residuals(0)[0], ref.history["r_max"]) < 1e-8
    assert rel(bt.coeffs(0), ref.c) < 1e-9
    assert rel(bt.get_state(0)["lam"], ref.lam) < 1e-8
