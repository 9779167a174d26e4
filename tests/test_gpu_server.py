"""Continuous-batching server through the C ABI.

* A problem's result is the same alone and in the mix: problems submitted while
  others are resident (and admitted as slots free up) finish with exactly the
  coefficients and iteration counts of the same problem solved alone.
* Admission respects the slot limit and the device-memory budget; queued problems
  wait and complete.
* Trace replay reports a latency, iteration count and convergence flag per request.
* Against the FP64 oracle: a served FP64 result equals the oracle's stopped run.
"""
import numpy as np
import pytest

from oracle import am
from paper_2011_04240_amd import mato
from paper_2011_04240_amd import scenarios as sc

pytestmark = pytest.mark.gpu

T, TF, A, B = 60, 6.0, 0.3, 0.6


def say(*a):
    print(*a, flush=True)


def _alone(n, s, g, precision, tol, cap):
    p = mato.Plan(n, T, 11, TF, A, B, 1.0, precision)
    b = mato.Batch([p], [s], [g])
    b.run(cap, tol, 10)
    it, conv = b.status(0)
    return b.coeffs(0), it, conv


def _drain(srv, ids, ns):
    out = {}
    for _ in range(100000):
        running, queued = srv.step()
        for k, i in enumerate(ids):
            if k in out:
                continue
            st, it, conv, rmax = srv.poll(i)
            if st == 2:
                out[k] = (srv.result(i, ns[k]), it, conv)
        if len(out) == len(ids):
            return out
    raise AssertionError("server did not drain")


@pytest.mark.parametrize("precision,graphs", [("fp32", False), ("fp64", False), ("fp32", True)])
def test_alone_vs_mix(precision, graphs):
    say("server alone vs mix", precision, "graphs" if graphs else "eager")
    ns = [4, 17, 9, 30, 17, 6, 23, 12]
    scen = [sc.random_density_box(n, seed=200 + k) for k, n in enumerate(ns)]
    tol, cap = 1e-3, 600
    srv = mato.Server(T=T, t_final=TF, a=A, b=B, precision=precision, max_slots=4, chunk=7, max_iters=cap, tol=tol,
                      use_graphs=graphs)
    ids = [srv.submit(*scen[k]) for k in range(3)]
    srv.step()
    srv.step()
    ids += [srv.submit(*scen[k]) for k in range(3, len(ns))]     # arrive while others are resident
    out = _drain(srv, ids, ns)
    for k, n in enumerate(ns):
        c, it, conv = _alone(n, scen[k][0], scen[k][1], precision, tol, cap)
        cs, its, convs = out[k]
        assert its == it and convs == conv, (k, its, it, convs, conv)
        np.testing.assert_array_equal(cs, c)


def test_queue_and_budget():
    say("server budget")
    ns = [10, 20, 10, 20, 14, 10]
    scen = [sc.random_density_box(n, seed=300 + k) for k, n in enumerate(ns)]
    budget = 2.3e6      # fits any one plan with two slots, not all three plans at once
    srv = mato.Server(T=T, t_final=TF, a=A, b=B, precision="fp32", max_slots=2, chunk=5, max_iters=300,
                      tol=1e-3, hbm_budget_bytes=budget)
    ids = [srv.submit(*x) for x in scen]
    running, queued = srv.step()
    assert running <= 2 and queued >= len(ns) - 2
    out = _drain(srv, ids, ns)
    assert len(out) == len(ns)
    dev_bytes, n_plans, running, queued = srv.stats()
    assert running == 0 and queued == 0
    assert dev_bytes <= budget


def test_trace_replay():
    say("server trace")
    rng = np.random.Generator(np.random.PCG64(7))
    ns = [int(x) for x in rng.integers(4, 25, size=24)]
    scen = [sc.random_density_box(n, seed=400 + k) for k, n in enumerate(ns)]
    arr = sc.poisson_arrivals(200.0, len(ns), seed=3)
    srv = mato.Server(T=T, t_final=TF, a=A, b=B, precision="fp32", max_slots=8, chunk=10, max_iters=400, tol=1e-3)
    srv.warm(4, 24)
    lat, its, conv, wall = srv.run_trace(arr, [x[0] for x in scen], [x[1] for x in scen])
    assert np.all(lat > 0) and np.all(its >= 1) and np.all(its <= 400)
    assert wall >= arr[-1]
    assert np.all(conv[its < 400] == 1)


def test_served_result_matches_oracle():
    say("server vs oracle")
    n = 8
    s, g = sc.random_density_box(n, seed=9)
    srv = mato.Server(T=T, t_final=TF, a=A, b=B, precision="fp64", max_slots=2, chunk=4, max_iters=500, tol=1e-3)
    i = srv.submit(s, g)
    out = _drain(srv, [i], [n])
    c, it, conv = out[0]
    ref = am.solve(am.make_plan(n, T, 11, TF, A, B, 1.0), s, g, 500, tol=1e-3)
    assert it == len(ref.history["r_max"]) and conv
    np.testing.assert_allclose(c, ref.c, rtol=0, atol=1e-8 * np.max(np.abs(ref.c)))


def test_server_errors():
    say("server errors")
    srv = mato.Server(T=T, t_final=TF, a=A, b=B, precision="fp32", max_slots=1)
    with pytest.raises(mato.MatoError) as e:
        srv.submit(np.zeros((1, 3)), np.zeros((1, 3)))
    assert e.value.status == mato.MATO_ERR_INVALID_ARG
    with pytest.raises(mato.MatoError) as e:
        mato.mato_server_poll(srv.handle, 12345)
    assert e.value.status == mato.MATO_ERR_NOT_FOUND
    s, g = sc.random_density_box(5, seed=1)
    g[0, 0] = np.inf
    with pytest.raises(mato.MatoError) as e:
        srv.submit(s, g)
    assert e.value.status == mato.MATO_ERR_NONFINITE


def test_request_that_never_fits_is_rejected():
    say("server rejects a request the budget can never hold")
    s40, g40 = sc.random_density_box(40, seed=501)
    s10, g10 = sc.random_density_box(10, seed=502)
    budget = 2.3e6      # holds the n = 10 plan and a slot, never the n = 40 plan (about 4.5 MB)
    srv = mato.Server(T=T, t_final=TF, a=A, b=B, precision="fp32", max_slots=2, chunk=5, max_iters=300,
                      tol=1e-3, hbm_budget_bytes=budget)
    big = srv.submit(s40, g40)
    small = srv.submit(s10, g10)
    srv.step()
    st, it, conv, _ = srv.poll(big)
    assert st == 3 and it == 0 and conv == 0
    with pytest.raises(mato.MatoError) as e:
        srv.result(big, 40)
    assert e.value.status == mato.MATO_ERR_OUT_OF_MEMORY
    with pytest.raises(mato.MatoError) as e:
        srv.poll(big)           # forgotten once collected
    assert e.value.status == mato.MATO_ERR_NOT_FOUND
    out = _drain(srv, [small], [10])
    c, it, conv = _alone(10, s10, g10, "fp32", 1e-3, 300)
    assert out[0][1] == it and out[0][2] == conv
    np.testing.assert_array_equal(out[0][0], c)


def test_trace_with_a_rejected_request_ends():
    say("server trace with a rejected request")
    ns = [8, 40, 8]
    scen = [sc.random_density_box(n, seed=600 + k) for k, n in enumerate(ns)]
    srv = mato.Server(T=T, t_final=TF, a=A, b=B, precision="fp32", max_slots=2, chunk=5, max_iters=300,
                      tol=1e-3, hbm_budget_bytes=2.3e6)
    lat, its, conv, wall = srv.run_trace([0.0, 0.001, 0.002], [x[0] for x in scen], [x[1] for x in scen])
    assert its[1] == 0 and conv[1] == 0
    assert its[0] > 0 and its[2] > 0 and conv[0] == 1 and conv[2] == 1


def test_empty_trace():
    say("server empty trace")
    srv = mato.Server(T=T, t_final=TF, a=A, b=B, precision="fp32", max_slots=2)
    lat, its, conv, wall = srv.run_trace([], [], [])
    assert len(lat) == 0 and len(its) == 0 and len(conv) == 0 and wall >= 0.0
    assert srv.stats()[2:] == (0, 0)
