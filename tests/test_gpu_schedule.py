"""Increasing-rho schedule (inverses cached for several rho, larger ones later, Sec. IV-A)
on the GPU against the oracle's solve_schedule, in batches and in the server."""
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


def say(*x):
    print(*x, flush=True)


def test_schedule_fp64_matches_oracle():
    say("schedule fp64 n4")
    s, g = sc.swap_circle(4, seed=0)
    rhos, starts = [1.0, 2.0, 4.0], [0, 10, 25]
    oplans = [am.make_plan(4, 50, 11, 5.0, 0.4, 0.8, r) for r in rhos]
    ref = am.solve_schedule(oplans, starts, s, g, 40)
    gplans = [mato.Plan(4, 50, 11, 5.0, 0.4, 0.8, r, "fp64") for r in rhos]
    b = mato.Batch([gplans[0]], [s], [g])
    b.set_rho_schedule([[p] for p in gplans], starts)
    b.step(7, use_graph=False)
    b.step(33, use_graph=True)
    r_max, _, cost = b.residuals(0)
    assert len(r_max) == 40
    assert rel(r_max, ref.history["r_max"]) < 1e-8
    assert rel(cost, ref.history["cost"]) < 1e-10
    assert rel(b.coeffs(0), ref.c) < 1e-9


def test_schedule_fp32_uneven_batch():
    say("schedule fp32 uneven batch")
    ns = [6, 13]
    rhos, starts = [1.0, 2.0, 4.0, 8.0], [0, 30, 60, 90]
    scen = [sc.random_density_box(n, seed=50 + k) for k, n in enumerate(ns)]
    gp = {n: [mato.Plan(n, 60, 11, 6.0, 0.3, 0.6, r, "fp32") for r in rhos] for n in ns}
    b = mato.Batch([gp[n][0] for n in ns], [x[0] for x in scen], [x[1] for x in scen])
    b.set_rho_schedule([[gp[n][j] for n in ns] for j in range(len(rhos))], starts)
    b.run(120, 0.0, 40)
    for k, n in enumerate(ns):
        oplans = [am.make_plan(n, 60, 11, 6.0, 0.3, 0.6, r) for r in rhos]
        ref = am.solve_schedule(oplans, starts, scen[k][0], scen[k][1], 120)
        r_max, _, cost = b.residuals(k)
        assert abs(cost[-1] - ref.history["cost"][-1]) / ref.history["cost"][-1] < 1e-3
        assert abs(r_max[-1] - ref.history["r_max"][-1]) <= 1e-3 * max(ref.history["r_max"][-1], 1e-3)


def test_server_schedule_alone_vs_mix():
    say("server schedule")
    T, TF = 60, 6.0
    rhos, starts = [1.0, 2.0, 4.0, 8.0, 16.0], [0, 20, 40, 60, 80]
    ns = [5, 14, 9, 22]
    scen = [sc.random_density_box(n, seed=600 + k) for k, n in enumerate(ns)]
    srv = mato.Server(T=T, t_final=TF, a=0.3, b=0.6, precision="fp32", max_slots=2, chunk=10, max_iters=400,
                      tol=1e-3, rho_schedule=(rhos, starts))
    ids = [srv.submit(*x) for x in scen]
    out = {}
    for _ in range(10000):
        srv.step()
        for k, i in enumerate(ids):
            if k not in out and srv.poll(i)[0] == 2:
                st, it, conv, _ = srv.poll(i)
                out[k] = (srv.result(i, ns[k]), it, conv)
        if len(out) == len(ids):
            break
    assert len(out) == len(ids)
    for k, n in enumerate(ns):
        plans = [mato.Plan(n, T, 11, TF, 0.3, 0.6, r, "fp32") for r in rhos]
        b = mato.Batch([plans[0]], [scen[k][0]], [scen[k][1]])
        b.set_rho_schedule([[p] for p in plans], starts)
        b.run(400, 1e-3, 10)
        it, conv = b.status(0)
        c, its, convs = out[k]
        assert its == it and convs == conv
        np.testing.assert_array_equal(c, b.coeffs(0))


def test_plan_create_many_matches_single():
    say("plan_create_many")
    rhos = [0.5, 1.0, 3.0, 9.0]
    for prec in ("fp64", "fp32", "bf16"):
        many = mato.Plan.schedule(7, 40, rhos, 11, 4.0, 0.3, 0.6, prec)
        for r, p in zip(rhos, many):
            one = mato.Plan(7, 40, 11, 4.0, 0.3, 0.6, r, prec)
            np.testing.assert_array_equal(p.inverse(), one.inverse())
            assert p.info()[4] == one.info()[4]


def test_schedule_structured_fp64_matches_oracle():
    say("schedule structured fp64 n6")
    s, g = sc.random_density_box(6, seed=7)
    rhos, starts = [1.0, 4.0, 16.0, 64.0], [0, 15, 30, 45]
    oplans = [am.make_plan(6, 40, 11, 4.0, 0.3, 0.6, r) for r in rhos]
    ref = am.solve_schedule(oplans, starts, s, g, 60)
    gplans = mato.Plan.schedule(6, 40, rhos, 11, 4.0, 0.3, 0.6, "fp64", solve="structured")
    b = mato.Batch([gplans[0]], [s], [g])
    b.set_rho_schedule([[p] for p in gplans], starts)
    b.step(60, use_graph=True)
    r_max, _, cost = b.residuals(0)
    assert rel(r_max, ref.history["r_max"]) < 1e-8
    assert rel(cost, ref.history["cost"]) < 1e-10
    assert rel(b.coeffs(0), ref.c) < 1e-9


def test_server_structured_alone_vs_mix_and_oracle():
    say("server structured")
    T, TF = 60, 6.0
    rhos, starts = [1.0, 2.0, 4.0, 8.0], [0, 20, 40, 60]
    ns = [5, 14, 9, 22, 3]
    scen = [sc.random_density_box(n, seed=700 + k) for k, n in enumerate(ns)]
    srv = mato.Server(T=T, t_final=TF, a=0.3, b=0.6, precision="fp32", max_slots=2, chunk=10, max_iters=300,
                      tol=1e-3, rho_schedule=(rhos, starts), solve="structured")
    ids = [srv.submit(*x) for x in scen]
    out = {}
    for _ in range(10000):
        srv.step()
        for k, i in enumerate(ids):
            if k not in out and srv.poll(i)[0] == 2:
                st, it, conv, _ = srv.poll(i)
                out[k] = (srv.result(i, ns[k]), it, conv)
        if len(out) == len(ids):
            break
    assert len(out) == len(ids)
    for k, n in enumerate(ns):
        plans = mato.Plan.schedule(n, T, rhos, 11, TF, 0.3, 0.6, "fp32", solve="structured")
        b = mato.Batch([plans[0]], [scen[k][0]], [scen[k][1]])
        b.set_rho_schedule([[p] for p in plans], starts)
        b.run(300, 1e-3, 10)
        it, conv = b.status(0)
        c, its, convs = out[k]
        assert its == it and convs == conv
        np.testing.assert_array_equal(c, b.coeffs(0))
    # the smallest request against the oracle, same iteration count
    k = ns.index(3)
    oplans = [am.make_plan(3, T, 11, TF, 0.3, 0.6, r) for r in rhos]
    ref = am.solve_schedule(oplans, starts, scen[k][0], scen[k][1], out[k][1])
    assert rel(out[k][0], ref.c) < 1e-3
