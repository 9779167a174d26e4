"""GPU parity of the HIP path against the FP64 oracle (through the C ABI).

Tolerances (relative to the infinity norm of the reference array):
  * single iteration from an injected FP32-representable oracle state: 1e-5 for
    MATO_FP32 and MATO_BF16_REFINED; 1e-8 for MATO_FP64 (the product c = K^{-1} q
    cancels: sum |K^{-1}||q| / |c| reaches ~1e4 at n = 64, times u K ~ 1e-13 for
    K = 17n terms gives ~1e-9 on c; residual norms are differences of such values);
  * whole runs: final smoothness cost and max ||f_c|| within 1e-3 (FP32) and
    1e-8 (FP64) relative;
  * the offline inverse: 1e-10 relative to the oracle's FP64 inverse.
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
    den = np.max(np.abs(b)) if b.size else 1.0
    return float(np.max(np.abs(a - b)) / (den if den > 0 else 1.0)) if b.size else 0.0


def say(*a):
    print(*a, flush=True)


CASES = {
    "swap_circle_n4_T50": dict(n=4, T=50, tf=5.0, a=0.4, b=0.8, gen=lambda: sc.swap_circle(4, seed=0)),
    "swap_sphere_n16_T100": dict(n=16, T=100, tf=10.0, a=0.3, b=0.6, gen=lambda: sc.swap_sphere(16, seed=0)),
    "box_n37_T53_ragged": dict(n=37, T=53, tf=6.0, a=0.3, b=0.6, gen=lambda: sc.random_density_box(37, seed=3)),
    "box_n64_T100": dict(n=64, T=100, tf=10.0, a=0.3, b=0.6, gen=lambda: sc.random_box(64, seed=0)),
}


def _oracle_plan(c):
    return am.make_plan(c["n"], c["T"], 11, c["tf"], c["a"], c["b"], 1.0)


def _gpu_plan(c, precision, solve="dense"):
    return mato.Plan(c["n"], c["T"], 11, c["tf"], c["a"], c["b"], 1.0, precision, solve=solve)


@pytest.mark.parametrize("name", ["swap_circle_n4_T50", "swap_sphere_n16_T100", "box_n37_T53_ragged"])
def test_plan_inverse_matches_oracle(name):
    c = CASES[name]
    say("plan inverse", name)
    gp = _gpu_plan(c, "fp64")
    op = _oracle_plan(c)
    assert rel(gp.inverse(), op.Kinv) < 1e-10
    n, T, nc, pr, cond = gp.info()
    assert (n, T, nc) == (c["n"], c["T"], 11)
    assert 0.2 < cond / np.linalg.cond(op.K, 1) < 5.0


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16"])
def test_initial_state_matches_oracle(precision):
    c = CASES["swap_sphere_n16_T100"]
    say("initial state", precision)
    s, g = c["gen"]()
    op = _oracle_plan(c)
    st = am.initial_state(op, s, g)
    b = mato.Batch([_gpu_plan(c, precision)], [s], [g])
    gs = b.get_state(0)
    assert rel(gs["c"], st.c) < 1e-12
    np.testing.assert_array_equal(gs["lam"], 0)
    g_ref = am.linear_term(op, am.collision_rhs(op, st.d, st.alpha, st.beta, st.lam))
    tol = 1e-12 if precision == "fp64" else 1e-5
    assert rel(b.linear_term(0), g_ref) < tol


def _single_step(name, precision, k_oracle=5, shifted=False, solve="dense"):
    c = CASES[name]
    s, g = c["gen"]()
    op = _oracle_plan(c)
    st = am.initial_state(op, s, g)
    for _ in range(k_oracle):
        st = am.iterate(op, st, shifted)
    S = np.float64 if precision == "fp64" else np.float32
    lam = st.lam.astype(S)
    proj = st.proj(op).astype(S)
    b_fc = proj.astype(np.float64) - lam.astype(np.float64) / op.rho
    ref = am.iterate_rhs(op, b_fc, lam.astype(np.float64), st.beq, shifted)
    g_next = am.linear_term(op, ref["proj"] - ref["lam"] / op.rho)

    gp = _gpu_plan(c, precision, solve)
    bt = mato.Batch([gp], [s], [g])
    bt.set_state(0, st.c, lam, proj)
    if shifted:
        bt.set_projection(True)
    assert rel(bt.linear_term(0), ref["g"]) < (1e-10 if precision == "fp64" else 1e-5)
    bt.debug(True)
    bt.step(1, use_graph=False)
    out = bt.get_state(0, proj=True, d=True, X=True)
    r_max, r_rms, cost = bt.residuals(0)
    errs = dict(c=rel(out["c"], ref["c"]), X=rel(out["X"], ref["X"]), proj=rel(out["proj"], ref["proj"]),
                d=rel(out["d"], ref["d"]), lam=rel(out["lam"], ref["lam"]),
                g=rel(bt.linear_term(0), g_next),
                r_max=abs(r_max[-1] - ref["r_max"]) / ref["r_max"],
                r_rms=abs(r_rms[-1] - ref["r_rms"]) / ref["r_rms"],
                cost=abs(cost[-1] - ref["cost"]) / ref["cost"])
    return errs


@pytest.mark.parametrize("name", ["swap_circle_n4_T50", "swap_sphere_n16_T100", "box_n37_T53_ragged", "box_n64_T100"])
@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp64"])
def test_single_step_parity(name, precision):
    say("single step", name, precision)
    errs = _single_step(name, precision)
    say("  errors", {k: "%.2e" % v for k, v in errs.items()})
    tol = 1e-8 if precision == "fp64" else 1e-5
    for k, v in errs.items():
        assert v < tol, (k, v, errs)


@pytest.mark.parametrize("name", ["swap_sphere_n16_T100", "box_n37_T53_ragged"])
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_single_step_parity_shifted_projection(name, precision):
    say("single step shifted", name, precision)
    errs = _single_step(name, precision, shifted=True)
    say("  errors", {k: "%.2e" % v for k, v in errs.items()})
    tol = 1e-8 if precision == "fp64" else 1e-5
    for k, v in errs.items():
        assert v < tol, (k, v, errs)


def test_full_run_shifted_projection_fp64():
    c = CASES["swap_circle_n4_T50"]
    say("full run shifted fp64")
    s, g = c["gen"]()
    op = _oracle_plan(c)
    st = am.solve(op, s, g, 100, shifted=True)
    bt = mato.Batch([_gpu_plan(c, "fp64")], [s], [g])
    bt.set_projection(True)
    bt.run(100, 0.0, 25)
    r_max, _, cost = bt.residuals(0)
    assert rel(r_max, st.history["r_max"]) < 1e-8
    assert rel(bt.coeffs(0), st.c) < 1e-9


def test_full_run_fp64_swap_circle():
    """Config: n = 4 on a 3 m circle, T = 50, 5 s, a = 0.4, b = 0.8, rho = 1, 200 iterations, FP64."""
    c = CASES["swap_circle_n4_T50"]
    say("full run fp64 n4")
    s, g = c["gen"]()
    op = _oracle_plan(c)
    st = am.solve(op, s, g, 200)
    bt = mato.Batch([_gpu_plan(c, "fp64")], [s], [g])
    bt.run(200, 0.0, 50)
    r_max, r_rms, cost = bt.residuals(0)
    assert len(r_max) == 200
    assert rel(r_max, st.history["r_max"]) < 1e-8
    assert rel(cost, st.history["cost"]) < 1e-10
    assert rel(bt.coeffs(0), st.c) < 1e-9


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_full_run_fp32_swap_sphere(precision):
    """Config: n = 16 on a 4 m sphere, T = 100, 10 s, a = 0.3, b = 0.6, rho = 1, 300 iterations."""
    c = CASES["swap_sphere_n16_T100"]
    say("full run", precision, "n16")
    s, g = c["gen"]()
    op = _oracle_plan(c)
    st = am.solve(op, s, g, 300)
    bt = mato.Batch([_gpu_plan(c, precision)], [s], [g])
    bt.run(300, 0.0, 100)
    r_max, r_rms, cost = bt.residuals(0)
    say("  final cost %.6e vs %.6e, r_max %.6e vs %.6e" % (cost[-1], st.history["cost"][-1],
                                                          r_max[-1], st.history["r_max"][-1]))
    assert abs(cost[-1] - st.history["cost"][-1]) / st.history["cost"][-1] < 1e-3
    assert abs(r_max[-1] - st.history["r_max"][-1]) / st.history["r_max"][-1] < 1e-3


def test_graph_and_eager_agree_bitwise():
    c = CASES["box_n37_T53_ragged"]
    say("graph vs eager")
    s, g = c["gen"]()
    b1 = mato.Batch([_gpu_plan(c, "fp32")], [s], [g])
    b2 = mato.Batch([_gpu_plan(c, "fp32")], [s], [g])
    b1.step(37, use_graph=True)
    b2.step(37, use_graph=False)
    b1.sync()
    b2.sync()
    s1, s2 = b1.get_state(0), b2.get_state(0)
    np.testing.assert_array_equal(s1["c"], s2["c"])
    np.testing.assert_array_equal(s1["lam"], s2["lam"])
    b1.step(5, use_graph=True)          # replay again after eager work
    b2.step(5, use_graph=False)
    np.testing.assert_array_equal(b1.get_state(0)["lam"], b2.get_state(0)["lam"])


def test_tiles_do_not_change_iterates():
    c = CASES["swap_sphere_n16_T100"]
    say("tile independence")
    s, g = c["gen"]()
    outs = []
    for ipw, thr in [(256, 256), (2048, 512), (16384, 1024)]:
        b = mato.Batch([_gpu_plan(c, "fp32")], [s], [g])
        b.set_tiles(ipw, thr)
        b.step(20, use_graph=False)
        outs.append(b.get_state(0))
    for o in outs[1:]:
        np.testing.assert_array_equal(o["c"], outs[0]["c"])
        np.testing.assert_array_equal(o["lam"], outs[0]["lam"])


# ------------------------------------------------------------ structured solve ---
@pytest.mark.parametrize("name", ["swap_circle_n4_T50", "swap_sphere_n16_T100", "box_n37_T53_ragged"])
def test_structured_inverse_matches_oracle(name):
    """The two-block form of K^{-1} expanded to (17n)^2 equals the oracle's dense inverse."""
    c = CASES[name]
    say("structured inverse", name)
    gp = _gpu_plan(c, "fp64", "structured")
    desc, rho = mato.mato_plan_describe(gp.handle)
    assert desc.solve == mato.MATO_SOLVE_STRUCTURED and (desc.n, desc.n_obs, rho) == (c["n"], 0, 1.0)
    assert rel(gp.inverse(), _oracle_plan(c).Kinv) < 1e-10


@pytest.mark.parametrize("name", ["swap_circle_n4_T50", "swap_sphere_n16_T100", "box_n37_T53_ragged", "box_n64_T100"])
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_single_step_parity_structured(name, precision):
    say("single step structured", name, precision)
    errs = _single_step(name, precision, solve="structured")
    say("  errors", {k: "%.2e" % v for k, v in errs.items()})
    tol = 1e-8 if precision == "fp64" else 1e-5
    for k, v in errs.items():
        assert v < tol, (k, v, errs)


def test_full_run_structured_fp64_swap_circle():
    c = CASES["swap_circle_n4_T50"]
    say("full run structured fp64 n4")
    s, g = c["gen"]()
    st = am.solve(_oracle_plan(c), s, g, 200)
    bt = mato.Batch([_gpu_plan(c, "fp64", "structured")], [s], [g])
    bt.run(200, 0.0, 50)
    r_max, r_rms, cost = bt.residuals(0)
    assert len(r_max) == 200
    assert rel(r_max, st.history["r_max"]) < 1e-8
    assert rel(cost, st.history["cost"]) < 1e-10
    assert rel(bt.coeffs(0), st.c) < 1e-9


def test_structured_and_dense_runs_agree_fp64():
    """n = 37, T = 53 (ragged), 120 iterations: the two solves differ only by rounding."""
    c = CASES["box_n37_T53_ragged"]
    say("structured vs dense fp64 n37")
    s, g = c["gen"]()
    out = []
    for solve in ("dense", "structured"):
        bt = mato.Batch([_gpu_plan(c, "fp64", solve)], [s], [g])
        bt.run(120, 0.0, 40)
        out.append((bt.coeffs(0), bt.residuals(0)))
    assert rel(out[1][0], out[0][0]) < 1e-8
    assert rel(out[1][1][0], out[0][1][0]) < 1e-6


def test_structured_graph_and_eager_agree_bitwise():
    c = CASES["box_n37_T53_ragged"]
    say("structured graph vs eager")
    s, g = c["gen"]()
    b1 = mato.Batch([_gpu_plan(c, "fp32", "structured")], [s], [g])
    b2 = mato.Batch([_gpu_plan(c, "fp32", "structured")], [s], [g])
    b1.step(37, use_graph=True)
    b2.step(37, use_graph=False)
    s1, s2 = b1.get_state(0), b2.get_state(0)
    np.testing.assert_array_equal(s1["c"], s2["c"])
    np.testing.assert_array_equal(s1["lam"], s2["lam"])
