"""Error of every recorded result against the FP64 oracle over a whole run, per precision:
n = 64 agents in the random box, T = 100, 300 iterations, rho = 1 (the precision
configuration).  Printed as a table; bounds: FP32 and BF16-refined final cost, max ||f_c||,
coefficients and multipliers within 1e-3 relative (the stated whole-run tolerance); FP64 within
1e-8 (multipliers 1e-7)."""
import numpy as np
import pytest

from oracle import am
from paper_2011_04240_amd import mato
from paper_2011_04240_amd import scenarios as sc

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def reference():
    s, g = sc.random_box(64, seed=0)
    say("oracle n64 x 300 iterations")
    st = am.solve(am.make_plan(64, 100, 11, 10.0, 0.3, 0.6, 1.0), s, g, 300)
    return s, g, st


@pytest.mark.parametrize("precision,solve", [("bf16", "dense"), ("fp32", "dense"), ("fp64", "dense"),
                                             ("fp32", "structured"), ("fp64", "structured")])
def test_whole_run_errors_n64(reference, precision, solve):
    s, g, ref = reference
    b = mato.Batch([mato.Plan(64, 100, 11, 10.0, 0.3, 0.6, 1.0, precision, solve=solve)], [s], [g])
    b.run(300, 0.0, 100)
    r_max, r_rms, cost = b.residuals(0)
    st = b.get_state(0)
    hr, hrr, hc = (np.asarray(ref.history[k]) for k in ("r_max", "r_rms", "cost"))
    err = {
        "cost_final": abs(cost[-1] - hc[-1]) / hc[-1],
        "r_max_final": abs(r_max[-1] - hr[-1]) / hr[-1],
        "r_rms_final": abs(r_rms[-1] - hrr[-1]) / hrr[-1],
        "cost_history": float(np.max(np.abs(cost - hc) / hc)),
        "c_final": float(np.max(np.abs(st["c"] - ref.c)) / np.max(np.abs(ref.c))),
        "lambda_final": float(np.max(np.abs(st["lam"] - ref.lam)) / np.max(np.abs(ref.lam))),
    }
    say("  %-5s %-10s " % (precision, solve) + "  ".join("%s %.2e" % kv for kv in err.items()))
    tol = 1e-8 if precision == "fp64" else 1e-3
    assert err["cost_final"] < tol and err["r_max_final"] < tol, err
    # the final coefficients and multipliers at the whole-run tolerance; in FP64 the multipliers
    # carry the sum of 300 rho f_c steps, each within ~1e-10 of the oracle's: bound 1e-7
    assert err["c_final"] < tol, err
    assert err["lambda_final"] < (1e-7 if precision == "fp64" else 1e-3), err
