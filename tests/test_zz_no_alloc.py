"""mato_solve_noalloc (the whole solve with every device buffer carved from the library's
fixed scratch array) against mato_solve_run + sync + coeffs + residuals + status on the
same plan and inputs: bitwise equal, on consecutive calls whose second problem is
smaller, after a call that the array cannot hold (UNSUPPORTED), and in FP64."""
import numpy as np
import pytest

from paper_2011_04240_amd import mato
from paper_2011_04240_amd import scenarios as sc

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def _reference(plan, s, g, iters, tol, every):
    h, status = mato.mato_solve_run(plan.handle, s, g, iters, tol, every)
    try:
        mato.mato_solve_sync(h)
        c = np.empty((plan.n, 3, plan.n_coef))
        mato.mato_solve_coeffs(h, c)
        cap = max(iters, 1)
        r = [np.zeros(cap) for _ in range(3)]
        nw = mato.mato_residuals(h, r[0], r[1], r[2], cap)
        it, conv = mato.mato_batch_status(h, 0)
    finally:
        mato.mato_solve_destroy(h)
    return status, c, [x[:nw] for x in r], it, conv


def _noalloc(plan, s, g, iters, tol, every):
    c = np.full((plan.n, 3, plan.n_coef), np.nan)
    cap = max(iters, 1)
    r = [np.full(cap, np.nan) for _ in range(3)]
    status, nw, it, conv = mato.mato_solve_noalloc(plan.handle, s, g, iters, tol, every, c, r[0], r[1], r[2], cap)
    return status, c, [x[:nw] for x in r], it, conv


def _same(plan, s, g, iters, tol, every):
    ref = _reference(plan, s, g, iters, tol, every)
    out = _noalloc(plan, s, g, iters, tol, every)
    assert out[0] == ref[0] and out[3] == ref[3] and out[4] == ref[4], (out[0], ref[0], out[3:], ref[3:])
    np.testing.assert_array_equal(out[1], ref[1])
    for a, b in zip(out[2], ref[2]):
        assert len(a) == len(b) == min(ref[3], iters)
        np.testing.assert_array_equal(a, b)
    return out


def test_noalloc_matches_solve_run():
    say("noalloc: n = 24 then n = 9, FP32 dense")
    p24 = mato.Plan(24, 100, 11, 10.0, 0.3, 0.6, 1.0, "fp32")
    s, g = sc.random_density_box(24, seed=600)
    out = _same(p24, s, g, 300, 1e-3, 10)
    say("  n = 24: %d iterations, converged %d, final r_max %.3e" % (out[3], out[4], out[2][0][-1]))
    p9 = mato.Plan(9, 100, 11, 10.0, 0.3, 0.6, 1.0, "fp32")
    s9, g9 = sc.random_density_box(9, seed=602)
    out = _same(p9, s9, g9, 120, 0.0, 40)
    say("  n = 9: %d iterations" % out[3])


def test_noalloc_rejects_what_does_not_fit_and_recovers():
    say("noalloc: a problem beyond the scratch array, then a small one")
    big = mato.Plan(160, 300, 11, 10.0, 0.3, 0.6, 1.0, "fp32")     # multipliers alone: 45.8 MB
    s, g = sc.random_density_box(160, seed=1)
    with pytest.raises(mato.MatoError) as e:
        _noalloc(big, s, g, 5, 0.0, 5)
    assert e.value.status == mato.MATO_ERR_UNSUPPORTED
    big.close()
    p = mato.Plan(12, 60, 11, 6.0, 0.3, 0.6, 1.0, "fp64")
    s, g = sc.random_density_box(12, seed=600)
    out = _same(p, s, g, 50, 0.0, 25)
    say("  fp64 n = 12 after the rejection: %d iterations" % out[3])


def test_noalloc_bf16_structured():
    say("noalloc: BF16 dense and FP32 structured")
    for prec, solve in (("bf16", "dense"), ("fp32", "structured")):
        p = mato.Plan(16, 100, 11, 10.0, 0.3, 0.6, 1.0, prec, solve=solve)
        s, g = sc.random_density_box(16, seed=600)
        out = _same(p, s, g, 200, 1e-3, 10)
        say("  %s %s: %d iterations" % (prec, solve, out[3]))
