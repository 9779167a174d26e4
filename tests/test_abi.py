"""C ABI surface (no GPU): libmato.so loads, exports every function include/mato.h
declares, the ctypes binding covers exactly those, and argument validation of
plan creation answers before any device work."""
import ctypes
import os
import re

import pytest

from paper_2011_04240_amd import mato

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(mato_[a-z0-9_]+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    L = mato.lib()
    declared = _declared()
    assert len(declared) > 20
    missing = [n for n in sorted(declared) if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    assert set(mato.SIGNATURES) == _declared()


def test_binding_constants_match_the_header():
    txt = open(os.path.join(ROOT, "include", "mato.h")).read()
    defines = dict(re.findall(r"#define\s+(MATO_[A-Z0-9_]+)\s+(-?\d+)\b", txt))
    assert len(defines) >= 12
    for name, value in defines.items():
        assert getattr(mato, name) == int(value), name


def test_version_string():
    assert "gfx950" in mato.mato_version()


@pytest.mark.parametrize("args,status", [
    (dict(n=1), mato.MATO_ERR_INVALID_ARG),
    (dict(n=mato.MATO_MAX_AGENTS + 1), mato.MATO_ERR_UNSUPPORTED),
    (dict(a=0.0), mato.MATO_ERR_INVALID_ARG),
    (dict(b=-1.0), mato.MATO_ERR_INVALID_ARG),
    (dict(rho=0.0), mato.MATO_ERR_INVALID_ARG),
    (dict(t_final=float("nan")), mato.MATO_ERR_INVALID_ARG),
    (dict(n_coef=5), mato.MATO_ERR_INVALID_ARG),
    (dict(T=8), mato.MATO_ERR_INVALID_ARG),
    (dict(precision=7), mato.MATO_ERR_INVALID_ARG),
])
def test_plan_argument_validation(args, status):
    kw = dict(n=4, T=50, n_coef=11, t_final=5.0, a=0.4, b=0.8, rho=1.0, precision=mato.MATO_FP32)
    kw.update(args)
    with pytest.raises(mato.MatoError) as e:
        mato.mato_plan_create(**kw)
    assert e.value.status == status


def test_null_handles_are_rejected():
    L = mato.lib()
    assert L.mato_batch_step(None, 1, 0.0, 0) == mato.MATO_ERR_INVALID_ARG
    assert L.mato_plan_info(None, None, None, None, None, None) == mato.MATO_ERR_INVALID_ARG
    assert L.mato_batch_create(0, None, None, None, None, ctypes.byref(ctypes.c_void_p())) == mato.MATO_ERR_INVALID_ARG


@pytest.mark.parametrize("precision,solve", [
    (mato.MATO_BF16_REFINED, mato.MATO_SOLVE_STRUCTURED),   # no BF16 product in the structured step
    (mato.MATO_FP32, 2),                                     # unknown solve kind
])
def test_solve_kind_validation(precision, solve):
    with pytest.raises(mato.MatoError) as e:
        mato.mato_plan_create_ex(mato.plan_desc(4, 50, 11, 5.0, 0.4, 0.8, precision, solve), [1.0])
    assert e.value.status == mato.MATO_ERR_INVALID_ARG


@pytest.mark.parametrize("n_obs", [-1, mato.MATO_MAX_OBSTACLES + 1])
def test_obstacle_count_validation(n_obs):
    with pytest.raises(mato.MatoError) as e:
        mato.mato_plan_create_ex(mato.plan_desc(4, 50, n_obs=n_obs), [1.0])
    assert e.value.status == mato.MATO_ERR_INVALID_ARG


def test_server_rejects_structured_bf16():
    cfg = mato.ServerConfig(100, mato._Basis(0, 11, 10.0), 0.3, 0.6, 1.0, mato.MATO_BF16_REFINED, 4, 0.0, 10,
                            100, 1e-3, 0)
    cfg.solve = mato.MATO_SOLVE_STRUCTURED
    with pytest.raises(mato.MatoError) as e:
        mato.mato_server_create(cfg)
    assert e.value.status == mato.MATO_ERR_INVALID_ARG
