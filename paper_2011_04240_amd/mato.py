"""ctypes binding of libmato (C ABI in include/mato.h).

Argument marshalling only: every step of the iteration runs in the HIP kernels
of libmato.so.  The functions below carry the C names; ``Plan`` and ``Batch``
are thin owners of the handles.  Arrays may be NumPy arrays (host) or torch
tensors (host or device); they are passed by pointer.  The library must have
been built (``python -m paper_2011_04240_amd.build``): loading fails loudly
otherwise, there is no fallback.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmato.so")

MATO_OK = 0
MATO_ERR_INVALID_ARG = -1
MATO_ERR_OUT_OF_MEMORY = -2
MATO_ERR_SINGULAR = -3
MATO_ERR_NONFINITE = -4
MATO_ERR_HIP = -5
MATO_ERR_UNSUPPORTED = -6
MATO_ERR_NOT_FOUND = -7
MATO_WARN_NOT_CONVERGED = 1
MATO_MAX_AGENTS = 160
MATO_MAX_STAGES = 16
MATO_MAX_OBSTACLES = 1024
MATO_HISTORY_CAP = 4096

MATO_FP64, MATO_FP32, MATO_BF16_REFINED = 0, 1, 2
PRECISIONS = {"fp64": MATO_FP64, "fp32": MATO_FP32, "bf16": MATO_BF16_REFINED}
MATO_SOLVE_DENSE, MATO_SOLVE_STRUCTURED = 0, 1
SOLVES = {"dense": MATO_SOLVE_DENSE, "structured": MATO_SOLVE_STRUCTURED}


class MatoError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("mato status %d: %s" % (status, msg))
        self.status = status


class _Basis(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n_coef", ctypes.c_int32), ("t_final", ctypes.c_double)]


class PlanDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("n_obs", ctypes.c_int32), ("T", ctypes.c_int32), ("basis", _Basis),
                ("a", ctypes.c_double), ("b", ctypes.c_double), ("precision", ctypes.c_int32),
                ("solve", ctypes.c_int32)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("T", ctypes.c_int32), ("basis", _Basis), ("a", ctypes.c_double), ("b", ctypes.c_double),
                ("rho", ctypes.c_double), ("precision", ctypes.c_int32), ("max_slots", ctypes.c_int32),
                ("hbm_budget_bytes", ctypes.c_double), ("chunk", ctypes.c_int32), ("max_iters", ctypes.c_int32),
                ("tol", ctypes.c_double), ("projection", ctypes.c_int32), ("rho_stages", ctypes.c_int32),
                ("rho_values", ctypes.c_double * 16), ("rho_start", ctypes.c_int32 * 16), ("solve", ctypes.c_int32),
                ("use_graphs", ctypes.c_int32)]


_lib = None
_vp, _i32, _f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
_pi32, _pf64, _pvp = ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_void_p)

# name -> (restype, argtypes)
SIGNATURES = {
    "mato_last_error": (ctypes.c_char_p, []),
    "mato_version": (ctypes.c_char_p, []),
    "mato_plan_create": (_i32, [_i32, _i32, ctypes.POINTER(_Basis), _f64, _f64, _f64, _i32, _vp, _pvp]),
    "mato_plan_destroy": (None, [_vp]),
    "mato_plan_create_many": (_i32, [_i32, _i32, ctypes.POINTER(_Basis), _f64, _f64, _pf64, _i32, _i32, _vp, _pvp]),
    "mato_plan_create_ex": (_i32, [ctypes.POINTER(PlanDesc), _pf64, _i32, _vp, _pvp]),
    "mato_plan_describe": (_i32, [_vp, ctypes.POINTER(PlanDesc), _pf64]),
    "mato_plan_info": (_i32, [_vp, _pi32, _pi32, _pi32, _pi32, _pf64]),
    "mato_plan_inverse": (_i32, [_vp, _vp]),
    "mato_batch_create": (_i32, [_i32, _pvp, _vp, _vp, _vp, _pvp]),
    "mato_batch_create_ex": (_i32, [_i32, _pvp, _vp, _vp, _vp, _vp, _pvp]),
    "mato_batch_destroy": (None, [_vp]),
    "mato_batch_step": (_i32, [_vp, _i32, _f64, _i32]),
    "mato_batch_run": (_i32, [_vp, _i32, _f64, _i32]),
    "mato_batch_sync": (_i32, [_vp]),
    "mato_batch_status": (_i32, [_vp, _i32, _pi32, _pi32]),
    "mato_batch_coeffs": (_i32, [_vp, _i32, _vp]),
    "mato_batch_residuals": (_i32, [_vp, _i32, _vp, _vp, _vp, _i32, _pi32]),
    "mato_batch_debug": (_i32, [_vp, _i32]),
    "mato_batch_get_state": (_i32, [_vp, _i32, _vp, _vp, _vp, _vp, _vp]),
    "mato_batch_set_state": (_i32, [_vp, _i32, _vp, _vp, _vp]),
    "mato_batch_linear_term": (_i32, [_vp, _i32, _vp]),
    "mato_batch_set_rho_schedule": (_i32, [_vp, _i32, _pvp, _pi32]),
    "mato_batch_set_projection": (_i32, [_vp, _i32]),
    "mato_batch_set_tiles": (_i32, [_vp, _i32, _i32]),
    "mato_batch_get_tiles": (_i32, [_vp, _pi32, _pi32]),
    "mato_batch_autotune": (_i32, [_vp, _pi32, _pi32]),
    "mato_batch_timing": (_i32, [_vp, _i32]),
    "mato_batch_last_times": (_i32, [_vp, _pf64, _pf64, _pi32]),
    "mato_server_create": (_i32, [ctypes.POINTER(ServerConfig), _vp, _pvp]),
    "mato_server_destroy": (None, [_vp]),
    "mato_server_warm": (_i32, [_vp, _i32, _i32]),
    "mato_server_submit": (_i32, [_vp, _i32, _vp, _vp, ctypes.POINTER(ctypes.c_int64)]),
    "mato_server_submit_ex": (_i32, [_vp, _i32, _vp, _vp, _i32, _vp, ctypes.POINTER(ctypes.c_int64)]),
    "mato_server_step": (_i32, [_vp, _pi32, _pi32]),
    "mato_server_poll": (_i32, [_vp, ctypes.c_int64, _pi32, _pi32, _pi32, _pf64]),
    "mato_server_result": (_i32, [_vp, ctypes.c_int64, _vp]),
    "mato_server_stats": (_i32, [_vp, _pf64, _pi32, _pi32, _pi32]),
    "mato_server_run_trace": (_i32, [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _pf64]),
    "mato_solve_run": (_i32, [_vp, _vp, _vp, _i32, _f64, _i32, _pvp]),
    "mato_solve_coeffs": (_i32, [_vp, _vp]),
    "mato_residuals": (_i32, [_vp, _vp, _vp, _vp, _i32, _pi32]),
    "mato_solve_destroy": (None, [_vp]),
    "mato_solve_sync": (_i32, [_vp]),
    "mato_step": (_i32, [_vp, _i32]),
    "mato_get_state": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "mato_set_state": (_i32, [_vp, _vp, _vp, _vp]),
    "mato_solve_noalloc": (_i32, [_vp, _vp, _vp, _i32, _f64, _i32, _vp, _vp, _vp, _vp, _i32, _pi32, _pi32, _pi32]),
    "mato_stream_copy": (_i32, [ctypes.c_int64, _i32, _i32, _vp, _pf64]),
    "mato_stream_update": (_i32, [ctypes.c_int64, _i32, _i32, _vp, _pf64]),
    "mato_stream_read": (_i32, [ctypes.c_int64, _i32, _i32, _vp, _pf64]),
    "mato_stream_create": (_i32, [_pvp]),
    "mato_stream_destroy": (_i32, [_vp]),
}


def lib():
    """Load libmato.so (built in-tree).  Raises if it is missing: there is no fallback."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libmato.so not built at %s; run `python -m paper_2011_04240_amd.build`" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status):
    if status < 0:
        raise MatoError(status, lib().mato_last_error().decode())
    return status


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, np.ndarray):
        if not x.flags["C_CONTIGUOUS"]:
            raise ValueError("array must be C-contiguous")
        return ctypes.c_void_p(x.ctypes.data)
    if hasattr(x, "data_ptr"):
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return ctypes.c_void_p(x.data_ptr())
    raise TypeError("expected a NumPy array or a torch tensor, got %r" % type(x))


def _stream_ptr(stream):
    if stream is None:
        return None
    if isinstance(stream, Stream):
        return stream.handle
    if hasattr(stream, "cuda_stream"):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


class Stream:
    """A HIP stream created by the library's runtime (batches on different streams overlap)."""

    def __init__(self):
        h = ctypes.c_void_p()
        _check(lib().mato_stream_create(ctypes.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib().mato_stream_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --------------------------------------------------------- thin C wrappers ---
def mato_version():
    return lib().mato_version().decode()


def mato_plan_create(n, T, n_coef, t_final, a, b, rho, precision, stream=None):
    h = ctypes.c_void_p()
    basis = _Basis(0, n_coef, t_final)
    _check(lib().mato_plan_create(n, T, ctypes.byref(basis), a, b, rho, precision, _stream_ptr(stream),
                                  ctypes.byref(h)))
    return h


def mato_plan_create_many(n, T, n_coef, t_final, a, b, rhos, precision, stream=None):
    out = (ctypes.c_void_p * len(rhos))()
    r = (ctypes.c_double * len(rhos))(*rhos)
    basis = _Basis(0, n_coef, t_final)
    _check(lib().mato_plan_create_many(n, T, ctypes.byref(basis), a, b, r, len(rhos), precision,
                                       _stream_ptr(stream), out))
    return [ctypes.c_void_p(x) for x in out]


def mato_plan_create_ex(desc, rhos, stream=None):
    out = (ctypes.c_void_p * len(rhos))()
    r = (ctypes.c_double * len(rhos))(*rhos)
    _check(lib().mato_plan_create_ex(ctypes.byref(desc), r, len(rhos), _stream_ptr(stream), out))
    return [ctypes.c_void_p(x) for x in out]


def mato_plan_describe(plan):
    d = PlanDesc()
    rho = _f64()
    _check(lib().mato_plan_describe(plan, ctypes.byref(d), ctypes.byref(rho)))
    return d, rho.value


def mato_plan_destroy(plan):
    lib().mato_plan_destroy(plan)


def mato_plan_info(plan):
    n, T, nc, pr = _i32(), _i32(), _i32(), _i32()
    cond = _f64()
    _check(lib().mato_plan_info(plan, ctypes.byref(n), ctypes.byref(T), ctypes.byref(nc), ctypes.byref(pr),
                                ctypes.byref(cond)))
    return n.value, T.value, nc.value, pr.value, cond.value


def mato_plan_inverse(plan, out):
    _check(lib().mato_plan_inverse(plan, _ptr(out)))


def mato_batch_create(plans, starts, goals, stream=None):
    arr = (ctypes.c_void_p * len(plans))(*[p.value if isinstance(p, ctypes.c_void_p) else p for p in plans])
    h = ctypes.c_void_p()
    _check(lib().mato_batch_create(len(plans), arr, _ptr(starts), _ptr(goals), _stream_ptr(stream),
                                   ctypes.byref(h)))
    return h


def mato_batch_create_ex(plans, starts, goals, obstacles, stream=None):
    arr = (ctypes.c_void_p * len(plans))(*[p.value if isinstance(p, ctypes.c_void_p) else p for p in plans])
    h = ctypes.c_void_p()
    _check(lib().mato_batch_create_ex(len(plans), arr, _ptr(starts), _ptr(goals), _ptr(obstacles),
                                      _stream_ptr(stream), ctypes.byref(h)))
    return h


def mato_batch_destroy(batch):
    lib().mato_batch_destroy(batch)


def mato_batch_step(batch, k, tol=0.0, use_graph=True):
    return _check(lib().mato_batch_step(batch, k, tol, int(bool(use_graph))))


def mato_batch_run(batch, iters, tol=0.0, check_every=10):
    return _check(lib().mato_batch_run(batch, iters, tol, check_every))


def mato_batch_sync(batch):
    return _check(lib().mato_batch_sync(batch))


def mato_batch_status(batch, q):
    it, conv = _i32(), _i32()
    _check(lib().mato_batch_status(batch, q, ctypes.byref(it), ctypes.byref(conv)))
    return it.value, bool(conv.value)


def mato_batch_coeffs(batch, q, out):
    _check(lib().mato_batch_coeffs(batch, q, _ptr(out)))


def mato_batch_residuals(batch, q, r_max, r_rms, cost, cap):
    nw = _i32()
    _check(lib().mato_batch_residuals(batch, q, _ptr(r_max), _ptr(r_rms), _ptr(cost), cap, ctypes.byref(nw)))
    return nw.value


def mato_batch_debug(batch, enable):
    _check(lib().mato_batch_debug(batch, int(bool(enable))))


def mato_batch_get_state(batch, q, c=None, lam=None, proj=None, d=None, X=None):
    _check(lib().mato_batch_get_state(batch, q, _ptr(c), _ptr(lam), _ptr(proj), _ptr(d), _ptr(X)))


def mato_batch_set_state(batch, q, c, lam, proj):
    _check(lib().mato_batch_set_state(batch, q, _ptr(c), _ptr(lam), _ptr(proj)))


def mato_batch_linear_term(batch, q, out):
    _check(lib().mato_batch_linear_term(batch, q, _ptr(out)))


def mato_batch_set_rho_schedule(batch, plans, start_iter):
    """plans: stage-major list of plan handles ([stage][problem]); start_iter per stage."""
    arr = (ctypes.c_void_p * len(plans))(*[p.value if isinstance(p, ctypes.c_void_p) else p for p in plans])
    st = (ctypes.c_int32 * len(start_iter))(*start_iter)
    _check(lib().mato_batch_set_rho_schedule(batch, len(start_iter), arr, st))


def mato_batch_set_projection(batch, mode):
    _check(lib().mato_batch_set_projection(batch, mode))


def mato_batch_set_tiles(batch, items_per_wg, threads):
    _check(lib().mato_batch_set_tiles(batch, items_per_wg, threads))


def mato_batch_get_tiles(batch):
    a, b = _i32(), _i32()
    _check(lib().mato_batch_get_tiles(batch, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def mato_batch_autotune(batch):
    a, b = _i32(), _i32()
    _check(lib().mato_batch_autotune(batch, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def mato_batch_timing(batch, enable):
    _check(lib().mato_batch_timing(batch, int(bool(enable))))


def mato_batch_last_times(batch):
    t, p, n = _f64(), _f64(), _i32()
    _check(lib().mato_batch_last_times(batch, ctypes.byref(t), ctypes.byref(p), ctypes.byref(n)))
    return t.value, p.value, n.value


def mato_server_create(cfg, stream=None):
    h = ctypes.c_void_p()
    _check(lib().mato_server_create(ctypes.byref(cfg), _stream_ptr(stream), ctypes.byref(h)))
    return h


def mato_server_destroy(server):
    lib().mato_server_destroy(server)


def mato_server_warm(server, n_min, n_max):
    _check(lib().mato_server_warm(server, n_min, n_max))


def mato_server_submit(server, n, starts, goals):
    i = ctypes.c_int64()
    _check(lib().mato_server_submit(server, n, _ptr(starts), _ptr(goals), ctypes.byref(i)))
    return i.value


def mato_server_submit_ex(server, n, starts, goals, n_obs, obstacles):
    i = ctypes.c_int64()
    _check(lib().mato_server_submit_ex(server, n, _ptr(starts), _ptr(goals), n_obs, _ptr(obstacles),
                                       ctypes.byref(i)))
    return i.value


def mato_server_step(server):
    r, q = _i32(), _i32()
    _check(lib().mato_server_step(server, ctypes.byref(r), ctypes.byref(q)))
    return r.value, q.value


def mato_server_poll(server, req):
    st, it, cv = _i32(), _i32(), _i32()
    rm = _f64()
    _check(lib().mato_server_poll(server, req, ctypes.byref(st), ctypes.byref(it), ctypes.byref(cv), ctypes.byref(rm)))
    return st.value, it.value, bool(cv.value), rm.value


def mato_server_result(server, req, out):
    _check(lib().mato_server_result(server, req, _ptr(out)))


def mato_server_stats(server):
    b, p, r, q = _f64(), _i32(), _i32(), _i32()
    _check(lib().mato_server_stats(server, ctypes.byref(b), ctypes.byref(p), ctypes.byref(r), ctypes.byref(q)))
    return b.value, p.value, r.value, q.value


def mato_server_run_trace(server, arrival_s, ns, starts, goals, latency, iters, converged):
    wall = _f64()
    _check(lib().mato_server_run_trace(server, len(ns), _ptr(arrival_s), _ptr(ns), _ptr(starts), _ptr(goals),
                                       _ptr(latency), _ptr(iters), _ptr(converged), ctypes.byref(wall)))
    return wall.value


# ---------------------------------------------------- single-problem wrappers ---
def mato_solve_run(plan, starts, goals, iters, tol=0.0, check_every=10):
    h = ctypes.c_void_p()
    status = _check(lib().mato_solve_run(plan, _ptr(starts), _ptr(goals), iters, tol, check_every, ctypes.byref(h)))
    return h, status


def mato_solve_sync(solve):
    _check(lib().mato_solve_sync(solve))


def mato_step(solve, k):
    _check(lib().mato_step(solve, k))


def mato_solve_coeffs(solve, out):
    _check(lib().mato_solve_coeffs(solve, _ptr(out)))


def mato_residuals(solve, r_max, r_rms, cost, cap):
    nw = _i32()
    _check(lib().mato_residuals(solve, _ptr(r_max), _ptr(r_rms), _ptr(cost), cap, ctypes.byref(nw)))
    return nw.value


def mato_get_state(solve, c=None, lam=None, proj=None, d=None, X=None):
    _check(lib().mato_get_state(solve, _ptr(c), _ptr(lam), _ptr(proj), _ptr(d), _ptr(X)))


def mato_set_state(solve, c, lam, proj):
    _check(lib().mato_set_state(solve, _ptr(c), _ptr(lam), _ptr(proj)))


def mato_solve_destroy(solve):
    lib().mato_solve_destroy(solve)


def mato_solve_noalloc(plan, starts, goals, iters, tol, check_every, c, r_max, r_rms, cost, cap):
    """Returns (status, entries written, iterations done, converged)."""
    nw, it, conv = _i32(), _i32(), _i32()
    status = _check(lib().mato_solve_noalloc(plan, _ptr(starts), _ptr(goals), iters, tol, check_every, _ptr(c),
                                             _ptr(r_max), _ptr(r_rms), _ptr(cost), cap, ctypes.byref(nw),
                                             ctypes.byref(it), ctypes.byref(conv)))
    return status, nw.value, it.value, conv.value


def mato_stream_copy(nbytes, grid=1024, iters=10, stream=None):
    ms = _f64()
    _check(lib().mato_stream_copy(nbytes, grid, iters, _stream_ptr(stream), ctypes.byref(ms)))
    return ms.value


def mato_stream_update(nbytes, grid=1024, iters=10, stream=None):
    ms = _f64()
    _check(lib().mato_stream_update(nbytes, grid, iters, _stream_ptr(stream), ctypes.byref(ms)))
    return ms.value


def mato_stream_read(nbytes, grid=1024, iters=10, stream=None):
    ms = _f64()
    _check(lib().mato_stream_read(nbytes, grid, iters, _stream_ptr(stream), ctypes.byref(ms)))
    return ms.value


# ---------------------------------------------------------------- owners ---
def plan_desc(n, T, n_coef=11, t_final=10.0, a=0.3, b=0.6, precision="fp32", solve="dense", n_obs=0):
    pr = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    sv = SOLVES[solve] if isinstance(solve, str) else int(solve)
    return PlanDesc(n, n_obs, T, _Basis(0, n_coef, t_final), a, b, pr, sv)


class Plan:
    """K^{-1} of the x/y/z step for one (n, n_obs, T, basis, rho); a, b are the spheroid dimensions."""

    def __init__(self, n, T, n_coef=11, t_final=10.0, a=0.3, b=0.6, rho=1.0, precision="fp32", stream=None,
                 handle=None, solve="dense", n_obs=0):
        self.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        self.solve = SOLVES[solve] if isinstance(solve, str) else int(solve)
        self.n, self.T, self.n_coef, self.n_obs = n, T, n_coef, n_obs
        self.t_final, self.a, self.b, self.rho = t_final, a, b, rho
        if handle is None:
            desc = plan_desc(n, T, n_coef, t_final, a, b, self.precision, self.solve, n_obs)
            handle = mato_plan_create_ex(desc, [rho], stream)[0]
        self.handle = handle

    @classmethod
    def schedule(cls, n, T, rhos, n_coef=11, t_final=10.0, a=0.3, b=0.6, precision="fp32", stream=None,
                 solve="dense", n_obs=0):
        """Plans for several rho (a rho schedule), inverted together."""
        desc = plan_desc(n, T, n_coef, t_final, a, b, precision, solve, n_obs)
        hs = mato_plan_create_ex(desc, list(rhos), stream)
        return [cls(n, T, n_coef, t_final, a, b, r, desc.precision, handle=h, solve=desc.solve, n_obs=n_obs)
                for r, h in zip(rhos, hs)]

    @property
    def n_rows(self):
        """Collision rows: agent pairs, then agent-obstacle pairs."""
        return self.n * (self.n - 1) // 2 + self.n * self.n_obs

    @property
    def scalar(self):
        return np.float64 if self.precision == MATO_FP64 else np.float32

    def info(self):
        return mato_plan_info(self.handle)

    def inverse(self):
        N = self.n * (self.n_coef + 6)
        out = np.empty((N, N), dtype=np.float64)
        mato_plan_inverse(self.handle, out)
        return out

    def close(self):
        if getattr(self, "handle", None):
            mato_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching request loop (problems of any agent count up to MATO_MAX_AGENTS)."""

    def __init__(self, T=100, n_coef=11, t_final=10.0, a=0.3, b=0.6, rho=1.0, precision="fp32", max_slots=64,
                 hbm_budget_bytes=0.0, chunk=10, max_iters=2000, tol=1e-3, shifted=False, rho_schedule=None,
                 stream=None, solve="dense", use_graphs=False):
        self.T, self.n_coef = T, n_coef
        self.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        cfg = ServerConfig(T, _Basis(0, n_coef, t_final), a, b, rho, self.precision, max_slots, hbm_budget_bytes,
                           chunk, max_iters, tol, int(bool(shifted)))
        cfg.solve = SOLVES[solve] if isinstance(solve, str) else int(solve)
        cfg.use_graphs = int(bool(use_graphs))
        if rho_schedule is not None:
            values, starts = rho_schedule
            cfg.rho_stages = len(values)
            for j, (v, t) in enumerate(zip(values, starts)):
                cfg.rho_values[j] = v
                cfg.rho_start[j] = t
        self.handle = mato_server_create(cfg, stream)

    def warm(self, n_min, n_max):
        mato_server_warm(self.handle, n_min, n_max)

    def submit(self, starts, goals, obstacles=None):
        """obstacles: optional [n_obs][x, y, z, l_xy, l_z] static obstacles of this request."""
        starts = np.ascontiguousarray(starts, np.float64)
        goals = np.ascontiguousarray(goals, np.float64)
        if obstacles is None or len(obstacles) == 0:
            return mato_server_submit(self.handle, starts.shape[0], starts, goals)
        obs = np.ascontiguousarray(np.asarray(obstacles, np.float64).reshape(-1, 5))
        return mato_server_submit_ex(self.handle, starts.shape[0], starts, goals, obs.shape[0], obs)

    def step(self):
        return mato_server_step(self.handle)

    def poll(self, req):
        return mato_server_poll(self.handle, req)

    def result(self, req, n):
        out = np.empty((n, 3, self.n_coef), np.float64)
        mato_server_result(self.handle, req, out)
        return out

    def stats(self):
        return mato_server_stats(self.handle)

    def run_trace(self, arrival_s, starts_list, goals_list):
        ns = np.ascontiguousarray([np.asarray(s).shape[0] for s in starts_list], np.int32)
        arr = np.ascontiguousarray(arrival_s, np.float64)
        if len(ns) == 0:
            wall = mato_server_run_trace(self.handle, arr, ns, None, None, None, None, None)
            return np.zeros(0), np.zeros(0, np.int32), np.zeros(0, np.int32), wall
        starts = np.ascontiguousarray(np.concatenate([np.asarray(s, np.float64).reshape(-1, 3) for s in starts_list]))
        goals = np.ascontiguousarray(np.concatenate([np.asarray(g, np.float64).reshape(-1, 3) for g in goals_list]))
        lat = np.zeros(len(ns))
        its = np.zeros(len(ns), np.int32)
        conv = np.zeros(len(ns), np.int32)
        wall = mato_server_run_trace(self.handle, arr, ns, starts, goals, lat, its, conv)
        return lat, its, conv, wall

    def close(self):
        if getattr(self, "handle", None):
            mato_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Independent problems iterated together; problem q uses plans[q]."""

    def __init__(self, plans, starts_list, goals_list, stream=None, obstacles_list=None):
        """obstacles_list[q]: problem q's obstacles [n_obs][x, y, z, l_xy, l_z] (plans with n_obs > 0)."""
        self.plans = list(plans)
        self.ns = [p.n for p in self.plans]
        starts = np.ascontiguousarray(np.concatenate([np.asarray(s, np.float64).reshape(-1, 3) for s in starts_list]))
        goals = np.ascontiguousarray(np.concatenate([np.asarray(g, np.float64).reshape(-1, 3) for g in goals_list]))
        obs = None
        if obstacles_list is not None:
            rows = [np.asarray(o, np.float64).reshape(-1, 5) for o in obstacles_list]
            if sum(len(r) for r in rows):
                obs = np.ascontiguousarray(np.concatenate(rows))
        self.handle = mato_batch_create_ex([p.handle for p in self.plans], starts, goals, obs, stream)

    def __len__(self):
        return len(self.plans)

    def step(self, k, tol=0.0, use_graph=True):
        return mato_batch_step(self.handle, k, tol, use_graph)

    def run(self, iters, tol=0.0, check_every=10):
        return mato_batch_run(self.handle, iters, tol, check_every)

    def sync(self):
        mato_batch_sync(self.handle)

    def status(self, q):
        return mato_batch_status(self.handle, q)

    def coeffs(self, q):
        p = self.plans[q]
        out = np.empty((p.n, 3, p.n_coef), dtype=np.float64)
        mato_batch_coeffs(self.handle, q, out)
        return out

    def residuals(self, q, cap=1 << 20):
        it, _ = self.status(q)
        m = max(0, min(it, cap))
        r_max, r_rms, cost = (np.empty(max(m, 1)) for _ in range(3))
        w = mato_batch_residuals(self.handle, q, r_max, r_rms, cost, m)
        return r_max[:w], r_rms[:w], cost[:w]

    def debug(self, enable=True):
        mato_batch_debug(self.handle, enable)

    def get_state(self, q, proj=False, d=False, X=False):
        p = self.plans[q]
        np_, S = p.n_rows, p.scalar
        c = np.empty((p.n, 3, p.n_coef), np.float64)
        lam = np.empty((np_, p.T, 3), S)
        pj = np.empty((np_, p.T, 3), S) if proj else None
        dd = np.empty((np_, p.T), S) if d else None
        xx = np.empty((p.n, 3, p.T), S) if X else None
        mato_batch_get_state(self.handle, q, c, lam, pj, dd, xx)
        out = dict(c=c, lam=lam)
        if proj:
            out["proj"] = pj
        if d:
            out["d"] = dd
        if X:
            out["X"] = xx
        return out

    def set_state(self, q, c, lam, proj):
        S = self.plans[q].scalar
        mato_batch_set_state(self.handle, q, np.ascontiguousarray(c, np.float64),
                             np.ascontiguousarray(lam, S), np.ascontiguousarray(proj, S))

    def linear_term(self, q):
        p = self.plans[q]
        out = np.empty((p.n, 3, p.n_coef), np.float64)
        mato_batch_linear_term(self.handle, q, out)
        return out

    def set_rho_schedule(self, stage_plans, start_iter):
        """stage_plans[j][q]: problem q's plan in stage j (stage 0: the creation plans)."""
        flat = [p.handle for stage in stage_plans for p in stage]
        self._stage_plans = stage_plans            # keep them alive with the batch
        mato_batch_set_rho_schedule(self.handle, flat, list(start_iter))

    def set_projection(self, shifted):
        mato_batch_set_projection(self.handle, int(bool(shifted)))

    def set_tiles(self, items_per_wg, threads):
        mato_batch_set_tiles(self.handle, items_per_wg, threads)

    def get_tiles(self):
        return mato_batch_get_tiles(self.handle)

    def autotune(self):
        return mato_batch_autotune(self.handle)

    def timing(self, enable=True):
        mato_batch_timing(self.handle, enable)

    def last_times(self):
        return mato_batch_last_times(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            mato_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
