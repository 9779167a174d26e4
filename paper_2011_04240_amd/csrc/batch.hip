// C ABI of batches and single solves (include/mato.h) on top of the engine
// (engine.h): a fixed set of independent problems placed in one device arena and
// advanced together, one pass of the while-loop of Algorithm 1 per iteration.
#include <mutex>

#include "engine.h"

namespace mato {

static_assert(kHistCap == MATO_HISTORY_CAP, "device history capacity differs from the header's");

template <typename S>
using BatchImpl = Engine<S>;

// ----------------------------------------------------------- creation ---
// ext: when not null, every device buffer of the batch is carved from this region of
// ext_cap bytes (no device allocation, no graphs, no pinned staging).
template <typename S>
static mato_status batch_create(int count, const mato_plan* plans, const double* starts,
                                const double* goals, const double* obstacles, hipStream_t st,
                                BatchImpl<S>** out, char* ext = nullptr, size_t ext_cap = 0) {
    auto* B = new BatchImpl<S>();
    B->ext = ext;
    B->ext_cap = ext_cap;
    B->precision = plans[0]->precision;
    B->solve = plans[0]->solve;
    B->refine = (B->precision == MATO_FP32) ? 1 : (B->precision == MATO_BF16_REFINED ? 2 : 0);
    if (const char* e = getenv("MATO_REFINE")) {
        B->refine = std::max(0, std::min(kMaxRefine, atoi(e)));
        B->refine_fixed = true;
    }
    if (B->solve == MATO_SOLVE_STRUCTURED) B->refine = 0;     // the structured step is FP64 throughout
    B->refine_base = B->refine;
    B->stream = st;
    auto fail = [&](mato_status s) { delete B; return s; };
    int agents = 0, nobs = 0;
    std::vector<size_t> offs;
    size_t total = 0;
    for (int q = 0; q < count; ++q) {
        offs.push_back(total);
        total += BatchImpl<S>::slot_bytes(plans[q]);
        agents += plans[q]->n;
        nobs += plans[q]->n_obs;
    }
    if (nobs > 0 && !obstacles) {
        set_error("the plans have %d obstacles in total but none were given", nobs);
        return fail(MATO_ERR_INVALID_ARG);
    }
    std::vector<double> hs((size_t)agents * 3), hg((size_t)agents * 3), ho((size_t)nobs * 5);
    if (hipMemcpy(hs.data(), starts, sizeof(double) * hs.size(), hipMemcpyDefault) != hipSuccess ||
        hipMemcpy(hg.data(), goals, sizeof(double) * hg.size(), hipMemcpyDefault) != hipSuccess ||
        (nobs > 0 && hipMemcpy(ho.data(), obstacles, sizeof(double) * ho.size(), hipMemcpyDefault) != hipSuccess)) {
        (void)hipGetLastError();
        set_error("cannot read starts/goals/obstacles");
        return fail(MATO_ERR_INVALID_ARG);
    }
    mato_status s;
    if ((s = B->init_capacity(count)) != MATO_OK) return fail(s);
    B->arena_bytes = std::max<size_t>(total, 256);
    if (ext) {
        size_t cap = 0;
        if ((s = B->dev_buf(&B->arena, &cap, B->arena_bytes)) != MATO_OK) return fail(s);
    } else if (hipMalloc(&B->arena, B->arena_bytes) != hipSuccess) {
        (void)hipGetLastError();
        set_error("device allocation of %zu bytes failed", B->arena_bytes);
        return fail(MATO_ERR_OUT_OF_MEMORY);
    }
    if (hipMemsetAsync(B->arena, 0, B->arena_bytes, st) != hipSuccess) {
        set_error("arena clear failed");
        return fail(MATO_ERR_HIP);
    }
    int a0 = 0, o0 = 0;
    for (int q = 0; q < count; ++q) {
        if ((s = B->attach(q, plans[q], &hs[(size_t)a0 * 3], &hg[(size_t)a0 * 3], B->arena + offs[q],
                           plans[q]->n_obs ? &ho[(size_t)o0 * 5] : nullptr)) != MATO_OK)
            return fail(s);
        a0 += plans[q]->n;
        o0 += plans[q]->n_obs;
    }
    if ((s = B->enqueue_init_all()) != MATO_OK) return fail(s);
    if (hipStreamSynchronize(st) != hipSuccess) {
        set_error("initialisation failed: %s", hipGetErrorString(hipGetLastError()));
        return fail(MATO_ERR_HIP);
    }
    *out = B;
    return MATO_OK;
}

template <typename F>
static mato_status dispatch(mato_batch b, F&& f) {
    if (!b || !b->impl) { set_error("null batch"); return MATO_ERR_INVALID_ARG; }
    if (b->precision == MATO_FP64) return f(static_cast<BatchImpl<double>*>(b->impl));
    return f(static_cast<BatchImpl<float>*>(b->impl));
}

template <typename S>
static mato_status check_q(BatchImpl<S>* B, int q) {
    if (q < 0 || q >= B->count()) { set_error("problem index %d out of range", q); return MATO_ERR_INVALID_ARG; }
    return MATO_OK;
}

// host staging + copy to a caller pointer of unknown kind
static mato_status copy_out(void* dst, const void* src, size_t bytes) {
    MATO_HIP(hipMemcpy(dst, src, bytes, hipMemcpyDefault));
    return MATO_OK;
}

}  // namespace mato

using namespace mato;

// ---------------------------------------------------------------- C ABI ---
extern "C" mato_status mato_batch_create(int32_t count, const mato_plan* plans, const double* starts,
                                         const double* goals, void* hip_stream, mato_batch* out) {
    return mato_batch_create_ex(count, plans, starts, goals, nullptr, hip_stream, out);
}

extern "C" mato_status mato_batch_create_ex(int32_t count, const mato_plan* plans, const double* starts,
                                            const double* goals, const double* obstacles, void* hip_stream,
                                            mato_batch* out) {
    if (!out || !plans || !starts || !goals || count < 1) { set_error("invalid arguments"); return MATO_ERR_INVALID_ARG; }
    *out = nullptr;
    for (int q = 0; q < count; ++q)
        if (!plans[q] || plans[q]->precision != plans[0]->precision || plans[q]->solve != plans[0]->solve) {
            set_error("plan %d is null or of another precision or solve kind", q);
            return MATO_ERR_INVALID_ARG;
        }
    auto* b = new mato_batch_s();
    b->precision = plans[0]->precision;
    mato_status s;
    if (b->precision == MATO_FP64) {
        BatchImpl<double>* B = nullptr;
        s = batch_create<double>(count, plans, starts, goals, obstacles, (hipStream_t)hip_stream, &B);
        b->impl = B;
    } else {
        BatchImpl<float>* B = nullptr;
        s = batch_create<float>(count, plans, starts, goals, obstacles, (hipStream_t)hip_stream, &B);
        b->impl = B;
    }
    if (s != MATO_OK) { delete b; return s; }
    *out = b;
    return MATO_OK;
}

extern "C" void mato_batch_destroy(mato_batch b) {
    if (!b) return;
    if (b->impl) {
        if (b->precision == MATO_FP64) {
            auto* B = static_cast<BatchImpl<double>*>(b->impl);
            (void)hipStreamSynchronize(B->stream);
            delete B;
        } else {
            auto* B = static_cast<BatchImpl<float>*>(b->impl);
            (void)hipStreamSynchronize(B->stream);
            delete B;
        }
    }
    delete b;
}

extern "C" mato_status mato_batch_step(mato_batch b, int32_t k, double tol, int32_t use_graph) {
    return dispatch(b, [&](auto* B) { return B->step(k, tol, use_graph != 0); });
}

extern "C" mato_status mato_batch_run(mato_batch b, int32_t iters, double tol, int32_t check_every) {
    return dispatch(b, [&](auto* B) { return B->run(iters, tol, check_every); });
}

extern "C" mato_status mato_batch_sync(mato_batch b) {
    return dispatch(b, [&](auto* B) -> mato_status {
        MATO_HIP(hipStreamSynchronize(B->stream));
        return MATO_OK;
    });
}

extern "C" mato_status mato_batch_status(mato_batch b, int32_t q, int32_t* iters, int32_t* converged) {
    return dispatch(b, [&](auto* B) -> mato_status {
        MATO_TRY(check_q(B, q));
        std::vector<int> ctrl;
        MATO_TRY(B->read_ctrl(ctrl));
        if (iters) *iters = ctrl[kCtrl * q];
        if (converged) *converged = ctrl[kCtrl * q + 4];
        if (ctrl[kCtrl * q + 2]) { set_error("problem %d produced non-finite values", q); return MATO_ERR_NONFINITE; }
        return MATO_OK;
    });
}

extern "C" mato_status mato_batch_coeffs(mato_batch b, int32_t q, double* c) {
    return dispatch(b, [&](auto* B) -> mato_status {
        MATO_TRY(check_q(B, q));
        if (!c) { set_error("null output"); return MATO_ERR_INVALID_ARG; }
        const auto& P = B->probs[q];
        std::vector<double> h((size_t)3 * P.ldc), o((size_t)P.n * 3 * P.nv);
        MATO_HIP(hipStreamSynchronize(B->stream));
        MATO_HIP(hipMemcpy(h.data(), P.base + P.o_c, sizeof(double) * h.size(), hipMemcpyDeviceToHost));
        for (int i = 0; i < P.n; ++i)
            for (int a = 0; a < 3; ++a)
                for (int k = 0; k < P.nv; ++k)
                    o[((size_t)i * 3 + a) * P.nv + k] = h[(size_t)a * P.ldc + (size_t)i * P.nv + k];
        return copy_out(c, o.data(), sizeof(double) * o.size());
    });
}

extern "C" mato_status mato_batch_residuals(mato_batch b, int32_t q, double* r_max, double* r_rms,
                                            double* cost, int32_t cap, int32_t* n_written) {
    return dispatch(b, [&](auto* B) -> mato_status {
        MATO_TRY(check_q(B, q));
        std::vector<int> ctrl;
        MATO_TRY(B->read_ctrl(ctrl));
        const int it = std::min(std::min(ctrl[kCtrl * q], kHistCap), std::max(0, (int)cap));
        std::vector<double> h((size_t)3 * std::max(it, 1));
        const auto& P = B->probs[q];
        if (it > 0) MATO_HIP(hipMemcpy(h.data(), P.base + P.o_hist, sizeof(double) * 3 * it, hipMemcpyDeviceToHost));
        std::vector<double> o0(it), o1(it), o2(it);
        for (int k = 0; k < it; ++k) { o0[k] = h[3 * k]; o1[k] = h[3 * k + 1]; o2[k] = h[3 * k + 2]; }
        if (it > 0) {
            if (r_max) MATO_TRY(copy_out(r_max, o0.data(), sizeof(double) * it));
            if (r_rms) MATO_TRY(copy_out(r_rms, o1.data(), sizeof(double) * it));
            if (cost) MATO_TRY(copy_out(cost, o2.data(), sizeof(double) * it));
        }
        if (n_written) *n_written = it;
        return MATO_OK;
    });
}

extern "C" mato_status mato_batch_debug(mato_batch b, int32_t enable) {
    return dispatch(b, [&](auto* B) { return B->enable_debug(enable != 0); });
}

template <typename S>
static mato_status get_state_impl(BatchImpl<S>* B, int q, void* c, void* lambda, void* proj, void* d, void* X) {
    MATO_TRY(check_q(B, q));
    const auto& P = B->probs[q];
    MATO_HIP(hipStreamSynchronize(B->stream));
    (void)c;
    const size_t npt = (size_t)P.np * P.T;
    std::vector<int> canon(P.np);                   // internal row -> canonical row
    for (int r = 0; r < P.np; ++r) canon[r] = canonical_row(P.plan->pairs[r], P.n, P.n_obs);
    auto pairwise_out = [&](const S* dsrc, void* dst) -> mato_status {
        std::vector<S> h(npt * 3), o(npt * 3);
        MATO_HIP(hipMemcpy(h.data(), dsrc, sizeof(S) * h.size(), hipMemcpyDeviceToHost));
        for (int t = 0; t < P.T; ++t)
            for (int a = 0; a < 3; ++a)
                for (int r = 0; r < P.np; ++r)
                    o[((size_t)canon[r] * P.T + t) * 3 + a] = h[((size_t)t * 3 + a) * P.np + r];
        return copy_out(dst, o.data(), sizeof(S) * o.size());
    };
    if (lambda) MATO_TRY(pairwise_out((const S*)(P.base + P.o_lam), lambda));
    const ProblemDesc<S>& D = B->hdesc[q];
    if ((proj || d) && !D.dbg_proj) { set_error("enable mato_batch_debug before reading proj or d"); return MATO_ERR_INVALID_ARG; }
    if (proj) MATO_TRY(pairwise_out(D.dbg_proj, proj));
    if (d) {
        std::vector<S> h(npt), o(npt);
        MATO_HIP(hipMemcpy(h.data(), D.dbg_d, sizeof(S) * npt, hipMemcpyDeviceToHost));
        for (int t = 0; t < P.T; ++t)
            for (int r = 0; r < P.np; ++r) o[(size_t)canon[r] * P.T + t] = h[(size_t)t * P.np + r];
        MATO_TRY(copy_out(d, o.data(), sizeof(S) * npt));
    }
    if (X) {
        // FP32 iterations keep the positions in LDS only: form X = P c of the current
        // coefficients here (the same FP64 products, rounded once)
        MATO_HIP(launch_positions<S>(B->ddesc + q, 1, kModeInit, P.nv == 11 ? 11 : 0, B->stream));
        MATO_HIP(hipStreamSynchronize(B->stream));
        const size_t nx = (size_t)P.n * 3 * P.T;
        std::vector<S> h(nx), o(nx);
        MATO_HIP(hipMemcpy(h.data(), D.X, sizeof(S) * nx, hipMemcpyDeviceToHost));
        for (int t = 0; t < P.T; ++t)
            for (int a = 0; a < 3; ++a)
                for (int i = 0; i < P.n; ++i) o[((size_t)i * 3 + a) * P.T + t] = h[((size_t)t * 3 + a) * P.n + i];
        MATO_TRY(copy_out(X, o.data(), sizeof(S) * nx));
    }
    return MATO_OK;
}

extern "C" mato_status mato_batch_get_state(mato_batch b, int32_t q, void* c, void* lambda, void* proj,
                                            void* d, void* X) {
    if (c) MATO_TRY(mato_batch_coeffs(b, q, (double*)c));
    return dispatch(b, [&](auto* B) { return get_state_impl(B, q, nullptr, lambda, proj, d, X); });
}

template <typename S>
static mato_status set_state_impl(BatchImpl<S>* B, int q, const double* c, const void* lambda, const void* proj) {
    MATO_TRY(check_q(B, q));
    if (!lambda || !proj) { set_error("lambda and proj are required"); return MATO_ERR_INVALID_ARG; }
    const auto& P = B->probs[q];
    const size_t npt = (size_t)P.np * P.T;
    MATO_HIP(hipStreamSynchronize(B->stream));
    std::vector<S> in(npt * 3), lam_i(npt * 3), proj_i(npt * 3);
    std::vector<int> canon(P.np);                   // internal row -> canonical row
    for (int r = 0; r < P.np; ++r) canon[r] = canonical_row(P.plan->pairs[r], P.n, P.n_obs);
    auto to_internal = [&](const void* src, std::vector<S>& dst) -> mato_status {
        MATO_HIP(hipMemcpy(in.data(), src, sizeof(S) * in.size(), hipMemcpyDefault));
        for (size_t e = 0; e < in.size(); ++e)
            if (!std::isfinite((double)in[e])) { set_error("non-finite state"); return MATO_ERR_NONFINITE; }
        for (int r = 0; r < P.np; ++r)
            for (int t = 0; t < P.T; ++t)
                for (int a = 0; a < 3; ++a)
                    dst[((size_t)t * 3 + a) * P.np + r] = in[((size_t)canon[r] * P.T + t) * 3 + a];
        return MATO_OK;
    };
    MATO_TRY(to_internal(lambda, lam_i));
    MATO_TRY(to_internal(proj, proj_i));
    MATO_HIP(hipMemcpy(P.base + P.o_lam, lam_i.data(), sizeof(S) * lam_i.size(), hipMemcpyHostToDevice));
    if (c) {
        std::vector<double> hc((size_t)P.n * 3 * P.nv), o((size_t)3 * P.ldc, 0.0);
        MATO_HIP(hipMemcpy(hc.data(), c, sizeof(double) * hc.size(), hipMemcpyDefault));
        for (int i = 0; i < P.n; ++i)
            for (int a = 0; a < 3; ++a)
                for (int k = 0; k < P.nv; ++k) o[(size_t)a * P.ldc + (size_t)i * P.nv + k] = hc[((size_t)i * 3 + a) * P.nv + k];
        MATO_HIP(hipMemcpy(P.base + P.o_c, o.data(), sizeof(double) * o.size(), hipMemcpyHostToDevice));
    }
    DevBuf<S> dprojb;
    DevBuf<WorkItem> ditemsb;
    DevBuf<ProblemDesc<S>> ddb;
    MATO_TRY(dprojb.alloc(proj_i.size()));
    S* dproj = dprojb.p;
    MATO_HIP(hipMemcpy(dproj, proj_i.data(), sizeof(S) * proj_i.size(), hipMemcpyHostToDevice));
    std::vector<WorkItem> items;
    for (const auto& w : B->hitems)
        if (w.prob == q) { WorkItem v = w; v.prob = 0; items.push_back(v); }
    ProblemDesc<S> D = B->hdesc[q];
    D.proj_in = dproj;
    MATO_TRY(ditemsb.alloc(items.size()));
    MATO_TRY(ddb.alloc(1));
    WorkItem* ditems = ditemsb.p;
    ProblemDesc<S>* dd = ddb.p;
    MATO_HIP(hipMemcpy(ditems, items.data(), sizeof(WorkItem) * items.size(), hipMemcpyHostToDevice));
    MATO_HIP(hipMemcpy(dd, &D, sizeof(D), hipMemcpyHostToDevice));
    int ctrl[kCtrl];
    MATO_HIP(hipMemcpy(ctrl, B->dctrl + kCtrl * q, sizeof(ctrl), hipMemcpyDeviceToHost));
    ctrl[1] = 0;
    ctrl[2] = 0;
    ctrl[3] = 1;
    ctrl[4] = 0;
    MATO_HIP(hipMemcpy(B->dctrl + kCtrl * q, ctrl, sizeof(ctrl), hipMemcpyHostToDevice));
    // positions of the new coefficients first: the pairwise pass measures b_fc against them
    if (c) MATO_HIP(launch_positions<S>(dd, 1, kModeInit, B->common_nv(), B->stream));
    MATO_HIP(launch_pairwise<S>(ditems, (int)items.size(), dd, kModeSetState, B->threads, B->lds, B->common_nv(), true,
                                B->stream));
    MATO_HIP(launch_qbuild<S>(dd, 1, kModeInit, B->common_nv(), P.n, B->stream));
    MATO_HIP(hipStreamSynchronize(B->stream));
    return MATO_OK;
}

extern "C" mato_status mato_batch_set_state(mato_batch b, int32_t q, const void* c, const void* lambda,
                                            const void* proj) {
    return dispatch(b, [&](auto* B) { return set_state_impl(B, q, (const double*)c, lambda, proj); });
}

extern "C" mato_status mato_batch_linear_term(mato_batch b, int32_t q, void* g) {
    return dispatch(b, [&](auto* B) -> mato_status {
        MATO_TRY(check_q(B, q));
        if (!g) { set_error("null output"); return MATO_ERR_INVALID_ARG; }
        const auto& P = B->probs[q];
        std::vector<double> h((size_t)3 * P.ldq), o((size_t)P.n * 3 * P.nv);
        MATO_HIP(hipStreamSynchronize(B->stream));
        MATO_HIP(hipMemcpy(h.data(), P.base + P.o_q, sizeof(double) * h.size(), hipMemcpyDeviceToHost));
        for (int i = 0; i < P.n; ++i)
            for (int a = 0; a < 3; ++a)
                for (int k = 0; k < P.nv; ++k)
                    o[((size_t)i * 3 + a) * P.nv + k] = h[(size_t)a * P.ldq + (size_t)i * P.nv + k];
        return copy_out(g, o.data(), sizeof(double) * o.size());
    });
}

extern "C" mato_status mato_batch_set_rho_schedule(mato_batch b, int32_t stages, const mato_plan* plans,
                                                   const int32_t* start_iter) {
    if (stages < 1 || stages > kMaxStages || !plans || !start_iter || start_iter[0] != 0) {
        set_error("a schedule needs 1..%d stages, plans and start_iter[0] = 0", kMaxStages);
        return MATO_ERR_INVALID_ARG;
    }
    for (int j = 1; j < stages; ++j)
        if (start_iter[j] <= start_iter[j - 1]) { set_error("start_iter must increase"); return MATO_ERR_INVALID_ARG; }
    return dispatch(b, [&](auto* B) -> mato_status {
        const int cnt = B->count();
        for (int q = 0; q < cnt; ++q) {
            const auto& P = B->probs[q];
            if (P.iters_host != 0) { set_error("set the schedule before the first iteration"); return MATO_ERR_INVALID_ARG; }
            if (plans[q] != P.plan) { set_error("stage 0 of problem %d must be its creation plan", q); return MATO_ERR_INVALID_ARG; }
            for (int j = 0; j < stages; ++j) {
                const mato_plan p = plans[(size_t)j * cnt + q];
                if (!p || p->n != P.plan->n || p->T != P.plan->T || p->nv != P.plan->nv ||
                    p->t_final != P.plan->t_final || p->precision != P.plan->precision || p->a != P.plan->a ||
                    p->b != P.plan->b || p->solve != P.plan->solve || p->n_obs != P.plan->n_obs) {
                    set_error("stage %d plan of problem %d does not match its sizes, basis, precision or solve kind",
                              j, q);
                    return MATO_ERR_INVALID_ARG;
                }
            }
        }
        MATO_HIP(hipStreamSynchronize(B->stream));
        for (int q = 0; q < cnt; ++q) {
            auto& P = B->probs[q];
            P.stages.clear();
            P.stage_start.clear();
            for (int j = 0; j < stages; ++j) {
                P.stages.push_back(plans[(size_t)j * cnt + q]);
                P.stage_start.push_back(start_iter[j]);
            }
            P.stage = 0;
        }
        return B->upload_desc();
    });
}

extern "C" mato_status mato_batch_set_projection(mato_batch b, int32_t mode) {
    if (mode != 0 && mode != 1) { set_error("projection mode must be 0 or 1"); return MATO_ERR_INVALID_ARG; }
    return dispatch(b, [&](auto* B) -> mato_status {
        MATO_HIP(hipStreamSynchronize(B->stream));
        for (auto& P : B->probs) P.shifted = mode;
        return B->upload_desc();
    });
}

extern "C" mato_status mato_batch_set_tiles(mato_batch b, int32_t items_per_wg, int32_t threads) {
    return dispatch(b, [&](auto* B) { return B->set_tiles(items_per_wg, threads); });
}

extern "C" mato_status mato_batch_get_tiles(mato_batch b, int32_t* items_per_wg, int32_t* threads) {
    return dispatch(b, [&](auto* B) -> mato_status {
        if (items_per_wg) *items_per_wg = B->items_per_wg;
        if (threads) *threads = B->threads;
        return MATO_OK;
    });
}

extern "C" mato_status mato_batch_autotune(mato_batch b, int32_t* items_per_wg, int32_t* threads) {
    return dispatch(b, [&](auto* B) { return B->autotune(items_per_wg, threads); });
}

extern "C" mato_status mato_batch_timing(mato_batch b, int32_t enable) {
    return dispatch(b, [&](auto* B) -> mato_status {
        B->timing = enable != 0;
        return MATO_OK;
    });
}

extern "C" mato_status mato_batch_last_times(mato_batch b, double* total_ms, double* pairwise_ms,
                                             int32_t* pairwise_launches) {
    return dispatch(b, [&](auto* B) -> mato_status {
        if (!B->last_timed) { set_error("timing was not enabled for the last step"); return MATO_ERR_INVALID_ARG; }
        MATO_HIP(hipEventSynchronize(B->ev1));
        float ms = 0.f;
        MATO_HIP(hipEventElapsedTime(&ms, B->ev0, B->ev1));
        if (total_ms) *total_ms = ms;
        double pw = 0.0;
        for (int k = 0; k + 1 < B->pw_used; k += 2) {
            float m = 0.f;
            MATO_HIP(hipEventElapsedTime(&m, B->pw_events[k], B->pw_events[k + 1]));
            pw += m;
        }
        if (pairwise_ms) *pairwise_ms = pw;
        if (pairwise_launches) *pairwise_launches = B->pw_used / 2;
        return MATO_OK;
    });
}

extern "C" mato_status mato_solve_run(mato_plan plan, const double* starts, const double* goals, int32_t iters,
                                      double tol, int32_t check_every, mato_solve* out) {
    if (!plan) { set_error("null plan"); return MATO_ERR_INVALID_ARG; }
    MATO_TRY(mato_batch_create(1, &plan, starts, goals, plan->stream, out));
    return mato_batch_run(*out, iters, tol, check_every);
}

extern "C" mato_status mato_solve_coeffs(mato_solve s, double* c) { return mato_batch_coeffs(s, 0, c); }

extern "C" mato_status mato_residuals(mato_solve s, double* r_max, double* r_rms, double* cost, int32_t cap,
                                      int32_t* n_written) {
    return mato_batch_residuals(s, 0, r_max, r_rms, cost, cap, n_written);
}

extern "C" mato_status mato_solve_sync(mato_solve s) { return mato_batch_sync(s); }

extern "C" mato_status mato_step(mato_solve s, int32_t k_steps) { return mato_batch_step(s, k_steps, 0.0, 1); }

extern "C" mato_status mato_get_state(mato_solve s, void* c, void* lambda, void* proj, void* d, void* X) {
    return mato_batch_get_state(s, 0, c, lambda, proj, d, X);
}

extern "C" mato_status mato_set_state(mato_solve s, const void* c, const void* lambda, const void* proj) {
    return mato_batch_set_state(s, 0, c, lambda, proj);
}

extern "C" void mato_solve_destroy(mato_solve s) { mato_batch_destroy(s); }

extern "C" mato_status mato_stream_create(void** out) {
    if (!out) { set_error("null argument"); return MATO_ERR_INVALID_ARG; }
    *out = nullptr;
    hipStream_t st = nullptr;
    MATO_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));   // default priority
    *out = st;
    return MATO_OK;
}

extern "C" mato_status mato_stream_destroy(void* stream) {
    if (!stream) { set_error("null stream"); return MATO_ERR_INVALID_ARG; }
    MATO_HIP(hipStreamDestroy((hipStream_t)stream));
    return MATO_OK;
}

// ------------------------------------------------- solve without allocation ---
// A fixed device array for callers that cannot allocate: every device buffer of
// mato_solve_noalloc (problem state, descriptors, work lists, control words) is carved
// from it.  Each device holds its own copy for the life of the process; host code uses
// only the address hipGetSymbolAddress returns for the current device, never the name.
namespace mato {
constexpr size_t kScratchBytes = (size_t)MATO_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu[kMaxDevices];     // one call at a time per device
static char* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of the array (looked up once per device, with
// that device current, under its lock).
static mato_status scratch_base(int dev, char** out) {
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            set_error("hipGetSymbolAddress of the scratch array failed: %s", hipGetErrorString(e));
            return MATO_ERR_HIP;
        }
        g_scratch_ptr[dev] = (char*)ptr;
    }
    *out = g_scratch_ptr[dev];
    return MATO_OK;
}
}  // namespace mato

extern "C" mato_status mato_solve_noalloc(mato_plan plan, const double* starts, const double* goals,
                                          int32_t iters, double tol, int32_t check_every, double* c,
                                          double* r_max, double* r_rms, double* cost, int32_t cap,
                                          int32_t* n_written, int32_t* iters_done, int32_t* converged) {
    if (!plan || !starts || !goals || !c) { set_error("null argument"); return MATO_ERR_INVALID_ARG; }
    if (iters < 0 || check_every < 1) { set_error("iters must be >= 0 and check_every >= 1"); return MATO_ERR_INVALID_ARG; }
    int dev = 0;
    MATO_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) { set_error("device %d beyond %d", dev, kMaxDevices); return MATO_ERR_UNSUPPORTED; }
    std::lock_guard<std::mutex> lock(g_scratch_mu[dev]);
    char* base = nullptr;
    MATO_TRY(scratch_base(dev, &base));
    mato_batch_s b;
    b.precision = plan->precision;
    mato_status s;
    if (b.precision == MATO_FP64) {
        BatchImpl<double>* B = nullptr;
        s = batch_create<double>(1, &plan, starts, goals, nullptr, plan->stream, &B, base, kScratchBytes);
        b.impl = B;
    } else {
        BatchImpl<float>* B = nullptr;
        s = batch_create<float>(1, &plan, starts, goals, nullptr, plan->stream, &B, base, kScratchBytes);
        b.impl = B;
    }
    if (s == MATO_OK) {
        const mato_status r = mato_batch_run(&b, iters, tol, check_every);
        s = (r < 0) ? r : MATO_OK;
        if (s == MATO_OK) s = mato_batch_coeffs(&b, 0, c);
        if (s == MATO_OK) s = mato_batch_residuals(&b, 0, r_max, r_rms, cost, cap, n_written);
        if (s == MATO_OK) s = mato_batch_status(&b, 0, iters_done, converged);
        if (s == MATO_OK) s = r;                       // keep the NOT_CONVERGED warning
    }
    if (b.impl) {
        if (b.precision == MATO_FP64)
            delete static_cast<BatchImpl<double>*>(b.impl);
        else
            delete static_cast<BatchImpl<float>*>(b.impl);
    }
    return s;
}
