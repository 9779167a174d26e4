// Continuous-batching request loop: planning problems of different agent counts
// arrive, wait in a FIFO queue, are admitted as slots and device memory free up,
// iterate together with every other resident problem (one launch per stage per
// iteration, uneven sizes in the same launches), and leave as soon as they reach
// the residual tolerance or the iteration cap.  K^{-1} is cached per agent count
// (Remarks 1-2: the inverse depends on n, the basis and rho only).
//
// Each scheduling step: (1) read every slot's control words and retire the
// finished problems (coefficients copied to the host, slot freed), (2) admit
// queued problems in arrival order while a slot is free and the device-memory
// budget allows its plan and its state, initialising them on their own, (3) run
// `chunk` iterations of all resident problems.
#include <chrono>
#include <deque>
#include <string>
#include <thread>

#include "engine.h"

using Clock = std::chrono::steady_clock;

struct mato_server_s {
    mato_server_config cfg;
    hipStream_t stream = nullptr;
    void* eng = nullptr;                       // mato::Engine<float> or <double>
    std::map<int64_t, mato_plan> plans;        // per (agent count, obstacle count, rho stage): plan_key()
    struct Req {
        int64_t id = 0;
        int n = 0, n_obs = 0;
        std::vector<double> starts, goals, c;
        std::vector<double> obstacles;         // [n_obs][5]
        int state = 0;                         // 0 queued, 1 running, 2 done, 3 rejected
        mato_status fail = MATO_OK;            // why a rejected request could not run
        std::string why;
        int slot = -1;
        int iters = 0, converged = 0, nonfinite = 0;
        double r_max = 0.0;
        double t_submit = 0.0, t_start = 0.0, t_done = 0.0;
    };
    std::map<int64_t, Req> reqs;
    std::deque<int64_t> queue;
    std::vector<int64_t> slot_req;
    int64_t next_id = 1;
    Clock::time_point t0;
    std::vector<int64_t> finished;             // ids retired by the last step

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

namespace mato {

static int64_t plan_key(int n, int n_obs, int stage) {
    return ((int64_t)n * (MATO_MAX_OBSTACLES + 1) + n_obs) * kMaxStages + stage;
}

static size_t plan_bytes_estimate(int n, int nv, int T, int precision, int solve) {
    if (solve == MATO_SOLVE_STRUCTURED)
        return (size_t)T * nv * 16 + (size_t)nv * (4 * nv + 4 * kNb) * 8 + (size_t)n * n * 2 + 4096;
    const size_t N = (size_t)n * (nv + kNb), M = (size_t)n * nv;
    const size_t Mp = (size_t)round_up((int)M, 64), ldk = (size_t)round_up((int)M, 32);
    const size_t op = precision == MATO_FP64 ? 8 : (precision == MATO_BF16_REFINED ? 4 : 4);
    return N * N * 8 + Mp * ldk * op + (size_t)T * nv * 16 + (size_t)n * n * 2 + 4096;
}

template <typename S>
struct ServerOps {
    static Engine<S>* E(mato_server s) { return static_cast<Engine<S>*>(s->eng); }

    static size_t device_bytes(mato_server s) {
        size_t b = 0;
        for (auto& kv : s->plans) b += kv.second->bytes;
        for (auto& P : E(s)->probs)
            if (P.own) b += P.block;
        return b;
    }

    static bool plan_in_use(mato_server s, mato_plan p) {
        for (auto& P : E(s)->probs) {
            if (!P.active) continue;
            if (P.plan == p) return true;
            for (auto q : P.stages)
                if (q == p) return true;
        }
        return false;
    }

    // Frees idle device memory (blocks of free slots, then unused plans) until `need`
    // more bytes fit the budget; the plans in `keep` must stay.
    static bool make_room(mato_server s, size_t need, const std::vector<mato_plan>& keep, int keep_slot) {
        const double budget = s->cfg.hbm_budget_bytes;
        if (budget <= 0) return true;
        auto fits = [&]() { return (double)(device_bytes(s) + need) <= budget; };
        if (fits()) return true;
        Engine<S>* e = E(s);
        for (int q = 0; q < e->count() && !fits(); ++q)
            if (q != keep_slot && !e->probs[q].active && e->probs[q].own) e->release_block(q);
        for (auto it = s->plans.begin(); it != s->plans.end() && !fits();) {
            if (!plan_keep(s, it->second, keep) && !plan_in_use(s, it->second)) {
                for (int q = 0; q < e->count(); ++q)
                    if (!e->probs[q].active && e->probs[q].plan == it->second) e->release_block(q);
                mato_plan_destroy(it->second);
                it = s->plans.erase(it);
            } else {
                ++it;
            }
        }
        return fits();
    }

    static int stages(mato_server s) { return s->cfg.rho_stages > 0 ? s->cfg.rho_stages : 1; }
    static double stage_rho(mato_server s, int j) { return s->cfg.rho_stages > 0 ? s->cfg.rho_values[j] : s->cfg.rho; }

    static bool plan_keep(mato_server s, mato_plan p, const std::vector<mato_plan>& keep) {
        for (auto k : keep)
            if (k == p) return true;
        return false;
    }

    // All stage plans of agent count n with n_obs obstacles (created on demand, together,
    // within the budget).
    static mato_status get_plans(mato_server s, int n, int n_obs, std::vector<mato_plan>* out) {
        out->clear();
        std::vector<int> missing;
        std::vector<double> rhos;
        for (int j = 0; j < stages(s); ++j)
            if (!s->plans.count(plan_key(n, n_obs, j))) {
                missing.push_back(j);
                rhos.push_back(stage_rho(s, j));
            }
        if (!missing.empty()) {
            std::vector<mato_plan> keep;
            for (int j = 0; j < stages(s); ++j) {
                auto it = s->plans.find(plan_key(n, n_obs, j));
                if (it != s->plans.end()) keep.push_back(it->second);
            }
            const size_t est = missing.size() * plan_bytes_estimate(n, s->cfg.basis.n_coef, s->cfg.T, s->cfg.precision,
                                                                       s->cfg.solve);
            if (!make_room(s, est, keep, -1)) return MATO_OK;     // not now: wait for memory
            std::vector<mato_plan> made(missing.size(), nullptr);
            mato_plan_desc d;
            d.n = n; d.n_obs = n_obs; d.T = s->cfg.T; d.basis = s->cfg.basis; d.a = s->cfg.a; d.b = s->cfg.b;
            d.precision = s->cfg.precision; d.solve = s->cfg.solve;
            MATO_TRY(mato_plan_create_ex(&d, rhos.data(), (int)rhos.size(), s->stream, made.data()));
            for (size_t m = 0; m < missing.size(); ++m) s->plans[plan_key(n, n_obs, missing[m])] = made[m];
        }
        for (int j = 0; j < stages(s); ++j) out->push_back(s->plans[plan_key(n, n_obs, j)]);
        return MATO_OK;
    }

    static mato_status retire(mato_server s) {
        Engine<S>* e = E(s);
        s->finished.clear();
        bool any = false;
        for (int64_t r : s->slot_req) any = any || r >= 0;
        if (!any) return MATO_OK;
        std::vector<int> ctrl;
        MATO_TRY(e->read_ctrl(ctrl));
        bool changed = false;
        for (int q = 0; q < e->count(); ++q) {
            if (s->slot_req[q] < 0) continue;
            const int* w = &ctrl[(size_t)kCtrl * q];
            if (!w[1]) continue;
            auto& R = s->reqs[s->slot_req[q]];
            auto& P = e->probs[q];
            R.iters = w[0];
            R.converged = w[4];
            R.nonfinite = w[2];
            std::vector<double> h((size_t)3 * P.ldc);
            MATO_HIP(hipMemcpy(h.data(), P.base + P.o_c, sizeof(double) * h.size(), hipMemcpyDeviceToHost));
            R.c.assign((size_t)P.n * 3 * P.nv, 0.0);
            for (int i = 0; i < P.n; ++i)
                for (int a = 0; a < 3; ++a)
                    for (int k = 0; k < P.nv; ++k)
                        R.c[((size_t)i * 3 + a) * P.nv + k] = h[(size_t)a * P.ldc + (size_t)i * P.nv + k];
            if (R.iters > 0) {
                double hr[3];
                const int k = std::min(R.iters, kHistCap) - 1;
                MATO_HIP(hipMemcpy(hr, P.base + P.o_hist + sizeof(double) * 3 * k, sizeof(hr), hipMemcpyDeviceToHost));
                R.r_max = hr[0];
            }
            R.state = 2;
            R.t_done = s->now();
            R.slot = -1;
            s->finished.push_back(R.id);
            s->slot_req[q] = -1;
            MATO_TRY(e->detach(q));
            changed = true;
        }
        (void)changed;
        return MATO_OK;
    }

    // The request at the head of the queue cannot run at all: it leaves the queue as
    // finished-with-failure so that the requests behind it are not held up.
    static void reject(mato_server s, mato_status st, const char* why) {
        auto& R = s->reqs[s->queue.front()];
        R.state = 3;
        R.fail = st;
        R.why = why;
        R.t_done = s->now();
        s->finished.push_back(R.id);
        s->queue.pop_front();
    }

    static mato_status admit(mato_server s) {
        Engine<S>* e = E(s);
        std::vector<int> admitted;
        while (!s->queue.empty()) {
            auto& R = s->reqs[s->queue.front()];
            std::vector<mato_plan> sp;
            const mato_status pst = get_plans(s, R.n, R.n_obs, &sp);
            if (pst != MATO_OK) { reject(s, pst, last_error()); continue; }
            if (sp.empty()) {
                // with nothing resident every evictable byte was already freed: it never fits
                if (e->active_count() == 0) {
                    reject(s, MATO_ERR_OUT_OF_MEMORY, "the device-memory budget cannot hold the plans of this request");
                    continue;
                }
                break;
            }
            const mato_plan plan = sp[0];
            const size_t need = Engine<S>::slot_bytes(plan);
            int q = -1;
            for (int k = 0; k < e->count(); ++k)                // the free slot with the smallest block that fits
                if (s->slot_req[k] < 0 && !e->probs[k].active && e->probs[k].own && e->probs[k].block >= need &&
                    (q < 0 || e->probs[k].block < e->probs[q].block))
                    q = k;
            for (int k = 0; k < e->count() && q < 0; ++k)      // any free slot
                if (s->slot_req[k] < 0 && !e->probs[k].active) q = k;
            if (q < 0) break;
            const bool reuse = e->probs[q].own && e->probs[q].block >= need;
            if (!reuse) {
                e->release_block(q);
                if (!make_room(s, Engine<S>::block_class(need), sp, q)) {
                    if (e->active_count() == 0) {
                        reject(s, MATO_ERR_OUT_OF_MEMORY,
                               "the device-memory budget cannot hold this request's plans and state together");
                        continue;
                    }
                    break;
                }
            }
            e->probs[q].iter_cap = s->cfg.max_iters;
            e->probs[q].shifted = s->cfg.projection;
            const mato_status ast = e->attach(q, plan, R.starts.data(), R.goals.data(), nullptr,
                                              R.n_obs > 0 ? R.obstacles.data() : nullptr);
            if (ast == MATO_ERR_HIP) return ast;                // the device itself failed
            if (ast != MATO_OK) {
                // this request cannot run here (e.g. its pairwise stage does not fit the
                // device): it leaves the queue, and the requests behind it are served
                e->probs[q].active = false;
                e->lists_dirty = true;
                reject(s, ast, last_error());
                continue;
            }
            e->probs[q].stages.clear();
            e->probs[q].stage_start.clear();
            if (s->cfg.rho_stages > 0)
                for (int j = 0; j < stages(s); ++j) {
                    e->probs[q].stages.push_back(sp[j]);
                    e->probs[q].stage_start.push_back(s->cfg.rho_start[j]);
                }
            s->slot_req[q] = R.id;
            R.state = 1;
            R.slot = q;
            R.t_start = s->now();
            s->queue.pop_front();
            admitted.push_back(q);
        }
        if (admitted.empty()) return MATO_OK;
        MATO_TRY(e->rebuild_lists());
        for (int q : admitted) MATO_TRY(e->enqueue_init_one(q));
        return MATO_OK;
    }

    static mato_status step(mato_server s, int* running, int* queued) {
        MATO_TRY(retire(s));
        MATO_TRY(admit(s));
        Engine<S>* e = E(s);
        int act = e->active_count();
        if (act > 0) MATO_TRY(e->step(s->cfg.chunk, s->cfg.tol, s->cfg.use_graphs != 0));
        if (running) *running = act;
        if (queued) *queued = (int)s->queue.size();
        return MATO_OK;
    }

    static mato_status create(mato_server s) {
        auto* e = new Engine<S>();
        s->eng = e;
        e->precision = s->cfg.precision;
        e->refine = (e->precision == MATO_FP32) ? 1 : (e->precision == MATO_BF16_REFINED ? 2 : 0);
        if (const char* v = getenv("MATO_REFINE")) {
            e->refine = std::max(0, std::min(kMaxRefine, atoi(v)));
            e->refine_fixed = true;
        }
        e->solve = s->cfg.solve;
        if (e->solve == MATO_SOLVE_STRUCTURED) e->refine = 0;
        e->refine_base = e->refine;
        e->stream = s->stream;
        e->tol = s->cfg.tol;
        MATO_TRY(e->init_capacity(s->cfg.max_slots));
        MATO_TRY(e->upload_desc());            // every slot starts inactive with valid control words
        s->slot_req.assign(s->cfg.max_slots, -1);
        return MATO_OK;
    }

    // UNSUPPORTED if the pairwise stage of an (n, n_obs) problem does not fit the device
    static mato_status check_size(int n, int n_obs) {
        typename Engine<S>::Prob P;
        P.n = n;
        P.n_obs = n_obs;
        P.np = n * (n - 1) / 2 + n * n_obs;
        return Engine<S>::check_lds(P);
    }

    static void destroy(mato_server s) { delete E(s); }
};

template <typename F>
static mato_status sdispatch(mato_server s, F&& f) {
    if (!s || !s->eng) { set_error("null server"); return MATO_ERR_INVALID_ARG; }
    if (s->cfg.precision == MATO_FP64) return f(ServerOps<double>());
    return f(ServerOps<float>());
}

}  // namespace mato

using namespace mato;

extern "C" mato_status mato_server_create(const mato_server_config* cfg, void* hip_stream, mato_server* out) {
    if (!cfg || !out) { set_error("null argument"); return MATO_ERR_INVALID_ARG; }
    *out = nullptr;
    if (cfg->max_slots < 1 || cfg->chunk < 1 || cfg->max_iters < 1 || cfg->T < cfg->basis.n_coef ||
        !(cfg->a > 0) || !(cfg->b > 0) || !(cfg->rho > 0) || !(cfg->basis.t_final > 0) ||
        (cfg->precision != MATO_FP64 && cfg->precision != MATO_FP32 && cfg->precision != MATO_BF16_REFINED) ||
        (cfg->projection != 0 && cfg->projection != 1) || cfg->rho_stages < 0 || cfg->rho_stages > kMaxStages ||
        (cfg->solve != MATO_SOLVE_DENSE && cfg->solve != MATO_SOLVE_STRUCTURED) ||
        (cfg->solve == MATO_SOLVE_STRUCTURED && cfg->precision == MATO_BF16_REFINED) ||
        (cfg->use_graphs != 0 && cfg->use_graphs != 1)) {
        set_error("invalid server configuration");
        return MATO_ERR_INVALID_ARG;
    }
    for (int j = 0; j < cfg->rho_stages; ++j)
        if (!(cfg->rho_values[j] > 0) || cfg->rho_start[j] % cfg->chunk != 0 || (j == 0 && cfg->rho_start[0] != 0) ||
            (j > 0 && cfg->rho_start[j] <= cfg->rho_start[j - 1])) {
            set_error("rho schedule: values > 0, starts 0 then increasing multiples of chunk");
            return MATO_ERR_INVALID_ARG;
        }
    auto* s = new mato_server_s();
    s->cfg = *cfg;
    s->stream = (hipStream_t)hip_stream;
    s->t0 = Clock::now();
    mato_status st = (cfg->precision == MATO_FP64) ? ServerOps<double>::create(s) : ServerOps<float>::create(s);
    if (st != MATO_OK) {
        if (s->eng) (cfg->precision == MATO_FP64) ? ServerOps<double>::destroy(s) : ServerOps<float>::destroy(s);
        delete s;
        return st;
    }
    *out = s;
    return MATO_OK;
}

extern "C" void mato_server_destroy(mato_server s) {
    if (!s) return;
    (void)hipStreamSynchronize(s->stream);
    if (s->eng) (s->cfg.precision == MATO_FP64) ? ServerOps<double>::destroy(s) : ServerOps<float>::destroy(s);
    for (auto& kv : s->plans) mato_plan_destroy(kv.second);
    delete s;
}

extern "C" mato_status mato_server_warm(mato_server s, int32_t n_min, int32_t n_max) {
    return sdispatch(s, [&](auto ops) -> mato_status {
        for (int n = std::max(2, (int)n_min); n <= n_max; ++n) {
            std::vector<mato_plan> p;
            MATO_TRY(ops.get_plans(s, n, 0, &p));
            if (p.empty()) { set_error("device-memory budget too small to hold the plans for n = %d", n); return MATO_ERR_OUT_OF_MEMORY; }
        }
        return MATO_OK;
    });
}

extern "C" mato_status mato_server_submit(mato_server s, int32_t n, const double* starts, const double* goals,
                                          int64_t* id) {
    return mato_server_submit_ex(s, n, starts, goals, 0, nullptr, id);
}

extern "C" mato_status mato_server_submit_ex(mato_server s, int32_t n, const double* starts, const double* goals,
                                             int32_t n_obs, const double* obstacles, int64_t* id) {
    if (!s || !starts || !goals || (n_obs > 0 && !obstacles)) { set_error("null argument"); return MATO_ERR_INVALID_ARG; }
    if (n < 2) { set_error("n = %d < 2", n); return MATO_ERR_INVALID_ARG; }
    if (n > MATO_MAX_AGENTS) { set_error("n = %d > %d", n, MATO_MAX_AGENTS); return MATO_ERR_UNSUPPORTED; }
    if (n_obs < 0 || n_obs > MATO_MAX_OBSTACLES) {
        set_error("n_obs = %d outside 0..%d", n_obs, MATO_MAX_OBSTACLES);
        return MATO_ERR_INVALID_ARG;
    }
    MATO_TRY(sdispatch(s, [&](auto ops) { return ops.check_size(n, n_obs); }));
    mato_server_s::Req R;
    R.n = n;
    R.n_obs = n_obs;
    R.starts.resize((size_t)n * 3);
    R.goals.resize((size_t)n * 3);
    R.obstacles.resize((size_t)n_obs * 5);
    if (hipMemcpy(R.starts.data(), starts, sizeof(double) * R.starts.size(), hipMemcpyDefault) != hipSuccess ||
        hipMemcpy(R.goals.data(), goals, sizeof(double) * R.goals.size(), hipMemcpyDefault) != hipSuccess ||
        (n_obs > 0 &&
         hipMemcpy(R.obstacles.data(), obstacles, sizeof(double) * R.obstacles.size(), hipMemcpyDefault) != hipSuccess)) {
        (void)hipGetLastError();
        set_error("cannot read starts/goals/obstacles");
        return MATO_ERR_INVALID_ARG;
    }
    for (size_t k = 0; k < R.starts.size(); ++k)
        if (!std::isfinite(R.starts[k]) || !std::isfinite(R.goals[k])) {
            set_error("non-finite start or goal");
            return MATO_ERR_NONFINITE;
        }
    for (int o = 0; o < n_obs; ++o) {
        const double* ob = &R.obstacles[(size_t)5 * o];
        for (int k = 0; k < 5; ++k)
            if (!std::isfinite(ob[k])) { set_error("non-finite obstacle"); return MATO_ERR_NONFINITE; }
        if (!(ob[3] > 0) || !(ob[4] > 0)) { set_error("obstacle semi-axes must be > 0"); return MATO_ERR_INVALID_ARG; }
    }
    R.id = s->next_id++;
    R.t_submit = s->now();
    s->queue.push_back(R.id);
    s->reqs[R.id] = std::move(R);
    if (id) *id = s->queue.back();
    return MATO_OK;
}

extern "C" mato_status mato_server_step(mato_server s, int32_t* running, int32_t* queued) {
    return sdispatch(s, [&](auto ops) { return ops.step(s, running, queued); });
}

extern "C" mato_status mato_server_poll(mato_server s, int64_t id, int32_t* state, int32_t* iters,
                                        int32_t* converged, double* r_max) {
    if (!s) { set_error("null server"); return MATO_ERR_INVALID_ARG; }
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) { set_error("unknown request %lld", (long long)id); return MATO_ERR_NOT_FOUND; }
    if (state) *state = it->second.state;
    if (iters) *iters = it->second.iters;
    if (converged) *converged = it->second.converged;
    if (r_max) *r_max = it->second.r_max;
    return MATO_OK;
}

extern "C" mato_status mato_server_result(mato_server s, int64_t id, double* c) {
    if (!s || !c) { set_error("null argument"); return MATO_ERR_INVALID_ARG; }
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) { set_error("unknown request %lld", (long long)id); return MATO_ERR_NOT_FOUND; }
    if (it->second.state == 3) {
        const mato_status st = it->second.fail;
        set_error("request %lld was rejected: %s", (long long)id, it->second.why.c_str());
        s->reqs.erase(it);
        return st;
    }
    if (it->second.state != 2) { set_error("request %lld is not finished", (long long)id); return MATO_ERR_INVALID_ARG; }
    if (hipMemcpy(c, it->second.c.data(), sizeof(double) * it->second.c.size(), hipMemcpyDefault) != hipSuccess) {
        (void)hipGetLastError();
        set_error("cannot write the result");
        return MATO_ERR_INVALID_ARG;
    }
    const int nonfinite = it->second.nonfinite;
    s->reqs.erase(it);
    if (nonfinite) { set_error("request %lld produced non-finite values", (long long)id); return MATO_ERR_NONFINITE; }
    return MATO_OK;
}

extern "C" mato_status mato_server_stats(mato_server s, double* device_bytes, int32_t* n_plans, int32_t* running,
                                         int32_t* queued) {
    return sdispatch(s, [&](auto ops) -> mato_status {
        if (device_bytes) *device_bytes = (double)ops.device_bytes(s);
        if (n_plans) *n_plans = (int32_t)s->plans.size();
        if (running) *running = ops.E(s)->active_count();
        if (queued) *queued = (int32_t)s->queue.size();
        return MATO_OK;
    });
}

extern "C" mato_status mato_server_run_trace(mato_server s, int32_t count, const double* arrival_s,
                                             const int32_t* n, const double* starts, const double* goals,
                                             double* latency_s, int32_t* iters, int32_t* converged,
                                             double* wall_s) {
    if (!s || count < 0 || (count > 0 && (!arrival_s || !n || !starts || !goals))) {
        set_error("invalid arguments");
        return MATO_ERR_INVALID_ARG;
    }
    for (int k = 1; k < count; ++k)
        if (arrival_s[k] < arrival_s[k - 1]) { set_error("arrival times must be non-decreasing"); return MATO_ERR_INVALID_ARG; }
    std::vector<size_t> off(count + 1, 0);
    for (int k = 0; k < count; ++k) off[k + 1] = off[k] + (size_t)n[k] * 3;
    std::map<int64_t, int> index;
    const double base = s->now();
    int next = 0, done = 0;
    while (done < count) {
        const double t = s->now() - base;
        while (next < count && arrival_s[next] <= t) {
            int64_t id = 0;
            MATO_TRY(mato_server_submit(s, n[next], starts + off[next], goals + off[next], &id));
            s->reqs[id].t_submit = base + arrival_s[next];
            index[id] = next;
            ++next;
        }
        int running = 0, queued = 0;
        MATO_TRY(mato_server_step(s, &running, &queued));
        for (int64_t id : s->finished) {
            auto it = index.find(id);
            if (it == index.end()) continue;
            const auto& R = s->reqs[id];
            const int k = it->second;
            if (latency_s) latency_s[k] = R.t_done - R.t_submit;
            if (iters) iters[k] = R.iters;
            if (converged) converged[k] = R.converged;
            s->reqs.erase(id);
            index.erase(it);
            ++done;
        }
        if (running == 0 && queued == 0 && next < count) {
            const double wait = arrival_s[next] - (s->now() - base);
            if (wait > 0) std::this_thread::sleep_for(std::chrono::duration<double>(wait));
        }
    }
    if (wall_s) *wall_s = s->now() - base;
    return MATO_OK;
}
