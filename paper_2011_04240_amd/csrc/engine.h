// Host engine of libmato: a set of problem slots advanced together, one pass of
// the while-loop of Algorithm 1 per iteration:
//
//   [inverse product]   c = c_eq + K11^{-1} g                     (eq. (kkt_step_x))
//   [refinement x R]    r = g - H c (FP64);  c += K11^{-1} r
//   [positions]         X = P c                                   (eq. (param); FP32: inside the pairwise launch)
//   [pairwise]          delta; alpha, beta; d; lambda; b_fc; S    (eqs. (sphere_project)-(lag_update), (b_f))
//   [linear term]       g = rho P^T S = rho A_fc^T b_fc; residual record with the
//                       smoothness cost; convergence test
//
// Active slots with the same plan form one group whose right-hand sides are the
// columns of one matrix-matrix product; all pairwise work of all active slots is
// one launch over a work list of (slot, block of instants) items.  A fixed batch
// places every slot in one arena; the server attaches and detaches slots (each
// with its own device block) between iterations.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>

#include "common.h"

namespace mato {

template <typename S>
hipError_t launch_pairwise(const WorkItem*, int, const ProblemDesc<S>*, int, int, size_t, int, bool, hipStream_t);
template <typename S>
hipError_t set_pairwise_lds_limit(size_t);
template <typename S>
hipError_t launch_qbuild(const ProblemDesc<S>*, int, int, int, int, hipStream_t);
template <typename S>
hipError_t launch_residual(const ProblemDesc<S>*, int, hipStream_t);
template <typename S>
hipError_t launch_positions(const ProblemDesc<S>*, int, int, int, hipStream_t);
template <typename S>
hipError_t launch_solve_positions(const ProblemDesc<S>*, int, int, hipStream_t);
template <typename S>
hipError_t launch_init(const ProblemDesc<S>*, const double* const*, int, hipStream_t);
template <typename S>
hipError_t launch_ceq(const ProblemDesc<S>*, const double* const*, int, hipStream_t);
hipError_t launch_gemm(int, int, const GemmTile*, int, const GemmGroup*, const GemmCol*, int, hipStream_t);

inline int device_cu_count() {
    static int cached = -1;
    if (cached < 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
            cached = v;
        else
            cached = 256;
    }
    return cached;
}

inline int device_lds_limit() {
    static int cached = -1;
    if (cached < 0) {
        int dev = 0, v = 65536;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
            cached = v;
        else
            cached = 65536;
    }
    return cached;
}

// Grows a device buffer to hold at least `count` elements (contents are not kept).
template <typename T>
inline mato_status ensure_device(T** p, size_t* cap, size_t count) {
    if (*p && *cap >= count) return MATO_OK;
    dfree(*p);
    *p = nullptr;
    const size_t n = std::max<size_t>(count, 1);
    if (hipMalloc(p, sizeof(T) * n) != hipSuccess) {
        (void)hipGetLastError();
        set_error("device allocation of %zu bytes failed", sizeof(T) * n);
        return MATO_ERR_OUT_OF_MEMORY;
    }
    *cap = n;
    return MATO_OK;
}

template <typename S>
struct Engine {
    struct Prob {
        mato_plan plan = nullptr;
        int n = 0, np = 0, T = 0, nv = 0, ldq = 0, ldc = 0;
        int n_obs = 0;                       // static obstacles (np counts their rows)
        size_t o_obs = 0;
        size_t o_lam = 0, o_ssum = 0, o_X = 0, o_lflag = 0, o_c = 0, o_ceq = 0, o_q = 0, o_r = 0, o_qf = 0,
               o_rf = 0, o_part = 0, o_hist = 0, bytes = 0;
        char* base = nullptr;        // device block of this slot
        size_t block = 0;            // bytes of that block (own blocks only)
        bool own = false;            // the block is the slot's own allocation
        bool active = false;
        int nslab = 0;
        int iter_cap = 0;
        int shifted = 0;
        std::vector<mato_plan> stages;       // rho schedule (empty: the plan throughout)
        std::vector<int> stage_start;        // first iteration of each stage
        int stage = 0;
        int iters_host = 0;                  // iterations enqueued since attach
        std::vector<double> starts, goals;   // [n][3]
        std::vector<double> obstacles;       // [n_obs][5]: x, y, z, l_xy, l_z
    };

    int precision = MATO_FP32;
    int solve = MATO_SOLVE_DENSE;            // every plan of the engine has this solve kind
    int refine = 1;                          // FP64 corrections after the inverse product
    int refine_base = 1;                     // the precision's default
    bool refine_fixed = false;               // set by MATO_REFINE: no adaptation
    // The FP32 correction contracts by about u kappa per pass and kappa grows with rho (n + n_obs):
    // from this product on, FP32 batches take one more correction (the ten-rho schedule to 512 left
    // 32-agent swaps and one of six 128-agent boxes at the iteration cap with one correction)
    static constexpr double kRefineRhoN = 4096.0;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    std::vector<Prob> probs;                 // slots
    char* arena = nullptr;                   // fixed batches: one block for every slot
    size_t arena_bytes = 0;

    int* dctrl = nullptr;                    // [slots][kCtrl]
    std::vector<ProblemDesc<S>> hdesc;
    ProblemDesc<S>* ddesc = nullptr;
    double** dk0c = nullptr;
    double** dkinv = nullptr;
    std::vector<double*> hk0c, hkinv;        // host copies of the per-slot pointer tables

    std::vector<WorkItem> hitems;
    WorkItem* ditems = nullptr;
    size_t ditems_cap = 0;
    WorkItem* dscratch = nullptr;            // work items of one slot (initialisation, set-state)
    size_t dscratch_cap = 0;
    // pairwise launch shape until set or tuned: about 8 instants per work item at n = 64, so
    // that the FP32 kernel's per-item work (positions, boxes, broad phase) spreads over them
    int items_per_wg = 16384, threads = 256;
    bool tiles_set = false;                  // set_tiles / autotune chose the shape
    int n_active = 0;                        // active slots when the work list was built
    size_t lds = 0;

    std::vector<GemmGroup> hgroups;
    std::vector<GemmTile> htiles;
    int gemm_width = 64;                     // right-hand sides per product tile (64, or 48 in FP32 and BF16)
    GemmGroup* dgroups = nullptr;
    GemmTile* dtiles = nullptr;
    GemmCol* dcolsq = nullptr;
    GemmCol* dcolsr = nullptr;
    size_t cap_groups = 0, cap_tiles = 0, cap_colsq = 0, cap_colsr = 0;
    bool lists_dirty = true;
    bool has_obs = false;                    // some active slot has static obstacles

    double tol = 0.0;
    bool debug = false;
    S* dbg = nullptr;                        // debug outputs (d e and d) of every slot
    size_t dbg_bytes = 0;

    hipGraphExec_t g1 = nullptr, gC = nullptr;
    static constexpr int kChunk = 16;

    // pinned staging ring of the host-to-device uploads: a region is reused only after the
    // stream has been waited on, so the copies need neither a wait nor a live host source
    static constexpr size_t kRingBytes = (size_t)1 << 20;
    char* ring = nullptr;
    size_t ring_off = 0;

    bool timing = false;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    std::vector<hipEvent_t> pw_events;       // pairs around pairwise launches
    int pw_used = 0;
    bool last_timed = false;

    // Device memory carved from a caller-provided region instead of hipMalloc (entry points
    // that must not allocate): 256-byte steps, never freed by the engine; uploads then copy
    // straight from the caller's host memory and iterations are launched eagerly (no graphs).
    char* ext = nullptr;
    size_t ext_cap = 0, ext_used = 0;

    template <typename T>
    mato_status dev_buf(T** p, size_t* cap, size_t count) {
        if (!ext) return ensure_device(p, cap, count);
        if (*p && *cap >= count) return MATO_OK;
        const size_t n = std::max<size_t>(count, 1);
        const size_t bytes = (sizeof(T) * n + 255) & ~(size_t)255;
        if (ext_used + bytes > ext_cap) {
            set_error("the problem needs more than the %zu bytes of the fixed device scratch", ext_cap);
            return MATO_ERR_UNSUPPORTED;
        }
        *p = reinterpret_cast<T*>(ext + ext_used);
        ext_used += bytes;
        *cap = n;
        return MATO_OK;
    }

    ~Engine() {
        if (ext) {                        // carved from the caller's region: nothing to free
            arena = nullptr;
            dctrl = nullptr;
            ddesc = nullptr;
            dk0c = dkinv = nullptr;
            ditems = dscratch = nullptr;
            dgroups = nullptr;
            dtiles = nullptr;
            dcolsq = dcolsr = nullptr;
        }
        if (ring) (void)hipHostFree(ring);
        if (g1) (void)hipGraphExecDestroy(g1);
        if (gC) (void)hipGraphExecDestroy(gC);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        for (auto& P : probs)
            if (P.own) dfree(P.base);
        dfree(arena);
        dfree(dctrl);
        dfree(ddesc);
        dfree(dk0c);
        dfree(dkinv);
        dfree(ditems);
        dfree(dscratch);
        dfree(dgroups);
        dfree(dtiles);
        dfree(dcolsq);
        dfree(dcolsr);
        dfree(dbg);
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
        for (auto e : pw_events) (void)hipEventDestroy(e);
    }

    int count() const { return (int)probs.size(); }

    // Stream-ordered copy of `bytes` host bytes to `dst`; `src` may be reused on return.
    mato_status upload(void* dst, const void* src, size_t bytes) {
        if (bytes == 0) return MATO_OK;
        if (ext) {                                       // no staging ring: copy and wait
            MATO_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, stream));
            MATO_HIP(hipStreamSynchronize(stream));
            return MATO_OK;
        }
        if (!ring && hipHostMalloc((void**)&ring, kRingBytes, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            ring = nullptr;
        }
        if (!ring || bytes > kRingBytes / 2) {           // no ring, or too large for it: copy and wait
            MATO_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, stream));
            MATO_HIP(hipStreamSynchronize(stream));
            return MATO_OK;
        }
        if (ring_off + bytes > kRingBytes) {             // wrap: every earlier copy from the ring is done
            MATO_HIP(hipStreamSynchronize(stream));
            ring_off = 0;
        }
        memcpy(ring + ring_off, src, bytes);
        MATO_HIP(hipMemcpyAsync(dst, ring + ring_off, bytes, hipMemcpyHostToDevice, stream));
        ring_off = (ring_off + bytes + 255) & ~(size_t)255;
        return MATO_OK;
    }

    int active_count() const {
        int k = 0;
        for (const auto& P : probs) k += P.active;
        return k;
    }

    // number of basis coefficients shared by every active slot (0 if they differ)
    int common_nv() const {
        int nv = -1;
        for (const auto& P : probs) {
            if (!P.active) continue;
            if (nv < 0) nv = P.nv;
            if (P.nv != nv) return 0;
        }
        return nv < 0 ? 0 : nv;
    }

    // largest agent count among the slots (sizes the linear-term kernel's LDS)
    int max_agents() const {
        int m = 1;
        for (const auto& P : probs) m = std::max(m, P.n);
        return m;
    }

    // ------------------------------------------------------------ layout ---
    static void layout(Prob& P) {
        auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
        size_t off = 0;
        P.o_lam = off;  off += al(sizeof(S) * (size_t)P.T * 3 * P.np);
        P.o_ssum = off; off += al(sizeof(S) * (size_t)P.T * 3 * P.n);
        P.o_X = off;    off += al(sizeof(S) * (size_t)P.T * 3 * P.n);
        P.o_lflag = off; off += al(sizeof(unsigned) * (size_t)P.T * ((P.np + 63) / 64));
        P.o_c = off;    off += al(sizeof(double) * 3 * (size_t)P.ldc);
        P.o_ceq = off;  off += al(sizeof(double) * 3 * (size_t)P.ldc);
        P.o_q = off;    off += al(sizeof(double) * 3 * (size_t)P.ldq);
        P.o_r = off;    off += al(sizeof(double) * 3 * (size_t)P.ldq);
        P.o_qf = off;   off += al(sizeof(float) * 3 * (size_t)P.ldq);
        P.o_rf = off;   off += al(sizeof(float) * 3 * (size_t)P.ldq);
        P.o_part = off; off += al(sizeof(double) * 4 * (size_t)P.T);   // at most T slabs
        P.o_hist = off; off += al(sizeof(double) * 3 * kHistCap);
        P.o_obs = off;  off += al(sizeof(S) * kObs * (size_t)std::max(P.n_obs, 1));
        P.bytes = off;
    }

    static void describe(Prob& P, mato_plan plan) {
        P.plan = plan;
        P.n = plan->n;
        P.n_obs = plan->n_obs;
        P.np = P.n * (P.n - 1) / 2 + P.n * P.n_obs;
        P.T = plan->T;
        P.nv = plan->nv;
        P.ldq = round_up(P.n * (P.nv + kNb), 32);   // >= the operand stride ldk = round_up(11n, 32)
        P.ldc = P.n * P.nv;
        layout(P);
    }

    static size_t slot_bytes(mato_plan plan) {
        Prob P;
        describe(P, plan);
        return P.bytes;
    }

    // Size of a slot's own device block for `bytes` of problem state: the next power of two
    // (at least 64 KB), so that blocks freed by finished problems fit most later ones and
    // admissions rarely allocate.
    static size_t block_class(size_t bytes) {
        size_t c = (size_t)1 << 16;
        while (c < bytes) c <<= 1;
        return c;
    }

    // Control words, descriptors and per-slot pointer tables for `cap` slots.
    mato_status init_capacity(int cap) {
        probs.resize(cap);
        hdesc.assign(cap, ProblemDesc<S>());
        hk0c.assign(cap, nullptr);
        hkinv.assign(cap, nullptr);
        size_t c1 = 0, c2 = 0, c3 = 0, c4 = 0;
        MATO_TRY(dev_buf(&dctrl, &c1, (size_t)kCtrl * cap));
        MATO_TRY(dev_buf(&ddesc, &c2, (size_t)cap));
        MATO_TRY(dev_buf(&dk0c, &c3, (size_t)cap));
        MATO_TRY(dev_buf(&dkinv, &c4, (size_t)cap));
        MATO_HIP(hipMemsetAsync(dctrl, 0, sizeof(int) * kCtrl * cap, stream));
        MATO_HIP(hipMemsetAsync(dk0c, 0, sizeof(double*) * cap, stream));
        MATO_HIP(hipMemsetAsync(dkinv, 0, sizeof(double*) * cap, stream));
        MATO_HIP(hipStreamSynchronize(stream));
        if (!ext) {                                      // HIP events only for timing
            if (!ev0) MATO_HIP(hipEventCreate(&ev0));
            if (!ev1) MATO_HIP(hipEventCreate(&ev1));
        }
        return MATO_OK;
    }

    void fill_desc(int q) {
        const Prob& P = probs[q];
        ProblemDesc<S>& D = hdesc[q];
        memset(&D, 0, sizeof(D));
        D.ctrl = dctrl + kCtrl * q;
        if (!P.plan || !P.base) return;
        const mato_plan pl = P.plan;
        char* b = P.base;
        D.n = P.n; D.np = P.np; D.T = P.T; D.nv = P.nv; D.ldq = P.ldq; D.ldc = P.ldc;
        D.n_obs = P.n_obs;
        D.obs = (const S*)(b + P.o_obs);
        D.nslab = P.nslab; D.hist_cap = kHistCap;
        D.a = pl->a; D.b = pl->b; D.rho = pl->rho;
        D.ia2 = (S)(1.0 / (pl->a * pl->a));
        D.ib2 = (S)(1.0 / (pl->b * pl->b));
        D.lz = (S)pl->b;
        D.srho = (S)pl->rho;
        D.sirho = (S)(1.0 / pl->rho);
        D.P = pl->dP; D.Pdd = pl->dPdd; D.PtP = pl->dPtP; D.PddtPdd = pl->dPddtPdd; D.A = pl->dA;
        D.pairs = pl->dPairs;
        D.smat = pl->dS;
        D.lam = (S*)(b + P.o_lam);
        D.ssum = (S*)(b + P.o_ssum);
        D.X = (S*)(b + P.o_X);
        D.lflag = (unsigned*)(b + P.o_lflag);
        D.c = (double*)(b + P.o_c);
        D.ceq = (double*)(b + P.o_ceq);
        D.q = (double*)(b + P.o_q);
        D.r = (double*)(b + P.o_r);
        D.qf = (float*)(b + P.o_qf);
        D.rf = (float*)(b + P.o_rf);
        D.part = (double*)(b + P.o_part);
        D.hist = (double*)(b + P.o_hist);
        D.tol = tol;
        D.iter_cap = P.iter_cap;
        D.shifted = P.shifted;
        D.rho_next = pl->rho;
        D.sirho_next = (S)(1.0 / pl->rho);
        D.switch_at = 0;
        if (P.stage + 1 < (int)P.stages.size()) {
            D.switch_at = P.stage_start[P.stage + 1];
            D.rho_next = P.stages[P.stage + 1]->rho;
            D.sirho_next = (S)(1.0 / P.stages[P.stage + 1]->rho);
        }
        if (debug && dbg) {
            size_t off = 0;
            for (int k = 0; k < q; ++k) off += (size_t)probs[k].T * 4 * probs[k].np;
            D.dbg_proj = dbg + off;
            D.dbg_d = dbg + off + (size_t)P.T * 3 * P.np;
        }
    }

    mato_status upload_desc() {
        for (int q = 0; q < count(); ++q) fill_desc(q);
        MATO_TRY(upload(ddesc, hdesc.data(), sizeof(ProblemDesc<S>) * count()));
        return MATO_OK;
    }

    // work items of slot q: instants in blocks of tc
    void slot_items(int q, std::vector<WorkItem>& out, size_t* maxlds, int as_prob) {
        Prob& P = probs[q];
        const int cap = device_lds_limit() - 1024;   // room for the kernel's static reduction buffer
        const size_t per_t = pairwise_lds_per_instant(P);
        const size_t fixed = pairwise_lds_fixed(P, threads);
        int tc = std::max(1, items_per_wg / std::max(1, P.np));
        tc = std::min(tc, P.T);
        if (!tiles_set) {
            // a few problems: keep about four work items per compute unit rather than long ones
            const long want = 4L * device_cu_count();
            tc = std::min(tc, std::max(1, (int)((long)P.T * std::max(1, n_active) / want)));
        }
        while (tc > 1 && per_t * tc + fixed > (size_t)cap) --tc;
        *maxlds = std::max(*maxlds, per_t * tc + fixed);
        P.nslab = (P.T + tc - 1) / tc;
        for (int s = 0; s < P.nslab; ++s) {
            WorkItem w;
            w.prob = as_prob;
            w.t0 = s * tc;
            w.tc = std::min(tc, P.T - w.t0);
            w.slab = s;
            out.push_back(w);
        }
    }

    // LDS of the pairwise kernel per instant of a work item.  FP32: positions (x, y, z, 0),
    // 16 n bytes, the fixed-point corrections of the per-agent sums, 24 n bytes, an area
    // that first holds the basis row (8 n_v bytes), and the multiplier group flags before
    // and after the pass, 8 bytes per 64 rows.  FP64: the FP64 sum over agents of X,
    // positions X and b_fc (or its corrections) and two flag words per 32 pairs.
    static size_t pairwise_lds_per_instant(const Prob& P) {
        if (std::is_same<S, float>::value)
            return (size_t)16 * P.n + std::max((size_t)24 * P.n, (size_t)8 * P.nv) + (size_t)8 * ((P.np + 63) / 64);
        return (size_t)3 * sizeof(double) + (size_t)3 * (P.n + P.np) * sizeof(S) +
               (size_t)2 * ((P.np + 31) / 32) * sizeof(unsigned);
    }

    // LDS of the pairwise kernel per work item besides the instants: the obstacle table;
    // FP32 also the agents' bounding boxes (24 n bytes), per 64 rows the kept-row bits and
    // the group's flag over the item (12 bytes), and a 64-row list per wavefront (512 bytes).
    static size_t pairwise_lds_fixed(const Prob& P, int nthreads) {
        size_t f = (size_t)kObs * P.n_obs * sizeof(S);
        if (std::is_same<S, float>::value)
            f += (size_t)24 * P.n + (size_t)12 * ((P.np + 63) / 64) + (size_t)512 * (nthreads / 64);
        return f;
    }

    static mato_status check_lds(const Prob& P) {
        const size_t per_t = pairwise_lds_per_instant(P) + pairwise_lds_fixed(P, 1024);
        if (per_t > (size_t)(device_lds_limit() - 1024)) {
            set_error("n = %d, n_obs = %d needs %zu bytes of LDS per instant, device allows %d", P.n, P.n_obs,
                      per_t, device_lds_limit() - 1024);
            return MATO_ERR_UNSUPPORTED;
        }
        return MATO_OK;
    }

    // Work list, product groups and tiles of the active slots.
    mato_status rebuild_lists() {
        // the buffers below may be reallocated: nothing queued may still read them
        MATO_HIP(hipStreamSynchronize(stream));
        hitems.clear();
        size_t maxlds = 0;
        has_obs = false;
        for (const auto& P : probs) has_obs = has_obs || (P.active && P.n_obs > 0);
        n_active = 0;
        for (const auto& P : probs) n_active += P.active ? 1 : 0;
        for (int q = 0; q < count(); ++q)
            if (probs[q].active) slot_items(q, hitems, &maxlds, q);
        lds = maxlds;
        MATO_TRY(dev_buf(&ditems, &ditems_cap, hitems.size()));
        if (!hitems.empty())
            MATO_TRY(upload(ditems, hitems.data(), sizeof(WorkItem) * hitems.size()));
        if (lds > 0 && set_pairwise_lds_limit<S>(lds) != hipSuccess) {
            (void)hipGetLastError();
            set_error("cannot raise the LDS limit of the pairwise kernel to %zu bytes", lds);
            return MATO_ERR_UNSUPPORTED;
        }
        std::map<mato_plan, std::vector<int>> members;
        std::vector<mato_plan> order;
        for (int q = 0; q < count(); ++q) {
            if (!probs[q].active || solve == MATO_SOLVE_STRUCTURED) continue;
            if (!members.count(probs[q].plan)) order.push_back(probs[q].plan);
            members[probs[q].plan].push_back(q);
        }
        if (!refine_fixed && precision == MATO_FP32 && solve == MATO_SOLVE_DENSE) {
            refine = refine_base;
            for (const mato_plan pl : order)
                if (pl->rho * (double)(pl->n + pl->n_obs) >= kRefineRhoN) refine = refine_base + 1;
        }
        std::vector<GemmCol> colq, colr;
        hgroups.clear();
        htiles.clear();
        // tile width: 64 right-hand sides, or 48 (FP32, BF16) when that lowers the number of
        // tiles the busiest compute unit works through times the tile's work
        gemm_width = 64;
        if (precision != MATO_FP64) {
            auto makespan = [&](int w) {
                long tiles = 0;
                for (const mato_plan pl : order)
                    tiles += (long)(round_up(pl->n * pl->nv, 64) / 64) * ((3 * (long)members[pl].size() + w - 1) / w);
                return ((tiles + device_cu_count() - 1) / device_cu_count()) * w;
            };
            if (!order.empty() && makespan(48) < makespan(64)) gemm_width = 48;
        }
        for (size_t g = 0; g < order.size(); ++g) {
            const mato_plan pl = order[g];
            const auto& mem = members[pl];
            GemmGroup G;
            G.Ahi = pl->dAhi;
            G.Amid = pl->dAlo;
            G.Alo = pl->dAlo ? (const void*)((const unsigned short*)pl->dAlo +
                                             (size_t)round_up(pl->n * pl->nv, 64) * pl->ldk) : nullptr;
            G.M = pl->n * pl->nv;
            G.K = pl->n * pl->nv;
            G.ldk = pl->ldk;
            G.ncols = 3 * (int)mem.size();
            G.first_col = (int)colq.size();
            for (int q : mem)
                for (int a = 0; a < 3; ++a) {
                    const Prob& P = probs[q];
                    GemmCol cq, cr;
                    cq.c = cr.c = (double*)(P.base + P.o_c) + (size_t)a * P.ldc;
                    cq.ceq = cr.ceq = (const double*)(P.base + P.o_ceq) + (size_t)a * P.ldc;
                    cq.b = (const double*)(P.base + P.o_q) + (size_t)a * P.ldq;
                    cr.b = (const double*)(P.base + P.o_r) + (size_t)a * P.ldq;
                    cq.bf = (const float*)(P.base + P.o_qf) + (size_t)a * P.ldq;
                    cr.bf = (const float*)(P.base + P.o_rf) + (size_t)a * P.ldq;
                    cq.ctrl = cr.ctrl = dctrl + kCtrl * q;
                    colq.push_back(cq);
                    colr.push_back(cr);
                }
            hgroups.push_back(G);
            const int Mp = round_up(G.M, 64);
            for (int c0 = 0; c0 < G.ncols; c0 += gemm_width)
                for (int m0 = 0; m0 < Mp; m0 += 64) htiles.push_back(GemmTile{(int)g, m0, c0, 0});
        }
        MATO_TRY(dev_buf(&dgroups, &cap_groups, hgroups.size()));
        MATO_TRY(dev_buf(&dtiles, &cap_tiles, htiles.size()));
        MATO_TRY(dev_buf(&dcolsq, &cap_colsq, colq.size()));
        MATO_TRY(dev_buf(&dcolsr, &cap_colsr, colr.size()));
        if (!hgroups.empty()) {
            MATO_TRY(upload(dgroups, hgroups.data(), sizeof(GemmGroup) * hgroups.size()));
            MATO_TRY(upload(dtiles, htiles.data(), sizeof(GemmTile) * htiles.size()));
            MATO_TRY(upload(dcolsq, colq.data(), sizeof(GemmCol) * colq.size()));
            MATO_TRY(upload(dcolsr, colr.data(), sizeof(GemmCol) * colr.size()));
        }
        MATO_TRY(upload_desc());          // slab counts may have changed
        drop_graphs();
        lists_dirty = false;
        return MATO_OK;
    }

    // --------------------------------------------------------- slots ---
    // Binds slot q to a problem: device block (arena part or own, reused when large
    // enough), boundary data, control words, descriptor.  Does not initialise.
    mato_status attach(int q, mato_plan plan, const double* starts, const double* goals, char* arena_part,
                       const double* obstacles = nullptr) {
        Prob& P = probs[q];
        describe(P, plan);
        MATO_TRY(check_lds(P));
        if (arena_part) {
            if (P.own) dfree(P.base);
            P.own = false;
            P.base = arena_part;
        } else {
            if (!P.own || P.block < P.bytes) {
                if (P.own) dfree(P.base);
                P.base = nullptr;
                P.own = false;
                const size_t cap = block_class(P.bytes);
                if (hipMalloc(&P.base, cap) != hipSuccess) {
                    (void)hipGetLastError();
                    P.base = nullptr;
                    set_error("device allocation of %zu bytes failed", cap);
                    return MATO_ERR_OUT_OF_MEMORY;
                }
                P.own = true;
                P.block = cap;
            }
            MATO_HIP(hipMemsetAsync(P.base, 0, P.bytes, stream));
        }
        P.starts.assign(starts, starts + 3 * (size_t)P.n);
        P.goals.assign(goals, goals + 3 * (size_t)P.n);
        P.obstacles.assign((size_t)5 * P.n_obs, 0.0);
        if (P.n_obs > 0) {
            if (!obstacles) {
                set_error("the plan has %d obstacles but none were given", P.n_obs);
                return MATO_ERR_INVALID_ARG;
            }
            P.obstacles.assign(obstacles, obstacles + (size_t)5 * P.n_obs);
            for (int o = 0; o < P.n_obs; ++o) {
                const double* ob = &P.obstacles[(size_t)5 * o];
                for (int k = 0; k < 5; ++k)
                    if (!std::isfinite(ob[k])) { set_error("non-finite obstacle"); return MATO_ERR_NONFINITE; }
                if (!(ob[3] > 0) || !(ob[4] > 0)) { set_error("obstacle semi-axes must be > 0"); return MATO_ERR_INVALID_ARG; }
            }
        }
        P.stage = 0;
        P.iters_host = 0;
        for (size_t k = 0; k < P.starts.size(); ++k)
            if (!std::isfinite(P.starts[k]) || !std::isfinite(P.goals[k])) {
                set_error("non-finite start or goal");
                return MATO_ERR_NONFINITE;
            }
        P.active = true;
        hk0c[q] = plan->dK0c;
        hkinv[q] = plan->dKinv;
        MATO_TRY(upload(dk0c + q, &hk0c[q], sizeof(double*)));
        MATO_TRY(upload(dkinv + q, &hkinv[q], sizeof(double*)));
        lists_dirty = true;
        return MATO_OK;
    }

    // Marks slot q inactive; its block is kept for reuse.
    mato_status detach(int q) {
        Prob& P = probs[q];
        if (!P.active) return MATO_OK;
        P.active = false;
        const int zero[kCtrl] = {0};
        MATO_TRY(upload(dctrl + kCtrl * q, zero, sizeof(zero)));
        lists_dirty = true;
        return MATO_OK;
    }

    // Releases the device block of an inactive slot.
    void release_block(int q) {
        Prob& P = probs[q];
        if (P.active || !P.own) return;
        dfree(P.base);
        P.base = nullptr;
        P.own = false;
        P.block = 0;
        P.plan = nullptr;
    }

    // Boundary rows of q: [start, 0, 0, goal, 0, 0] per agent and axis, FP64 and FP32;
    // and the obstacle table.
    mato_status upload_beq(int q) {
        const Prob& P = probs[q];
        if (P.n_obs > 0) {
            std::vector<S> ho((size_t)kObs * P.n_obs, S(0));
            for (int o = 0; o < P.n_obs; ++o) {
                const double* ob = &P.obstacles[(size_t)5 * o];
                S* e = &ho[(size_t)kObs * o];
                e[0] = (S)ob[0]; e[1] = (S)ob[1]; e[2] = (S)ob[2];
                e[3] = (S)(1.0 / (ob[3] * ob[3])); e[4] = (S)(1.0 / (ob[4] * ob[4])); e[5] = (S)ob[4];
            }
            MATO_TRY(upload(P.base + P.o_obs, ho.data(), sizeof(S) * ho.size()));
        }
        std::vector<double> hq((size_t)3 * P.ldq, 0.0);
        for (int a = 0; a < 3; ++a)
            for (int i = 0; i < P.n; ++i) {
                double* b = &hq[(size_t)a * P.ldq + (size_t)P.n * P.nv + (size_t)i * kNb];
                b[0] = P.starts[(size_t)i * 3 + a];
                b[3] = P.goals[(size_t)i * 3 + a];
            }
        const std::vector<float> hf(hq.begin(), hq.end());
        MATO_TRY(upload(P.base + P.o_q, hq.data(), sizeof(double) * hq.size()));
        MATO_TRY(upload(P.base + P.o_qf, hf.data(), sizeof(float) * hf.size()));
        return MATO_OK;
    }

    mato_status reset_ctrl(int q) {
        int w[kCtrl] = {0};
        w[3] = 1;
        MATO_TRY(upload(dctrl + kCtrl * q, w, sizeof(w)));
        return MATO_OK;
    }

    // Initialisation of Algorithm 1 for every active slot (fixed batches).
    mato_status enqueue_init_all() {
        if (lists_dirty) MATO_TRY(rebuild_lists());
        for (int q = 0; q < count(); ++q)
            if (probs[q].active) {
                MATO_TRY(reset_ctrl(q));
                MATO_TRY(upload_beq(q));
            }
        const int nv = common_nv();
        MATO_HIP(launch_init<S>(ddesc, dk0c, count(), stream));
        MATO_HIP(launch_ceq<S>(ddesc, dkinv, count(), stream));
        MATO_HIP(launch_positions<S>(ddesc, count(), kModeInit, nv, stream));
        MATO_HIP(launch_pairwise<S>(ditems, (int)hitems.size(), ddesc, kModeInit, threads, lds, nv, has_obs, stream));
        MATO_HIP(launch_qbuild<S>(ddesc, count(), kModeInit, nv, max_agents(), stream));
        return MATO_OK;
    }

    // Initialisation of one slot (server admission): kernels launched on that slot only.
    mato_status enqueue_init_one(int q) {
        if (lists_dirty) MATO_TRY(rebuild_lists());
        MATO_TRY(reset_ctrl(q));
        MATO_TRY(upload_beq(q));
        std::vector<WorkItem> items;
        size_t l = 0;
        slot_items(q, items, &l, 0);
        if (dscratch_cap < items.size()) {
            // the list of an earlier slot's initialisation may still be in use: let it finish first
            MATO_HIP(hipStreamSynchronize(stream));
            MATO_TRY(dev_buf(&dscratch, &dscratch_cap, std::max<size_t>(items.size(), (size_t)probs[q].T)));
        }
        MATO_TRY(upload(dscratch, items.data(), sizeof(WorkItem) * items.size()));
        const int nv = probs[q].nv == 11 ? 11 : 0;
        const ProblemDesc<S>* d = ddesc + q;
        MATO_HIP(launch_init<S>(d, dk0c + q, 1, stream));
        MATO_HIP(launch_ceq<S>(d, dkinv + q, 1, stream));
        MATO_HIP(launch_positions<S>(d, 1, kModeInit, nv, stream));
        MATO_HIP(launch_pairwise<S>(dscratch, (int)items.size(), d, kModeInit, threads, std::max(l, lds), nv, has_obs, stream));
        MATO_HIP(launch_qbuild<S>(d, 1, kModeInit, nv, probs[q].n, stream));
        return MATO_OK;
    }

    // --------------------------------------------------------- iterations ---
    hipError_t enqueue_iteration(hipStream_t st, bool events) {
        const int nv = common_nv();
        hipError_t e = hipSuccess;
        if (solve == MATO_SOLVE_STRUCTURED) {
            e = launch_solve_positions<S>(ddesc, count(), nv, st);
            if (e != hipSuccess) return e;
        } else {
            e = launch_gemm(precision, gemm_width, dtiles, (int)htiles.size(), dgroups, dcolsq, 0, st);
            if (e != hipSuccess) return e;
            for (int k = 0; k < refine; ++k) {
                e = launch_residual<S>(ddesc, count(), st);
                if (e != hipSuccess) return e;
                e = launch_gemm(precision, gemm_width, dtiles, (int)htiles.size(), dgroups, dcolsr, 1, st);
                if (e != hipSuccess) return e;
            }
            if constexpr (!std::is_same<S, float>::value) {     // FP32: the pairwise kernel forms X
                e = launch_positions<S>(ddesc, count(), kModeIter, nv, st);
                if (e != hipSuccess) return e;
            }
        }
        if (events) {
            while ((int)pw_events.size() < pw_used + 2) {
                hipEvent_t ev;
                e = hipEventCreate(&ev);
                if (e != hipSuccess) return e;
                pw_events.push_back(ev);
            }
            e = hipEventRecord(pw_events[pw_used], st);
            if (e != hipSuccess) return e;
        }
        e = launch_pairwise<S>(ditems, (int)hitems.size(), ddesc, kModeIter, threads, lds, nv, has_obs, st);
        if (e != hipSuccess) return e;
        if (events) {
            e = hipEventRecord(pw_events[pw_used + 1], st);
            if (e != hipSuccess) return e;
            pw_used += 2;
        }
        return launch_qbuild<S>(ddesc, count(), kModeIter, nv, max_agents(), st);
    }

    void drop_graphs() {
        if (g1) (void)hipGraphExecDestroy(g1);
        if (gC) (void)hipGraphExecDestroy(gC);
        g1 = gC = nullptr;
    }

    mato_status capture(int iters, hipGraphExec_t* out) {
        if (!cap_stream) MATO_HIP(hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking));
        MATO_HIP(hipStreamBeginCapture(cap_stream, hipStreamCaptureModeRelaxed));
        hipError_t e = hipSuccess;
        for (int k = 0; k < iters && e == hipSuccess; ++k) e = enqueue_iteration(cap_stream, false);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(cap_stream, &g);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            set_error("graph capture failed: %s", hipGetErrorString(e != hipSuccess ? e : e2));
            return MATO_ERR_HIP;
        }
        e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            set_error("graph instantiation failed: %s", hipGetErrorString(e));
            return MATO_ERR_HIP;
        }
        return MATO_OK;
    }

    mato_status set_tol(double new_tol) {
        if (new_tol != tol) {
            tol = new_tol;
            MATO_TRY(upload_desc());
        }
        return MATO_OK;
    }

    mato_status run_segment(int k, bool use_graph, bool per_kernel_events) {
        if (ext) use_graph = false;       // instantiating a graph may allocate
        if (lists_dirty) MATO_TRY(rebuild_lists());
        if (active_count() == 0 || k <= 0) return MATO_OK;
        if (use_graph) {
            if (!gC && k >= kChunk) MATO_TRY(capture(kChunk, &gC));
            if (!g1) MATO_TRY(capture(1, &g1));
            int left = k;
            while (left >= kChunk) {
                MATO_HIP(hipGraphLaunch(gC, stream));
                left -= kChunk;
            }
            while (left-- > 0) MATO_HIP(hipGraphLaunch(g1, stream));
        } else {
            for (int i = 0; i < k; ++i) MATO_HIP(enqueue_iteration(stream, per_kernel_events));
        }
        for (auto& P : probs)
            if (P.active) P.iters_host += k;
        return MATO_OK;
    }

    // Slots whose enqueued iteration count reached their next stage move to it: the
    // stage's plan (K^{-1}, rho) and its c_eq = K12^{-1} b_eq.
    mato_status advance_stages() {
        std::vector<int> moved;
        for (int q = 0; q < count(); ++q) {
            Prob& P = probs[q];
            if (!P.active || P.stage + 1 >= (int)P.stages.size()) continue;
            if (P.iters_host != P.stage_start[P.stage + 1]) continue;
            P.stage += 1;
            P.plan = P.stages[P.stage];
            moved.push_back(q);
        }
        if (moved.empty()) return MATO_OK;
        if (solve == MATO_SOLVE_STRUCTURED) {
            // only the moved slots' descriptors change (rho, the per-agent inverses): the work
            // lists and any captured graphs stay valid, and the uploads are stream-ordered after
            // the iterations already queued
            for (int q : moved) {
                fill_desc(q);
                hkinv[q] = probs[q].plan->dKinv;
                MATO_TRY(upload(dkinv + q, &hkinv[q], sizeof(double*)));
                MATO_TRY(upload(ddesc + q, &hdesc[q], sizeof(ProblemDesc<S>)));
            }
        } else {
            MATO_HIP(hipStreamSynchronize(stream));
            for (int q : moved) {
                hkinv[q] = probs[q].plan->dKinv;
                MATO_TRY(upload(dkinv + q, &hkinv[q], sizeof(double*)));
            }
            MATO_TRY(rebuild_lists());        // the product groups follow the plans
        }
        // c_eq of the moved slots in one launch over every slot (for the others it is
        // recomputed from the same plan and boundary data, so it does not change)
        MATO_HIP(launch_ceq<S>(ddesc, dkinv, count(), stream));
        return MATO_OK;
    }

    // iterations until some active slot reaches its next stage (large if none)
    int until_next_stage() const {
        int m = 1 << 30;
        for (const auto& P : probs)
            if (P.active && P.stage + 1 < (int)P.stages.size())
                m = std::min(m, std::max(1, P.stage_start[P.stage + 1] - P.iters_host));
        return m;
    }

    mato_status step(int k, double new_tol, bool use_graph) {
        if (k < 0) { set_error("negative iteration count"); return MATO_ERR_INVALID_ARG; }
        MATO_TRY(set_tol(new_tol));
        if (lists_dirty) MATO_TRY(rebuild_lists());
        pw_used = 0;
        last_timed = timing;
        const bool per_kernel_events = timing && !use_graph;
        if (timing) MATO_HIP(hipEventRecord(ev0, stream));
        int left = k;
        while (left > 0) {
            const int seg = std::min(left, until_next_stage());
            MATO_TRY(run_segment(seg, use_graph, per_kernel_events));
            MATO_TRY(advance_stages());
            left -= seg;
        }
        if (timing) MATO_HIP(hipEventRecord(ev1, stream));
        return MATO_OK;
    }

    mato_status read_ctrl(std::vector<int>& ctrl) {
        ctrl.resize((size_t)kCtrl * count());
        MATO_HIP(hipMemcpyAsync(ctrl.data(), dctrl, sizeof(int) * ctrl.size(), hipMemcpyDeviceToHost, stream));
        MATO_HIP(hipStreamSynchronize(stream));
        return MATO_OK;
    }

    mato_status run(int iters, double new_tol, int check_every) {
        if (iters < 0 || check_every < 1) { set_error("iters must be >= 0 and check_every >= 1"); return MATO_ERR_INVALID_ARG; }
        int done = 0;
        std::vector<int> ctrl;
        while (done < iters) {
            const int k = std::min(check_every, iters - done);
            MATO_TRY(step(k, new_tol, true));
            done += k;
            MATO_TRY(read_ctrl(ctrl));
            bool all = true;
            for (int q = 0; q < count(); ++q)
                if (probs[q].active) all = all && ctrl[kCtrl * q + 1];
            if (all) break;
        }
        MATO_TRY(read_ctrl(ctrl));
        bool nonfinite = false, pending = false;
        for (int q = 0; q < count(); ++q) {
            if (!probs[q].active) continue;
            nonfinite = nonfinite || ctrl[kCtrl * q + 2];
            pending = pending || !ctrl[kCtrl * q + 4];
        }
        if (nonfinite) { set_error("non-finite values in the iteration"); return MATO_ERR_NONFINITE; }
        if (pending && new_tol > 0) return MATO_WARN_NOT_CONVERGED;
        return MATO_OK;
    }

    mato_status set_tiles(int ipw, int thr) {
        if (ipw < 1 || (thr != 256 && thr != 512 && thr != 1024)) {
            set_error("items_per_wg must be >= 1 and threads one of 256, 512, 1024");
            return MATO_ERR_INVALID_ARG;
        }
        MATO_HIP(hipStreamSynchronize(stream));
        items_per_wg = ipw;
        threads = thr;
        tiles_set = true;
        return rebuild_lists();
    }

    std::string tune_key() const {
        hipDeviceProp_t prop;
        int dev = 0;
        std::string arch = "gfx";
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
        std::vector<int> ns;
        int T = 0;
        for (auto& P : probs)
            if (P.active) {
                ns.push_back(P.n);
                T = P.T;
            }
        std::sort(ns.begin(), ns.end());
        uint64_t h = 1469598103934665603ull;
        for (int v : ns) h = (h ^ (uint64_t)v) * 1099511628211ull;
        std::ostringstream o;
        o << arch.substr(0, arch.find(':')) << "|prec=" << precision << "|T=" << T << "|count=" << ns.size()
          << "|ns=" << std::hex << h;
        return o.str();
    }

    // Times the pairwise launch for candidate shapes on this batch's problems, keeps
    // the fastest and re-initialises the state (the timing runs overwrite it).
    mato_status autotune(int* ipw_out, int* thr_out) {
        const char* path = getenv("MATO_TUNE_CACHE");
        const std::string key = tune_key();
        if (path) {
            std::ifstream f(path);
            std::string k;
            int ipw, thr;
            while (f >> k >> ipw >> thr)
                if (k == key) {
                    MATO_TRY(set_tiles(ipw, thr));
                    if (ipw_out) *ipw_out = ipw;
                    if (thr_out) *thr_out = thr;
                    return MATO_OK;
                }
        }
        const int ipws[] = {512, 1024, 2048, 4096, 8192, 16384, 32768};
        const int thrs[] = {256, 512, 1024};
        float best = 1e30f;
        int bi = items_per_wg, bt = threads;
        hipEvent_t e0, e1;
        MATO_HIP(hipEventCreate(&e0));
        MATO_HIP(hipEventCreate(&e1));
        const int nv = common_nv();
        for (int ipw : ipws)
            for (int thr : thrs) {
                if (set_tiles(ipw, thr) != MATO_OK) continue;
                MATO_HIP(launch_pairwise<S>(ditems, (int)hitems.size(), ddesc, kModeIter, threads, lds, nv, has_obs, stream));
                MATO_HIP(hipEventRecord(e0, stream));
                const int reps = 5;
                for (int r = 0; r < reps; ++r)
                    MATO_HIP(launch_pairwise<S>(ditems, (int)hitems.size(), ddesc, kModeIter, threads, lds, nv, has_obs, stream));
                MATO_HIP(hipEventRecord(e1, stream));
                MATO_HIP(hipEventSynchronize(e1));
                float ms = 0.f;
                MATO_HIP(hipEventElapsedTime(&ms, e0, e1));
                if (ms < best) { best = ms; bi = ipw; bt = thr; }
            }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        MATO_TRY(set_tiles(bi, bt));
        MATO_TRY(enqueue_init_all());
        MATO_HIP(hipStreamSynchronize(stream));
        if (path) {
            std::ofstream f(path, std::ios::app);
            f << key << " " << bi << " " << bt << "\n";
        }
        if (ipw_out) *ipw_out = bi;
        if (thr_out) *thr_out = bt;
        return MATO_OK;
    }

    mato_status enable_debug(bool on) {
        MATO_HIP(hipStreamSynchronize(stream));
        if (on && !dbg) {
            size_t elems = 0;
            for (auto& P : probs) elems += (size_t)P.T * 4 * (size_t)P.np;
            dbg_bytes = sizeof(S) * std::max<size_t>(elems, 1);
            MATO_HIP(hipMalloc(&dbg, dbg_bytes));
            MATO_HIP(hipMemset(dbg, 0, dbg_bytes));
        }
        debug = on;
        return upload_desc();
    }
};

}  // namespace mato
