// Host runtime of libmato: batches of independent problems advanced together,
// one pass of the while-loop of Algorithm 1 per iteration:
//
//   [inverse product]   c = [K11^{-1}|K12^{-1}] [g ; b_eq]       (eq. (kkt_step_x))
//   [refinement x R]    r = [g - H c ; b_eq - A c] (FP64);  c += [K11^{-1}|K12^{-1}] r
//   [pairwise]          X = P c; delta; alpha, beta; d; lambda; b_fc; S   (eqs. (sphere_project)
//                       -(lag_update), (b_f))
//   [linear term]       g = rho P^T S = rho A_fc^T b_fc; residual record; convergence test
//
// Problems with the same plan form one group; their right-hand sides are the
// columns of one matrix-matrix product.  All pairwise work of all problems is one
// launch over a work list of (problem, block of instants) items.  Device memory
// for all problems lives in one arena.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>

#include "common.h"

namespace mato {

template <typename S>
hipError_t launch_pairwise(const WorkItem*, int, const ProblemDesc<S>*, int, int, size_t, int, hipStream_t);
template <typename S>
hipError_t set_pairwise_lds_limit(size_t);
template <typename S>
hipError_t launch_qbuild(const ProblemDesc<S>*, int, int, int, hipStream_t);
template <typename S>
hipError_t launch_residual(const ProblemDesc<S>*, int, hipStream_t);
template <typename S>
hipError_t launch_positions(const ProblemDesc<S>*, int, int, int, hipStream_t);
template <typename S>
hipError_t launch_init(const ProblemDesc<S>*, const double* const*, int, hipStream_t);
template <typename S>
hipError_t launch_ceq(const ProblemDesc<S>*, const double* const*, int, hipStream_t);
hipError_t launch_gemm(int, const GemmTile*, int, const GemmGroup*, const GemmCol*, int, hipStream_t);

static int device_lds_limit() {
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

template <typename S>
struct BatchImpl {
    struct Prob {
        mato_plan plan;
        int n, np, T, nv, ldq, ldc;
        size_t o_lam, o_ssum, o_X, o_misc, o_c, o_ceq, o_q, o_r, o_qf, o_rf, o_part, o_hist;
        int nslab = 0;
    };
    int precision = MATO_FP32;
    int refine = 1;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    std::vector<Prob> probs;
    std::vector<double> starts, goals;       // host copies, [problem offsets]
    std::vector<int> agent_off;

    char* arena = nullptr;
    size_t arena_bytes = 0;
    int* dctrl = nullptr;                    // [count][4]
    std::vector<ProblemDesc<S>> hdesc;
    ProblemDesc<S>* ddesc = nullptr;
    double** dk0c = nullptr;
    double** dkinv = nullptr;

    std::vector<WorkItem> hitems;
    WorkItem* ditems = nullptr;
    int items_per_wg = 2048, threads = 256;
    size_t lds = 0;

    std::vector<GemmGroup> hgroups;
    std::vector<GemmTile> htiles;
    GemmGroup* dgroups = nullptr;
    GemmTile* dtiles = nullptr;
    GemmCol* dcolsq = nullptr;
    GemmCol* dcolsr = nullptr;

    double tol = 0.0;
    bool debug = false;
    S* dbg = nullptr;                        // debug arena
    size_t dbg_bytes = 0;

    hipGraphExec_t g1 = nullptr, gC = nullptr;
    static constexpr int kChunk = 16;

    bool timing = false;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    std::vector<hipEvent_t> pw_events;       // pairs around pairwise launches
    int pw_used = 0;
    bool last_timed = false;

    ~BatchImpl() {
        if (g1) (void)hipGraphExecDestroy(g1);
        if (gC) (void)hipGraphExecDestroy(gC);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        dfree(arena);
        dfree(dctrl);
        dfree(ddesc);
        dfree(dk0c);
        dfree(dkinv);
        dfree(ditems);
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

    // number of basis coefficients shared by every problem (0 if they differ)
    int common_nv() const {
        int nv = probs.empty() ? 0 : probs[0].nv;
        for (const auto& P : probs)
            if (P.nv != nv) return 0;
        return nv;
    }

    // ------------------------------------------------------------ layout ---
    mato_status build_items() {
        hitems.clear();
        size_t maxlds = 0;
        const int cap = device_lds_limit() - 1024;   // room for the kernel's static reduction buffer
        for (int q = 0; q < count(); ++q) {
            Prob& P = probs[q];
            const size_t per_t = (size_t)3 * (P.n + P.np) * sizeof(S);
            int tc = std::max(1, items_per_wg / std::max(1, P.np));
            tc = std::min(tc, P.T);
            while (tc > 1 && per_t * tc > (size_t)cap) --tc;
            if (per_t * tc > (size_t)cap) {
                set_error("n = %d needs %zu bytes of LDS per instant, device allows %d", P.n, per_t, cap);
                return MATO_ERR_UNSUPPORTED;
            }
            maxlds = std::max(maxlds, per_t * tc);
            P.nslab = (P.T + tc - 1) / tc;
            for (int s = 0; s < P.nslab; ++s) {
                WorkItem w;
                w.prob = q;
                w.t0 = s * tc;
                w.tc = std::min(tc, P.T - w.t0);
                w.slab = s;
                hitems.push_back(w);
            }
        }
        lds = maxlds;
        return MATO_OK;
    }

    size_t part_bytes_for(const Prob& P) const { return sizeof(double) * 4 * (size_t)P.T; }

    mato_status allocate(hipStream_t st) {
        auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
        size_t off = 0;
        for (auto& P : probs) {
            P.o_lam = off;  off += al(sizeof(S) * (size_t)P.T * 3 * P.np);
            P.o_ssum = off; off += al(sizeof(S) * (size_t)P.T * 3 * P.n);
            P.o_X = off;    off += al(sizeof(S) * (size_t)P.T * 3 * P.n);
            P.o_misc = off; off += al(sizeof(double) * 4);
            P.o_c = off;    off += al(sizeof(double) * 3 * (size_t)P.ldc);
            P.o_ceq = off;  off += al(sizeof(double) * 3 * (size_t)P.ldc);
            P.o_q = off;    off += al(sizeof(double) * 3 * (size_t)P.ldq);
            P.o_r = off;    off += al(sizeof(double) * 3 * (size_t)P.ldq);
            P.o_qf = off;   off += al(sizeof(float) * 3 * (size_t)P.ldq);
            P.o_rf = off;   off += al(sizeof(float) * 3 * (size_t)P.ldq);
            P.o_part = off; off += al(part_bytes_for(P));   // at most T slabs
            P.o_hist = off; off += al(sizeof(double) * 3 * kHistCap);
        }
        arena_bytes = std::max<size_t>(off, 256);
        if (hipMalloc(&arena, arena_bytes) != hipSuccess) {
            (void)hipGetLastError();
            set_error("device allocation of %zu bytes failed", arena_bytes);
            return MATO_ERR_OUT_OF_MEMORY;
        }
        MATO_HIP(hipMemsetAsync(arena, 0, arena_bytes, st));
        MATO_HIP(hipMalloc(&dctrl, sizeof(int) * 4 * count()));
        MATO_HIP(hipMalloc(&ddesc, sizeof(ProblemDesc<S>) * count()));
        MATO_HIP(hipMalloc(&dk0c, sizeof(double*) * count()));
        MATO_HIP(hipMalloc(&dkinv, sizeof(double*) * count()));
        std::vector<double*> k0(count()), ki(count());
        for (int q = 0; q < count(); ++q) {
            k0[q] = probs[q].plan->dK0c;
            ki[q] = probs[q].plan->dKinv;
        }
        MATO_HIP(hipMemcpy(dk0c, k0.data(), sizeof(double*) * count(), hipMemcpyHostToDevice));
        MATO_HIP(hipMemcpy(dkinv, ki.data(), sizeof(double*) * count(), hipMemcpyHostToDevice));
        return MATO_OK;
    }

    void fill_desc() {
        hdesc.resize(count());
        for (int q = 0; q < count(); ++q) {
            const Prob& P = probs[q];
            const mato_plan pl = P.plan;
            ProblemDesc<S>& D = hdesc[q];
            memset(&D, 0, sizeof(D));
            D.n = P.n; D.np = P.np; D.T = P.T; D.nv = P.nv; D.ldq = P.ldq; D.ldc = P.ldc;
            D.nslab = P.nslab; D.hist_cap = kHistCap;
            D.a = pl->a; D.b = pl->b; D.rho = pl->rho;
            D.ia2 = (S)(1.0 / (pl->a * pl->a));
            D.ib2 = (S)(1.0 / (pl->b * pl->b));
            D.lz = (S)pl->b;
            D.srho = (S)pl->rho;
            D.sirho = (S)(1.0 / pl->rho);
            D.P = pl->dP; D.Pdd = pl->dPdd; D.PtP = pl->dPtP; D.PddtPdd = pl->dPddtPdd; D.A = pl->dA;
            D.pairs = pl->dPairs;
            D.lam = (S*)(arena + P.o_lam);
            D.ssum = (S*)(arena + P.o_ssum);
            D.X = (S*)(arena + P.o_X);
            D.misc = (double*)(arena + P.o_misc);
            D.c = (double*)(arena + P.o_c);
            D.ceq = (double*)(arena + P.o_ceq);
            D.q = (double*)(arena + P.o_q);
            D.r = (double*)(arena + P.o_r);
            D.qf = (float*)(arena + P.o_qf);
            D.rf = (float*)(arena + P.o_rf);
            D.part = (double*)(arena + P.o_part);
            D.hist = (double*)(arena + P.o_hist);
            D.ctrl = dctrl + 4 * q;
            D.tol = tol;
        }
        if (debug && dbg) {
            size_t off = 0;
            for (int q = 0; q < count(); ++q) {
                const Prob& P = probs[q];
                hdesc[q].dbg_proj = dbg + off; off += (size_t)P.T * 3 * P.np;
                hdesc[q].dbg_d = dbg + off;    off += (size_t)P.T * P.np;
            }
        }
    }

    mato_status upload_desc() {
        fill_desc();
        MATO_HIP(hipMemcpyAsync(ddesc, hdesc.data(), sizeof(ProblemDesc<S>) * count(), hipMemcpyHostToDevice, stream));
        MATO_HIP(hipStreamSynchronize(stream));
        return MATO_OK;
    }

    mato_status upload_items() {
        dfree(ditems);
        ditems = nullptr;
        MATO_HIP(hipMalloc(&ditems, sizeof(WorkItem) * std::max<size_t>(1, hitems.size())));
        MATO_HIP(hipMemcpy(ditems, hitems.data(), sizeof(WorkItem) * hitems.size(), hipMemcpyHostToDevice));
        if (set_pairwise_lds_limit<S>(std::max<size_t>(lds, 1)) != hipSuccess) {
            (void)hipGetLastError();
            set_error("cannot raise the LDS limit of the pairwise kernel to %zu bytes", lds);
            return MATO_ERR_UNSUPPORTED;
        }
        return MATO_OK;
    }

    mato_status build_gemm() {
        std::map<mato_plan, std::vector<int>> members;
        std::vector<mato_plan> order;
        for (int q = 0; q < count(); ++q) {
            if (!members.count(probs[q].plan)) order.push_back(probs[q].plan);
            members[probs[q].plan].push_back(q);
        }
        std::vector<GemmCol> colq, colr;
        hgroups.clear();
        htiles.clear();
        for (size_t g = 0; g < order.size(); ++g) {
            const mato_plan pl = order[g];
            const auto& mem = members[pl];
            GemmGroup G;
            G.Ahi = pl->dAhi;
            G.Alo = pl->dAlo;
            G.M = pl->n * pl->nv;
            G.K = pl->n * pl->nv;
            G.ldk = pl->ldk;
            G.ncols = 3 * (int)mem.size();
            G.first_col = (int)colq.size();
            for (int q : mem)
                for (int a = 0; a < 3; ++a) {
                    const Prob& P = probs[q];
                    GemmCol cq, cr;
                    cq.c = cr.c = (double*)(arena + P.o_c) + (size_t)a * P.ldc;
                    cq.ceq = cr.ceq = (const double*)(arena + P.o_ceq) + (size_t)a * P.ldc;
                    cq.b = (const double*)(arena + P.o_q) + (size_t)a * P.ldq;
                    cr.b = (const double*)(arena + P.o_r) + (size_t)a * P.ldq;
                    cq.bf = (const float*)(arena + P.o_qf) + (size_t)a * P.ldq;
                    cr.bf = (const float*)(arena + P.o_rf) + (size_t)a * P.ldq;
                    cq.ctrl = cr.ctrl = dctrl + 4 * q;
                    colq.push_back(cq);
                    colr.push_back(cr);
                }
            hgroups.push_back(G);
            const int Mp = round_up(G.M, 64);
            for (int c0 = 0; c0 < G.ncols; c0 += 64)
                for (int m0 = 0; m0 < Mp; m0 += 64) htiles.push_back(GemmTile{(int)g, m0, c0, 0});
        }
        MATO_HIP(hipMalloc(&dgroups, sizeof(GemmGroup) * hgroups.size()));
        MATO_HIP(hipMalloc(&dtiles, sizeof(GemmTile) * htiles.size()));
        MATO_HIP(hipMalloc(&dcolsq, sizeof(GemmCol) * colq.size()));
        MATO_HIP(hipMalloc(&dcolsr, sizeof(GemmCol) * colr.size()));
        MATO_HIP(hipMemcpy(dgroups, hgroups.data(), sizeof(GemmGroup) * hgroups.size(), hipMemcpyHostToDevice));
        MATO_HIP(hipMemcpy(dtiles, htiles.data(), sizeof(GemmTile) * htiles.size(), hipMemcpyHostToDevice));
        MATO_HIP(hipMemcpy(dcolsq, colq.data(), sizeof(GemmCol) * colq.size(), hipMemcpyHostToDevice));
        MATO_HIP(hipMemcpy(dcolsr, colr.data(), sizeof(GemmCol) * colr.size(), hipMemcpyHostToDevice));
        return MATO_OK;
    }

    // --------------------------------------------------------- launches ---
    mato_status enqueue_init() {
        // ctrl = {0 iterations, not converged, finite, active}
        std::vector<int> ctrl(4 * count(), 0);
        for (int q = 0; q < count(); ++q) ctrl[4 * q + 3] = 1;
        MATO_HIP(hipMemcpyAsync(dctrl, ctrl.data(), sizeof(int) * ctrl.size(), hipMemcpyHostToDevice, stream));
        // b_eq part of q for every problem and axis: [start, 0, 0, goal, 0, 0] per agent
        for (int q = 0; q < count(); ++q) {
            const Prob& P = probs[q];
            std::vector<double> hq((size_t)3 * P.ldq, 0.0);
            for (int a = 0; a < 3; ++a)
                for (int i = 0; i < P.n; ++i) {
                    double* b = &hq[(size_t)a * P.ldq + (size_t)P.n * P.nv + (size_t)i * kNb];
                    b[0] = starts[(size_t)(agent_off[q] + i) * 3 + a];
                    b[3] = goals[(size_t)(agent_off[q] + i) * 3 + a];
                }
            std::vector<float> hf(hq.begin(), hq.end());
            MATO_HIP(hipMemcpyAsync(arena + P.o_q, hq.data(), sizeof(double) * hq.size(), hipMemcpyHostToDevice, stream));
            MATO_HIP(hipMemcpyAsync(arena + P.o_qf, hf.data(), sizeof(float) * hf.size(), hipMemcpyHostToDevice, stream));
            MATO_HIP(hipStreamSynchronize(stream));
        }
        MATO_HIP(launch_init<S>(ddesc, dk0c, count(), stream));
        MATO_HIP(launch_ceq<S>(ddesc, dkinv, count(), stream));
        MATO_HIP(launch_positions<S>(ddesc, count(), kModeInit, common_nv(), stream));
        MATO_HIP(launch_pairwise<S>(ditems, (int)hitems.size(), ddesc, kModeInit, threads, lds, common_nv(), stream));
        MATO_HIP(launch_qbuild<S>(ddesc, count(), kModeInit, common_nv(), stream));
        return MATO_OK;
    }

    hipError_t enqueue_iteration(hipStream_t st, bool events) {
        hipError_t e = launch_gemm(precision, dtiles, (int)htiles.size(), dgroups, dcolsq, 0, st);
        if (e != hipSuccess) return e;
        for (int k = 0; k < refine; ++k) {
            e = launch_residual<S>(ddesc, count(), st);
            if (e != hipSuccess) return e;
            e = launch_gemm(precision, dtiles, (int)htiles.size(), dgroups, dcolsr, 1, st);
            if (e != hipSuccess) return e;
        }
        e = launch_positions<S>(ddesc, count(), kModeIter, common_nv(), st);
        if (e != hipSuccess) return e;
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
        e = launch_pairwise<S>(ditems, (int)hitems.size(), ddesc, kModeIter, threads, lds, common_nv(), st);
        if (e != hipSuccess) return e;
        if (events) {
            e = hipEventRecord(pw_events[pw_used + 1], st);
            if (e != hipSuccess) return e;
            pw_used += 2;
        }
        return launch_qbuild<S>(ddesc, count(), kModeIter, common_nv(), st);
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

    mato_status step(int k, double new_tol, bool use_graph) {
        if (k < 0) { set_error("negative iteration count"); return MATO_ERR_INVALID_ARG; }
        if (new_tol != tol) {
            tol = new_tol;
            MATO_TRY(upload_desc());
        }
        pw_used = 0;
        last_timed = timing;
        const bool per_kernel_events = timing && !use_graph;
        if (timing) MATO_HIP(hipEventRecord(ev0, stream));
        if (use_graph && k > 0) {
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
        if (timing) MATO_HIP(hipEventRecord(ev1, stream));
        return MATO_OK;
    }

    mato_status read_ctrl(std::vector<int>& ctrl) {
        ctrl.resize(4 * count());
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
            for (int q = 0; q < count(); ++q) all = all && ctrl[4 * q + 1];
            if (all) break;
        }
        MATO_TRY(read_ctrl(ctrl));
        bool nonfinite = false, pending = false;
        for (int q = 0; q < count(); ++q) {
            nonfinite = nonfinite || ctrl[4 * q + 2];
            pending = pending || !ctrl[4 * q + 1];
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
        MATO_TRY(build_items());
        MATO_TRY(upload_items());
        MATO_TRY(upload_desc());
        drop_graphs();
        return MATO_OK;
    }

    std::string tune_key() const {
        hipDeviceProp_t prop;
        int dev = 0;
        std::string arch = "gfx";
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
        std::vector<int> ns;
        for (auto& P : probs) ns.push_back(P.n);
        std::sort(ns.begin(), ns.end());
        uint64_t h = 1469598103934665603ull;
        for (int v : ns) h = (h ^ (uint64_t)v) * 1099511628211ull;
        std::ostringstream o;
        o << arch.substr(0, arch.find(':')) << "|prec=" << precision << "|T=" << probs[0].T
          << "|count=" << count() << "|ns=" << std::hex << h;
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
        const int ipws[] = {512, 1024, 2048, 4096, 8192, 16384};
        const int thrs[] = {256, 512, 1024};
        float best = 1e30f;
        int bi = items_per_wg, bt = threads;
        hipEvent_t e0, e1;
        MATO_HIP(hipEventCreate(&e0));
        MATO_HIP(hipEventCreate(&e1));
        for (int ipw : ipws)
            for (int thr : thrs) {
                if (set_tiles(ipw, thr) != MATO_OK) continue;
                MATO_HIP(launch_pairwise<S>(ditems, (int)hitems.size(), ddesc, kModeIter, threads, lds, common_nv(), stream));
                MATO_HIP(hipEventRecord(e0, stream));
                const int reps = 5;
                for (int r = 0; r < reps; ++r)
                    MATO_HIP(launch_pairwise<S>(ditems, (int)hitems.size(), ddesc, kModeIter, threads, lds, common_nv(), stream));
                MATO_HIP(hipEventRecord(e1, stream));
                MATO_HIP(hipEventSynchronize(e1));
                float ms = 0.f;
                MATO_HIP(hipEventElapsedTime(&ms, e0, e1));
                if (ms < best) { best = ms; bi = ipw; bt = thr; }
            }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        MATO_TRY(set_tiles(bi, bt));
        MATO_TRY(enqueue_init());
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

// ----------------------------------------------------------- creation ---
template <typename S>
static mato_status batch_create(int count, const mato_plan* plans, const double* starts,
                                const double* goals, hipStream_t st, BatchImpl<S>** out) {
    auto* B = new BatchImpl<S>();
    B->precision = plans[0]->precision;
    B->refine = (B->precision == MATO_FP32) ? 1 : (B->precision == MATO_BF16_REFINED ? 2 : 0);
    if (const char* e = getenv("MATO_REFINE")) B->refine = std::max(0, std::min(kMaxRefine, atoi(e)));
    B->stream = st;
    int agents = 0;
    for (int q = 0; q < count; ++q) {
        typename BatchImpl<S>::Prob P;
        P.plan = plans[q];
        P.n = plans[q]->n;
        P.np = P.n * (P.n - 1) / 2;
        P.T = plans[q]->T;
        P.nv = plans[q]->nv;
        P.ldq = round_up(P.n * (P.nv + kNb), 32);   // >= the operand stride ldk = round_up(11n, 32)
        P.ldc = P.n * P.nv;
        B->probs.push_back(P);
        B->agent_off.push_back(agents);
        agents += P.n;
    }
    B->starts.resize((size_t)agents * 3);
    B->goals.resize((size_t)agents * 3);
    auto fail = [&](mato_status s) { delete B; return s; };
    if (hipMemcpy(B->starts.data(), starts, sizeof(double) * B->starts.size(), hipMemcpyDefault) != hipSuccess ||
        hipMemcpy(B->goals.data(), goals, sizeof(double) * B->goals.size(), hipMemcpyDefault) != hipSuccess) {
        (void)hipGetLastError();
        set_error("cannot read starts/goals");
        return fail(MATO_ERR_INVALID_ARG);
    }
    for (size_t k = 0; k < B->starts.size(); ++k)
        if (!std::isfinite(B->starts[k]) || !std::isfinite(B->goals[k])) {
            set_error("non-finite start or goal");
            return fail(MATO_ERR_NONFINITE);
        }
    mato_status s;
    if ((s = B->build_items()) != MATO_OK) return fail(s);
    if ((s = B->allocate(st)) != MATO_OK) return fail(s);
    if ((s = B->upload_items()) != MATO_OK) return fail(s);
    if ((s = B->upload_desc()) != MATO_OK) return fail(s);
    if ((s = B->build_gemm()) != MATO_OK) return fail(s);
    if (hipEventCreate(&B->ev0) != hipSuccess || hipEventCreate(&B->ev1) != hipSuccess) {
        set_error("event creation failed");
        return fail(MATO_ERR_HIP);
    }
    if ((s = B->enqueue_init()) != MATO_OK) return fail(s);
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
    if (!out || !plans || !starts || !goals || count < 1) { set_error("invalid arguments"); return MATO_ERR_INVALID_ARG; }
    *out = nullptr;
    for (int q = 0; q < count; ++q)
        if (!plans[q] || plans[q]->precision != plans[0]->precision) {
            set_error("plan %d is null or of another precision", q);
            return MATO_ERR_INVALID_ARG;
        }
    auto* b = new mato_batch_s();
    b->precision = plans[0]->precision;
    mato_status s;
    if (b->precision == MATO_FP64) {
        BatchImpl<double>* B = nullptr;
        s = batch_create<double>(count, plans, starts, goals, (hipStream_t)hip_stream, &B);
        b->impl = B;
    } else {
        BatchImpl<float>* B = nullptr;
        s = batch_create<float>(count, plans, starts, goals, (hipStream_t)hip_stream, &B);
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
        if (iters) *iters = ctrl[4 * q];
        if (converged) *converged = ctrl[4 * q + 1] && !ctrl[4 * q + 2];
        if (ctrl[4 * q + 2]) { set_error("problem %d produced non-finite values", q); return MATO_ERR_NONFINITE; }
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
        MATO_HIP(hipMemcpy(h.data(), B->arena + P.o_c, sizeof(double) * h.size(), hipMemcpyDeviceToHost));
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
        const int it = std::min(std::min(ctrl[4 * q], kHistCap), std::max(0, (int)cap));
        std::vector<double> h((size_t)3 * std::max(it, 1));
        const auto& P = B->probs[q];
        if (it > 0) MATO_HIP(hipMemcpy(h.data(), B->arena + P.o_hist, sizeof(double) * 3 * it, hipMemcpyDeviceToHost));
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
    auto pairwise_out = [&](const S* dsrc, void* dst) -> mato_status {
        std::vector<S> h(npt * 3), o(npt * 3);
        MATO_HIP(hipMemcpy(h.data(), dsrc, sizeof(S) * h.size(), hipMemcpyDeviceToHost));
        for (int t = 0; t < P.T; ++t)
            for (int a = 0; a < 3; ++a)
                for (int p = 0; p < P.np; ++p)
                    o[((size_t)p * P.T + t) * 3 + a] = h[((size_t)t * 3 + a) * P.np + p];
        return copy_out(dst, o.data(), sizeof(S) * o.size());
    };
    if (lambda) MATO_TRY(pairwise_out((const S*)(B->arena + P.o_lam), lambda));
    const ProblemDesc<S>& D = B->hdesc[q];
    if ((proj || d) && !D.dbg_proj) { set_error("enable mato_batch_debug before reading proj or d"); return MATO_ERR_INVALID_ARG; }
    if (proj) MATO_TRY(pairwise_out(D.dbg_proj, proj));
    if (d) {
        std::vector<S> h(npt), o(npt);
        MATO_HIP(hipMemcpy(h.data(), D.dbg_d, sizeof(S) * npt, hipMemcpyDeviceToHost));
        for (int t = 0; t < P.T; ++t)
            for (int p = 0; p < P.np; ++p) o[(size_t)p * P.T + t] = h[(size_t)t * P.np + p];
        MATO_TRY(copy_out(d, o.data(), sizeof(S) * npt));
    }
    if (X) {
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
    auto to_internal = [&](const void* src, std::vector<S>& dst) -> mato_status {
        MATO_HIP(hipMemcpy(in.data(), src, sizeof(S) * in.size(), hipMemcpyDefault));
        for (size_t e = 0; e < in.size(); ++e)
            if (!std::isfinite((double)in[e])) { set_error("non-finite state"); return MATO_ERR_NONFINITE; }
        for (int p = 0; p < P.np; ++p)
            for (int t = 0; t < P.T; ++t)
                for (int a = 0; a < 3; ++a) dst[((size_t)t * 3 + a) * P.np + p] = in[((size_t)p * P.T + t) * 3 + a];
        return MATO_OK;
    };
    MATO_TRY(to_internal(lambda, lam_i));
    MATO_TRY(to_internal(proj, proj_i));
    MATO_HIP(hipMemcpy(B->arena + P.o_lam, lam_i.data(), sizeof(S) * lam_i.size(), hipMemcpyHostToDevice));
    if (c) {
        std::vector<double> hc((size_t)P.n * 3 * P.nv), o((size_t)3 * P.ldc, 0.0);
        MATO_HIP(hipMemcpy(hc.data(), c, sizeof(double) * hc.size(), hipMemcpyDefault));
        for (int i = 0; i < P.n; ++i)
            for (int a = 0; a < 3; ++a)
                for (int k = 0; k < P.nv; ++k) o[(size_t)a * P.ldc + (size_t)i * P.nv + k] = hc[((size_t)i * 3 + a) * P.nv + k];
        MATO_HIP(hipMemcpy(B->arena + P.o_c, o.data(), sizeof(double) * o.size(), hipMemcpyHostToDevice));
    }
    S* dproj = nullptr;
    WorkItem* ditems = nullptr;
    ProblemDesc<S>* dd = nullptr;
    MATO_HIP(hipMalloc(&dproj, sizeof(S) * proj_i.size()));
    MATO_HIP(hipMemcpy(dproj, proj_i.data(), sizeof(S) * proj_i.size(), hipMemcpyHostToDevice));
    std::vector<WorkItem> items;
    for (const auto& w : B->hitems)
        if (w.prob == q) { WorkItem v = w; v.prob = 0; items.push_back(v); }
    ProblemDesc<S> D = B->hdesc[q];
    D.proj_in = dproj;
    MATO_HIP(hipMalloc(&ditems, sizeof(WorkItem) * items.size()));
    MATO_HIP(hipMalloc(&dd, sizeof(ProblemDesc<S>)));
    MATO_HIP(hipMemcpy(ditems, items.data(), sizeof(WorkItem) * items.size(), hipMemcpyHostToDevice));
    MATO_HIP(hipMemcpy(dd, &D, sizeof(D), hipMemcpyHostToDevice));
    int ctrl[4];
    MATO_HIP(hipMemcpy(ctrl, B->dctrl + 4 * q, sizeof(ctrl), hipMemcpyDeviceToHost));
    ctrl[1] = 0;
    ctrl[2] = 0;
    ctrl[3] = 1;
    MATO_HIP(hipMemcpy(B->dctrl + 4 * q, ctrl, sizeof(ctrl), hipMemcpyHostToDevice));
    MATO_HIP(launch_pairwise<S>(ditems, (int)items.size(), dd, kModeSetState, B->threads, B->lds, B->common_nv(), B->stream));
    MATO_HIP(launch_qbuild<S>(dd, 1, kModeInit, B->common_nv(), B->stream));
    if (c) MATO_HIP(launch_positions<S>(dd, 1, kModeInit, B->common_nv(), B->stream));
    MATO_HIP(hipStreamSynchronize(B->stream));
    dfree(dproj);
    dfree(ditems);
    dfree(dd);
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
        MATO_HIP(hipMemcpy(h.data(), B->arena + P.o_q, sizeof(double) * h.size(), hipMemcpyDeviceToHost));
        for (int i = 0; i < P.n; ++i)
            for (int a = 0; a < 3; ++a)
                for (int k = 0; k < P.nv; ++k)
                    o[((size_t)i * 3 + a) * P.nv + k] = h[(size_t)a * P.ldq + (size_t)i * P.nv + k];
        return copy_out(g, o.data(), sizeof(double) * o.size());
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

extern "C" void mato_solve_destroy(mato_solve s) { mato_batch_destroy(s); }
