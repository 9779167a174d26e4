// Offline plan (Remarks 1-2, Sec. III-B): trajectory basis of eq. (param), the
// KKT matrix of eq. (kkt_step_x) and its FP64 inverse, computed once per
// (n, T, basis, rho) and shared by every problem with those sizes.
//
// The inverse is taken on the device by Gauss-Jordan elimination with partial
// pivoting on the augmented matrix [K | I]; the c-rows [K11^{-1} | K12^{-1}] are
// then stored in the arithmetic of the per-iteration product (FP32, a three-term
// BF16 split, or FP64).
#include <cmath>
#include <cstdarg>
#include <cstring>

#include "common.h"

namespace mato {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}
const char* last_error() { return g_err; }

// ------------------------------------------------------------ basis (host) ---
static double binom(int n, int k) {
    if (k < 0 || k > n) return 0.0;
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

static double bern(int deg, int j, double tau) {
    if (j < 0 || j > deg) return 0.0;
    return binom(deg, j) * std::pow(tau, j) * std::pow(1.0 - tau, deg - j);
}

// P, P-dot, P-ddot (T x nv) of a degree nv-1 Bernstein basis on tau_k = k/(T-1),
// derivatives in physical time t = t_final * tau.
static void bernstein_basis(int nv, int T, double tf, std::vector<double>& P,
                            std::vector<double>& Pd, std::vector<double>& Pdd) {
    const int N = nv - 1;
    P.assign((size_t)T * nv, 0.0);
    Pd.assign((size_t)T * nv, 0.0);
    Pdd.assign((size_t)T * nv, 0.0);
    for (int k = 0; k < T; ++k) {
        const double tau = (double)k / (double)(T - 1);
        for (int j = 0; j < nv; ++j) {
            P[(size_t)k * nv + j] = bern(N, j, tau);
            Pd[(size_t)k * nv + j] = N * (bern(N - 1, j - 1, tau) - bern(N - 1, j, tau)) / tf;
            Pdd[(size_t)k * nv + j] = N * (N - 1) *
                (bern(N - 2, j - 2, tau) - 2.0 * bern(N - 2, j - 1, tau) + bern(N - 2, j, tau)) / (tf * tf);
        }
    }
}

static void gram(const std::vector<double>& X, int T, int nv, std::vector<double>& G) {
    G.assign((size_t)nv * nv, 0.0);
    for (int a = 0; a < nv; ++a)
        for (int b = 0; b < nv; ++b) {
            double s = 0.0;
            for (int k = 0; k < T; ++k) s += X[(size_t)k * nv + a] * X[(size_t)k * nv + b];
            G[(size_t)a * nv + b] = s;
        }
}

// ------------------------------------------------------ device kernels ---
// K of eq. (kkt_step_x), unknowns [c (agent-major); nu (agent-major)]:
//   H_(i,k),(j,l) = delta_ij Pdd^T Pdd[k][l] + rho (n delta_ij - 1) P^T P[k][l]
// (the collision Gram A_fc^T A_fc = (n I - 1 1^T) (x) P^T P), A_eq = I (x) A.
// Written into the left half of the augmented matrix W = [K | I].
__global__ void assemble_kkt(double* __restrict__ W, int n, int n_obs, int nv, int nb, double rho,
                             const double* __restrict__ PtP, const double* __restrict__ PddtPdd,
                             const double* __restrict__ A) {
    const int N = n * (nv + nb);
    const size_t total = (size_t)N * 2 * N;
    const int nc = n * nv;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int r = (int)(e / (2 * N)), c = (int)(e % (2 * N));
        double v = 0.0;
        if (c >= N) {
            v = (c - N == r) ? 1.0 : 0.0;
        } else if (r < nc && c < nc) {
            const int i = r / nv, k = r % nv, j = c / nv, l = c % nv;
            v = rho * ((i == j ? n + n_obs : 0) - 1) * PtP[k * nv + l];
            if (i == j) v += PddtPdd[k * nv + l];
        } else if (r < nc && c >= nc) {
            const int i = r / nv, k = r % nv, j = (c - nc) / nb, b = (c - nc) % nb;
            v = (i == j) ? A[b * nv + k] : 0.0;
        } else if (r >= nc && c < nc) {
            const int i = (r - nc) / nb, b = (r - nc) % nb, j = c / nv, l = c % nv;
            v = (i == j) ? A[b * nv + l] : 0.0;
        }
        W[e] = v;
    }
}

// Augmented [[Pdd^T Pdd + sigma P^T P, A^T], [A, 0] | I] of one agent and axis
// ((nv + nb) x 2(nv + nb)), matrix blockIdx.y of a stack with stride ms and
// shift sigma[blockIdx.y].
__global__ void assemble_agent_kkt(double* __restrict__ W, int nv, int nb, const double* __restrict__ sigma,
                                   size_t ms, const double* __restrict__ PtP,
                                   const double* __restrict__ PddtPdd, const double* __restrict__ A) {
    const int N = nv + nb;
    double* Wm = W + ms * blockIdx.y;
    const double sg = sigma[blockIdx.y];
    for (int e = threadIdx.x; e < N * 2 * N; e += blockDim.x) {
        const int r = e / (2 * N), c = e % (2 * N);
        double v = 0.0;
        if (c >= N) v = (c - N == r) ? 1.0 : 0.0;
        else if (r < nv && c < nv) v = PddtPdd[r * nv + c] + sg * PtP[r * nv + c];
        else if (r < nv) v = A[(c - nv) * nv + r];
        else if (c < nv) v = A[(r - nv) * nv + c];
        Wm[e] = v;
    }
}

// Column absolute sums of the left half (for ||K||_1) or of the right half; matrix
// blockIdx.y of a stack with stride ms.
__global__ void column_abs_sums(const double* __restrict__ W, int N, int off, size_t ms, double* __restrict__ out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= N) return;
    const double* Wm = W + ms * blockIdx.y;
    double s = 0.0;
    for (int r = 0; r < N; ++r) s += fabs(Wm[(size_t)r * 2 * N + off + c]);
    out[(size_t)blockIdx.y * N + c] = s;
}

// Gauss-Jordan step k, part 1 (one workgroup per matrix of a stack with stride ms):
// pivot search over rows >= k (largest |W[r][k]|, lowest r on ties), row swap,
// pivot-row scaling, and a copy of column k (the elimination factors) into f.
__global__ __launch_bounds__(1024) void gj_pivot(double* __restrict__ Wst, int N, int k, size_t ms,
                                                 double* __restrict__ fst, int* __restrict__ flags) {
    __shared__ double sv[1024];
    __shared__ int si[1024];
    __shared__ double s_pv;
    double* W = Wst + ms * blockIdx.x;
    double* f = fst + (size_t)N * blockIdx.x;
    const int tid = threadIdx.x;
    const size_t ld = 2 * (size_t)N;
    double best = -1.0;
    int bi = N;
    for (int r = k + tid; r < N; r += blockDim.x) {
        const double v = fabs(W[r * ld + k]);
        if (v > best) { best = v; bi = r; }
    }
    sv[tid] = best;
    si[tid] = bi;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (tid < s) {
            const double v2 = sv[tid + s];
            const int i2 = si[tid + s];
            if (v2 > sv[tid] || (v2 == sv[tid] && i2 < si[tid])) { sv[tid] = v2; si[tid] = i2; }
        }
        __syncthreads();
    }
    const int p = si[0];
    if (tid == 0) {
        s_pv = (p < N) ? W[p * ld + k] : 0.0;
        if (!(fabs(s_pv) > 1e-300)) flags[blockIdx.x] = 1;
    }
    __syncthreads();                       // the pivot value is read before any row moves
    const double pv = s_pv;
    if (p != k && p < N) {
        for (size_t c = tid; c < ld; c += blockDim.x) {
            const double t = W[(size_t)k * ld + c];
            W[(size_t)k * ld + c] = W[(size_t)p * ld + c];
            W[(size_t)p * ld + c] = t;
        }
    }
    __syncthreads();
    const double inv = (fabs(pv) > 1e-300) ? 1.0 / pv : 1.0;
    for (size_t c = tid; c < ld; c += blockDim.x) W[(size_t)k * ld + c] *= inv;
    __syncthreads();
    for (int r = tid; r < N; r += blockDim.x) f[r] = (r == k) ? 0.0 : W[(size_t)r * ld + k];
}

// Gauss-Jordan step k, part 2: W[r][c] -= f[r] W[k][c] for every r != k and c >= k,
// matrix blockIdx.y of the stack.
__global__ void gj_eliminate(double* __restrict__ Wst, int N, int k, size_t ms, const double* __restrict__ fst) {
    double* W = Wst + ms * blockIdx.y;
    const double* f = fst + (size_t)N * blockIdx.y;
    const size_t ld = 2 * (size_t)N;
    const int ncols = 2 * N - k;
    const size_t total = (size_t)N * ncols;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int r = (int)(e / ncols), c = k + (int)(e % ncols);
        const double fr = f[r];
        if (fr != 0.0) W[(size_t)r * ld + c] -= fr * W[(size_t)k * ld + c];
    }
}

// Right half of W -> dense N x N inverse.
__global__ void extract_inverse(const double* __restrict__ W, int N, double* __restrict__ inv) {
    const size_t total = (size_t)N * N;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int r = (int)(e / N), c = (int)(e % N);
        inv[e] = W[(size_t)r * 2 * N + N + c];
    }
}

__device__ inline unsigned short bf16_bits_rne(float x) {
    unsigned int u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ inline float bf16_bits_to_float(unsigned short h) {
    return __uint_as_float(((unsigned int)h) << 16);
}

// GEMM operand: the leading M x M block of K^{-1} (row stride N), zero-padded to Mp x ldk.
// kind 0: fp32; 1: three bf16 terms of the FP64 value, hi = bf16(x), mid = bf16(x - hi),
// lo = bf16(x - hi - mid) (differences in FP64: 24 significant bits in all); 2: fp64.
__device__ inline unsigned short bf16_bits_rne_f64(double x) {
    return bf16_bits_rne((float)x);   // a double within FP32 range rounds to bf16 through fp32
}
__global__ void extract_crows(const double* __restrict__ inv, int N, int M, int Mp, int ldk,
                              int kind, void* __restrict__ hi, void* __restrict__ lo) {
    const size_t total = (size_t)Mp * ldk;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int r = (int)(e / ldk), c = (int)(e % ldk);
        const double v = (r < M && c < M) ? inv[(size_t)r * N + c] : 0.0;
        if (kind == 0) {
            ((float*)hi)[e] = (float)v;
        } else if (kind == 1) {
            const unsigned short h = bf16_bits_rne_f64(v);
            const double r1 = v - (double)bf16_bits_to_float(h);
            const unsigned short m = bf16_bits_rne_f64(r1);
            const double r2 = r1 - (double)bf16_bits_to_float(m);
            ((unsigned short*)hi)[e] = h;
            ((unsigned short*)lo)[e] = m;
            ((unsigned short*)lo)[total + e] = bf16_bits_rne_f64(r2);
        } else {
            ((double*)hi)[e] = v;
        }
    }
}

static int grid_for(size_t total, int block) {
    size_t g = (total + block - 1) / block;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (int)g;
}

// Inverts `count` N x N matrices assembled into the left halves of a stack of
// augmented matrices W (stride N x 2N), all in the same launches; inverse m goes to
// inv[m].  Returns SINGULAR on a zero pivot; writes ||K||_1 ||K^{-1}||_1 to cond[m].
static mato_status gauss_jordan(double* W, int N, int count, double* const* inv, double* cond, hipStream_t st) {
    const size_t ms = (size_t)N * 2 * N;
    DevBuf<double> fb, csb;
    DevBuf<int> flagb;
    MATO_TRY(fb.alloc((size_t)N * count));
    MATO_TRY(csb.alloc((size_t)N * count));
    MATO_TRY(flagb.alloc(count));
    double* f = fb.p;
    double* cs = csb.p;
    int* flag = flagb.p;
    MATO_HIP(hipMemsetAsync(flag, 0, sizeof(int) * count, st));
    std::vector<double> h((size_t)N * count), norm1(count, 0.0);
    column_abs_sums<<<dim3((N + 255) / 256, count), 256, 0, st>>>(W, N, 0, ms, cs);
    MATO_HIP(hipMemcpyAsync(h.data(), cs, sizeof(double) * h.size(), hipMemcpyDeviceToHost, st));
    MATO_HIP(hipStreamSynchronize(st));
    for (int m = 0; m < count; ++m)
        for (int c = 0; c < N; ++c) norm1[m] = std::max(norm1[m], h[(size_t)m * N + c]);
    for (int k = 0; k < N; ++k) {
        gj_pivot<<<count, 1024, 0, st>>>(W, N, k, ms, f, flag);
        const size_t work = (size_t)N * (2 * N - k);
        gj_eliminate<<<dim3(grid_for(work, 256), count), 256, 0, st>>>(W, N, k, ms, f);
    }
    MATO_HIP(hipGetLastError());
    column_abs_sums<<<dim3((N + 255) / 256, count), 256, 0, st>>>(W, N, N, ms, cs);
    std::vector<int> hflag(count, 0);
    MATO_HIP(hipMemcpyAsync(h.data(), cs, sizeof(double) * h.size(), hipMemcpyDeviceToHost, st));
    MATO_HIP(hipMemcpyAsync(hflag.data(), flag, sizeof(int) * count, hipMemcpyDeviceToHost, st));
    for (int m = 0; m < count; ++m)
        extract_inverse<<<grid_for((size_t)N * N, 256), 256, 0, st>>>(W + ms * m, N, inv[m]);
    MATO_HIP(hipStreamSynchronize(st));
    mato_status status = MATO_OK;
    for (int m = 0; m < count; ++m) {
        double ninv = 0.0;
        for (int c = 0; c < N; ++c) ninv = std::max(ninv, h[(size_t)m * N + c]);
        cond[m] = norm1[m] * ninv;
        if (hflag[m] || !std::isfinite(cond[m]) || cond[m] > 1e14) {
            set_error("KKT matrix is singular or too ill-conditioned (cond estimate %.3e)", cond[m]);
            status = MATO_ERR_SINGULAR;
        }
    }
    return status;
}

template <typename T>
static mato_status upload(T** dst, const std::vector<T>& src, size_t* bytes) {
    MATO_TRY(dalloc(dst, src.size()));
    MATO_HIP(hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice));
    *bytes += sizeof(T) * src.size();
    return MATO_OK;
}

// Builds plans that share n, T, basis, a, b and precision and differ in rho; their
// KKT matrices are inverted together.
static mato_status plans_build(std::vector<mato_plan>& ps) {
    mato_plan p0 = ps[0];
    const int n = p0->n, nv = p0->nv, nb = p0->nb, T = p0->T, cnt = (int)ps.size();
    hipStream_t st = p0->stream;
    bernstein_basis(nv, T, p0->t_final, p0->P, p0->Pd, p0->Pdd);
    gram(p0->P, T, nv, p0->PtP);
    gram(p0->Pdd, T, nv, p0->PddtPdd);
    p0->A.assign((size_t)nb * nv, 0.0);
    for (int j = 0; j < nv; ++j) {
        p0->A[0 * nv + j] = p0->P[j];
        p0->A[1 * nv + j] = p0->Pd[j];
        p0->A[2 * nv + j] = p0->Pdd[j];
        p0->A[3 * nv + j] = p0->P[(size_t)(T - 1) * nv + j];
        p0->A[4 * nv + j] = p0->Pd[(size_t)(T - 1) * nv + j];
        p0->A[5 * nv + j] = p0->Pdd[(size_t)(T - 1) * nv + j];
    }
    // Internal order of the collision rows (the layout of the multipliers on the device).
    // FP64 plans: the canonical order, pairs in the row order of A_fc, then agent-obstacle
    // rows agent-major.  FP32 / BF16 plans: the pairs in the rounds of a round-robin
    // tournament (circle method: with m = n rounded up to even, round r pairs agent m - 1
    // with r and (r + k) mod (m - 1) with (r - k) mod (m - 1), k = 1 .. m/2 - 1; pairs with
    // the ghost agent of an odd n are left out), so that neighbouring rows, which
    // neighbouring lanes of a wavefront process, involve different agents; then the
    // obstacle rows obstacle-major.  Every entry keeps its smaller agent first (delta =
    // X_i - X_j, i < j, whatever the order of the rows).
    std::vector<unsigned> pairs;
    auto add = [&](int i, int j) {
        if (i > j) std::swap(i, j);
        pairs.push_back((unsigned)i | ((unsigned)j << 16));
    };
    if (p0->precision == MATO_FP64) {
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) add(i, j);
        for (int i = 0; i < n; ++i)
            for (int o = 0; o < p0->n_obs; ++o) add(i, n + o);
    } else {
        const int m = n + (n & 1);
        for (int r = 0; r < m - 1; ++r) {
            if (m - 1 < n) add(m - 1, r);             // agent m - 1 exists when n is even
            for (int k = 1; k < m / 2; ++k) {
                const int a = (r + k) % (m - 1), b = (r - k + (m - 1)) % (m - 1);
                if (a < n && b < n) add(a, b);
            }
        }
        for (int o = 0; o < p0->n_obs; ++o)
            for (int i = 0; i < n; ++i) add(i, n + o);
    }
    for (auto p : ps) {
        if (p != p0) {
            p->P = p0->P; p->Pd = p0->Pd; p->Pdd = p0->Pdd;
            p->PtP = p0->PtP; p->PddtPdd = p0->PddtPdd; p->A = p0->A;
        }
        MATO_TRY(upload(&p->dP, p->P, &p->bytes));
        MATO_TRY(upload(&p->dPdd, p->Pdd, &p->bytes));
        MATO_TRY(upload(&p->dPtP, p->PtP, &p->bytes));
        MATO_TRY(upload(&p->dPddtPdd, p->PddtPdd, &p->bytes));
        MATO_TRY(upload(&p->dA, p->A, &p->bytes));
        MATO_TRY(upload(&p->dPairs, pairs, &p->bytes));
        p->pairs = pairs;
    }

    // Per-agent KKT matrices K_sigma = [[Pdd^T Pdd + sigma P^T P, A^T], [A, 0]].  K_0 is the
    // boundary-only minimum-acceleration problem (initialisation).  With the structured
    // solve also, for every rho, the mean block K_{rho n_obs} and the deviation block
    // K_{rho (n + n_obs)}: A_fc^T A_fc = ((n + n_obs) I - 1 1^T) (x) P^T P, whose eigenvalues
    // are n_obs on the agent mean and n + n_obs on every deviation from it, so
    //     K^{-1} = (1 1^T / n) (x) K_mean^{-1} + (I - 1 1^T / n) (x) K_dev^{-1}
    // in per-agent ordering, and c_i = K_mean^{-1} [g_mean; b_mean] + K_dev^{-1} [g_i - g_mean; b_i - b_mean].
    const bool structured = p0->solve == MATO_SOLVE_STRUCTURED;
    const int n_obs = p0->n_obs;
    {
        const int N0 = nv + nb, m0 = structured ? 2 * cnt + 1 : 1;
        const size_t ms0 = (size_t)N0 * 2 * N0;
        std::vector<double> sig(m0, 0.0);
        for (int m = 0; 2 * m + 2 < m0; ++m) {
            sig[2 * m + 1] = ps[m]->rho * n_obs;
            sig[2 * m + 2] = ps[m]->rho * (n + n_obs);
        }
        DevBuf<double> W0b, inv0b, dsigb;
        MATO_TRY(W0b.alloc(ms0 * m0));
        MATO_TRY(inv0b.alloc((size_t)N0 * N0 * m0));
        MATO_TRY(dsigb.alloc(m0));
        double *W0 = W0b.p, *inv0 = inv0b.p, *dsig = dsigb.p;
        MATO_HIP(hipMemcpy(dsig, sig.data(), sizeof(double) * m0, hipMemcpyHostToDevice));
        assemble_agent_kkt<<<dim3(1, m0), 256, 0, st>>>(W0, nv, nb, dsig, ms0, p0->dPtP, p0->dPddtPdd, p0->dA);
        std::vector<double*> invs(m0);
        for (int m = 0; m < m0; ++m) invs[m] = inv0 + (size_t)N0 * N0 * m;
        std::vector<double> conds(m0, 0.0);
        mato_status s = gauss_jordan(W0, N0, m0, invs.data(), conds.data(), st);
        std::vector<double> h((size_t)N0 * N0 * m0);
        if (s != MATO_OK) return s;
        MATO_HIP(hipMemcpy(h.data(), inv0, sizeof(double) * h.size(), hipMemcpyDeviceToHost));
        p0->K0inv_c.assign((size_t)nv * nb, 0.0);
        for (int r = 0; r < nv; ++r)
            for (int b = 0; b < nb; ++b) p0->K0inv_c[(size_t)r * nb + b] = h[(size_t)r * N0 + nv + b];
        for (auto p : ps) {
            if (p != p0) p->K0inv_c = p0->K0inv_c;
            MATO_TRY(upload(&p->dK0c, p->K0inv_c, &p->bytes));
        }
        if (structured) {
            for (int m = 0; m < cnt; ++m) {
                mato_plan p = ps[m];
                const double* K0i = h.data() + (size_t)N0 * N0 * (2 * m + 1);
                const double* Kni = h.data() + (size_t)N0 * N0 * (2 * m + 2);
                p->Ks0.assign(K0i, K0i + (size_t)N0 * N0);
                p->Ksn.assign(Kni, Kni + (size_t)N0 * N0);
                p->cond = std::max(conds[2 * m + 1], conds[2 * m + 2]);
                std::vector<double> S((size_t)2 * nv * nv + (size_t)2 * nv * nb);
                double* M1 = S.data();
                double* M2 = M1 + nv * nv;
                double* E0 = M2 + nv * nv;
                double* En = E0 + nv * nb;
                for (int r = 0; r < nv; ++r) {
                    for (int c = 0; c < nv; ++c) {
                        M1[r * nv + c] = Kni[(size_t)r * N0 + c];
                        M2[r * nv + c] = K0i[(size_t)r * N0 + c] - Kni[(size_t)r * N0 + c];
                    }
                    for (int b = 0; b < nb; ++b) {
                        E0[r * nb + b] = K0i[(size_t)r * N0 + nv + b];
                        En[r * nb + b] = Kni[(size_t)r * N0 + nv + b];
                    }
                }
                MATO_TRY(upload(&p->dS, S, &p->bytes));
            }
            MATO_HIP(hipStreamSynchronize(st));
            return MATO_OK;
        }
    }

    // KKT matrices of eq. (kkt_step_x), one per rho, inverted together
    const int N = n * (nv + nb), M = n * nv;
    const size_t ms = (size_t)N * 2 * N;
    DevBuf<double> Wb;
    MATO_TRY(Wb.alloc(ms * cnt));
    double* W = Wb.p;
    std::vector<double*> invs(cnt);
    std::vector<double> conds(cnt, 0.0);
    for (int m = 0; m < cnt; ++m) {
        MATO_TRY(dalloc(&ps[m]->dKinv, (size_t)N * N));
        ps[m]->bytes += sizeof(double) * (size_t)N * N;
        invs[m] = ps[m]->dKinv;
        assemble_kkt<<<grid_for(ms, 256), 256, 0, st>>>(W + ms * m, n, n_obs, nv, nb, ps[m]->rho, ps[m]->dPtP,
                                                        ps[m]->dPddtPdd, ps[m]->dA);
    }
    mato_status s = gauss_jordan(W, N, cnt, invs.data(), conds.data(), st);
    for (int m = 0; m < cnt; ++m) ps[m]->cond = conds[m];
    if (s != MATO_OK) return s;

    // GEMM operand: the (11n x 11n) block K11^{-1}; the K12^{-1} b_eq part is formed once
    // per problem in FP64
    const int Mp = round_up(M, 64);
    const int ldk = round_up(M, 32);
    const size_t elems = (size_t)Mp * ldk;
    int kind = 0;
    size_t esz = sizeof(float);
    if (p0->precision == MATO_BF16_REFINED) { kind = 1; esz = 2; }
    if (p0->precision == MATO_FP64) { kind = 2; esz = sizeof(double); }
    for (auto p : ps) {
        p->ldk = ldk;
        MATO_TRY(dalloc((char**)&p->dAhi, esz * elems));
        p->bytes += esz * elems;
        if (kind == 1) {
            MATO_TRY(dalloc((char**)&p->dAlo, 2 * esz * elems));
            p->bytes += 2 * esz * elems;
        }
        extract_crows<<<grid_for(elems, 256), 256, 0, st>>>(p->dKinv, N, M, Mp, ldk, kind, p->dAhi, p->dAlo);
    }
    MATO_HIP(hipGetLastError());
    MATO_HIP(hipStreamSynchronize(st));
    return MATO_OK;
}

}  // namespace mato

using namespace mato;

extern "C" const char* mato_last_error(void) { return mato::last_error(); }
extern "C" const char* mato_version(void) { return "mato 0.1 (gfx950)"; }

extern "C" void mato_plan_destroy(mato_plan p) {
    if (!p) return;
    dfree(p->dKinv);
    dfree(p->dP);
    dfree(p->dPdd);
    dfree(p->dPtP);
    dfree(p->dPddtPdd);
    dfree(p->dA);
    dfree(p->dK0c);
    dfree(p->dPairs);
    dfree(p->dAhi);
    dfree(p->dAlo);
    dfree(p->dS);
    delete p;
}

static mato_status check_plan_args(int32_t n, int32_t T, const mato_basis* basis, double a, double b,
                                   int32_t precision) {
    if (!basis) { set_error("null argument"); return MATO_ERR_INVALID_ARG; }
    if (basis->kind != MATO_BASIS_BERNSTEIN) { set_error("unknown basis kind %d", basis->kind); return MATO_ERR_INVALID_ARG; }
    if (basis->n_coef < 6 || basis->n_coef > kMaxCoef) { set_error("n_coef %d outside 6..%d", basis->n_coef, kMaxCoef); return MATO_ERR_INVALID_ARG; }
    if (n < 2) { set_error("n = %d < 2", n); return MATO_ERR_INVALID_ARG; }
    if (n > MATO_MAX_AGENTS) { set_error("n = %d > %d", n, MATO_MAX_AGENTS); return MATO_ERR_UNSUPPORTED; }
    if (T < basis->n_coef) { set_error("T = %d < n_coef", T); return MATO_ERR_INVALID_ARG; }
    if (!(a > 0) || !(b > 0) || !(basis->t_final > 0) || !std::isfinite(a) || !std::isfinite(b) ||
        !std::isfinite(basis->t_final)) {
        set_error("a, b and t_final must be finite and > 0");
        return MATO_ERR_INVALID_ARG;
    }
    if (precision != MATO_FP64 && precision != MATO_FP32 && precision != MATO_BF16_REFINED) {
        set_error("unknown precision %d", precision);
        return MATO_ERR_INVALID_ARG;
    }
    return MATO_OK;
}

extern "C" mato_status mato_plan_create_ex(const mato_plan_desc* d, const double* rhos, int32_t count,
                                           void* hip_stream, mato_plan* out) {
    if (!d || !out || !rhos || count < 1) { set_error("null argument or count < 1"); return MATO_ERR_INVALID_ARG; }
    for (int m = 0; m < count; ++m) out[m] = nullptr;
    MATO_TRY(check_plan_args(d->n, d->T, &d->basis, d->a, d->b, d->precision));
    if (d->n_obs < 0 || d->n_obs > MATO_MAX_OBSTACLES) {
        set_error("n_obs = %d outside 0..%d", d->n_obs, MATO_MAX_OBSTACLES);
        return MATO_ERR_INVALID_ARG;
    }
    if (d->solve != MATO_SOLVE_DENSE && d->solve != MATO_SOLVE_STRUCTURED) {
        set_error("unknown solve kind %d", d->solve);
        return MATO_ERR_INVALID_ARG;
    }
    if (d->solve == MATO_SOLVE_STRUCTURED && d->precision == MATO_BF16_REFINED) {
        set_error("the structured solve has no BF16 product: use MATO_FP32 or MATO_FP64");
        return MATO_ERR_INVALID_ARG;
    }
    for (int m = 0; m < count; ++m)
        if (!(rhos[m] > 0) || !std::isfinite(rhos[m])) { set_error("rho must be finite and > 0"); return MATO_ERR_INVALID_ARG; }
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) {
        set_error("no HIP device");
        return MATO_ERR_HIP;
    }
    std::vector<mato_plan> ps;
    for (int m = 0; m < count; ++m) {
        mato_plan p = new mato_plan_s();
        p->n = d->n; p->T = d->T; p->nv = d->basis.n_coef; p->nb = kNb; p->precision = d->precision;
        p->t_final = d->basis.t_final; p->a = d->a; p->b = d->b; p->rho = rhos[m]; p->cond = 0.0;
        p->solve = d->solve;
        p->n_obs = d->n_obs;
        p->stream = (hipStream_t)hip_stream;
        p->device = device;
        ps.push_back(p);
    }
    mato_status s = plans_build(ps);
    if (s != MATO_OK) {
        for (auto p : ps) mato_plan_destroy(p);
        return s;
    }
    for (int m = 0; m < count; ++m) out[m] = ps[m];
    return MATO_OK;
}

extern "C" mato_status mato_plan_create_many(int32_t n, int32_t T, const mato_basis* basis, double a, double b,
                                             const double* rhos, int32_t count, int32_t precision,
                                             void* hip_stream, mato_plan* out) {
    if (!basis) { set_error("null argument"); return MATO_ERR_INVALID_ARG; }
    mato_plan_desc d;
    d.n = n; d.n_obs = 0; d.T = T; d.basis = *basis; d.a = a; d.b = b; d.precision = precision;
    d.solve = MATO_SOLVE_DENSE;
    return mato_plan_create_ex(&d, rhos, count, hip_stream, out);
}

extern "C" mato_status mato_plan_create(int32_t n, int32_t T, const mato_basis* basis, double a,
                                        double b, double rho, int32_t precision, void* hip_stream,
                                        mato_plan* out) {
    if (!out || !basis) { set_error("null argument"); return MATO_ERR_INVALID_ARG; }
    *out = nullptr;
    MATO_TRY(check_plan_args(n, T, basis, a, b, precision));
    if (!(rho > 0) || !std::isfinite(rho)) { set_error("a, b, rho and t_final must be finite and > 0"); return MATO_ERR_INVALID_ARG; }
    return mato_plan_create_many(n, T, basis, a, b, &rho, 1, precision, hip_stream, out);
}

extern "C" mato_status mato_plan_info(mato_plan p, int32_t* n, int32_t* T, int32_t* n_coef,
                                      int32_t* precision, double* cond) {
    if (!p) { set_error("null plan"); return MATO_ERR_INVALID_ARG; }
    if (n) *n = p->n;
    if (T) *T = p->T;
    if (n_coef) *n_coef = p->nv;
    if (precision) *precision = p->precision;
    if (cond) *cond = p->cond;
    return MATO_OK;
}

extern "C" mato_status mato_plan_inverse(mato_plan p, double* kinv) {
    if (!p || !kinv) { set_error("null argument"); return MATO_ERR_INVALID_ARG; }
    const int n = p->n, nv = p->nv, nb = p->nb, N0 = nv + nb;
    const size_t N = (size_t)n * N0;
    if (p->solve == MATO_SOLVE_STRUCTURED) {
        // the two-block form, expanded into the ordering [c (agent-major); nu (agent-major)]
        std::vector<double> h(N * N);
        auto split = [&](size_t R, int* agent, int* local) {
            if (R < (size_t)n * nv) { *agent = (int)(R / nv); *local = (int)(R % nv); }
            else { const size_t u = R - (size_t)n * nv; *agent = (int)(u / nb); *local = nv + (int)(u % nb); }
        };
        for (size_t R = 0; R < N; ++R) {
            int i, kr;
            split(R, &i, &kr);
            for (size_t C = 0; C < N; ++C) {
                int j, kc;
                split(C, &j, &kc);
                const double e0 = p->Ks0[(size_t)kr * N0 + kc], en = p->Ksn[(size_t)kr * N0 + kc];   // mean, deviation
                h[R * N + C] = e0 / n + ((i == j ? 1.0 : 0.0) - 1.0 / n) * en;
            }
        }
        MATO_HIP(hipMemcpyAsync(kinv, h.data(), sizeof(double) * N * N, hipMemcpyDefault, p->stream));
    } else {
        MATO_HIP(hipMemcpyAsync(kinv, p->dKinv, sizeof(double) * N * N, hipMemcpyDefault, p->stream));
    }
    MATO_HIP(hipStreamSynchronize(p->stream));
    return MATO_OK;
}

extern "C" mato_status mato_plan_describe(mato_plan p, mato_plan_desc* d, double* rho) {
    if (!p) { set_error("null plan"); return MATO_ERR_INVALID_ARG; }
    if (d) {
        d->n = p->n; d->n_obs = p->n_obs; d->T = p->T;
        d->basis.kind = MATO_BASIS_BERNSTEIN; d->basis.n_coef = p->nv; d->basis.t_final = p->t_final;
        d->a = p->a; d->b = p->b; d->precision = p->precision; d->solve = p->solve;
    }
    if (rho) *rho = p->rho;
    return MATO_OK;
}
