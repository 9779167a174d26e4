// Internal declarations of libmato: device-side problem descriptors, work items,
// plan and batch handles, error plumbing.  Host and device code of every
// translation unit include this file; nothing here is part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/mato.h"

namespace mato {

constexpr int kAxes = 3;        // x, y, z
constexpr int kNb = 6;          // boundary rows per agent and axis: p, v, a at both ends
constexpr int kMaxCoef = 16;
constexpr int kHistCap = 4096;  // per-problem iteration history kept on the device
constexpr int kMaxRefine = 4;
constexpr int kMaxStages = MATO_MAX_STAGES;
constexpr int kObs = 8;         // obstacle table entry: x, y, z, 1/l_xy^2, 1/l_z^2, l_z, 0, 0 (scalar S)
constexpr int kCtrl = 8;        // control words per problem:
                                // [0] iterations, [1] stopped, [2] non-finite, [3] active, [4] converged

// ---------------------------------------------------------------- errors ---
void set_error(const char* fmt, ...);
const char* last_error();

#define MATO_HIP(call)                                                          \
    do {                                                                        \
        hipError_t e_ = (call);                                                 \
        if (e_ != hipSuccess) {                                                 \
            ::mato::set_error("%s failed: %s (%s:%d)", #call,                   \
                              hipGetErrorString(e_), __FILE__, __LINE__);       \
            return MATO_ERR_HIP;                                                \
        }                                                                       \
    } while (0)

#define MATO_TRY(call)                                                          \
    do {                                                                        \
        mato_status s_ = (call);                                                \
        if (s_ < 0) return s_;                                                  \
    } while (0)

inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

inline void dfree(void* p) {
    if (p) (void)hipFree(p);
}

// Device allocation with the library's error convention (OUT_OF_MEMORY, message set).
template <typename T>
inline mato_status dalloc(T** p, size_t count) {
    *p = nullptr;
    if (hipMalloc(p, sizeof(T) * std::max<size_t>(count, 1)) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        set_error("device allocation of %zu bytes failed", sizeof(T) * count);
        return MATO_ERR_OUT_OF_MEMORY;
    }
    return MATO_OK;
}

// Scratch device buffer freed when it goes out of scope (every return path).
template <typename T>
struct DevBuf {
    T* p = nullptr;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { dfree(p); }
    mato_status alloc(size_t count) { return dalloc(&p, count); }
};

// Pair p = (i, j), i < j, in the row order of A_fc: p(i, j) = i n - i(i+1)/2 + j - i - 1.
__host__ __device__ inline int row_offset(int i, int n) { return i * n - i * (i + 1) / 2; }

// Canonical collision row (agent pairs in the row order of A_fc, then agent-obstacle rows
// agent-major) of a pair-table entry i | j << 16 (partner j >= n: obstacle j - n).
__host__ __device__ inline int canonical_row(unsigned code, int n, int n_obs) {
    const int i = (int)(code & 0xffffu), j = (int)(code >> 16);
    if (j < n) return row_offset(i, n) + j - i - 1;
    return n * (n - 1) / 2 + i * n_obs + (j - n);
}

// -------------------------------------------------------- device descriptors ---
// One problem as the kernels see it.  S is the pairwise-stage scalar (float or
// double); coefficients, linear term, residuals and the boundary data are FP64.
template <typename S>
struct ProblemDesc {
    int n, np, T, nv;           // agents, collision rows (pairs, then agent-obstacle pairs), instants, coefficients
    int n_obs;                  // static obstacles
    int ldq;                    // stride of one axis of q / r: >= 17n, padded
    int ldc;                    // stride of one axis of c: >= 11n
    int nslab;                  // pairwise work items of this problem (residual partials)
    int hist_cap;
    double a, b;                // l_xy, l_z
    double rho;
    S ia2, ib2;                 // 1/l_xy^2, 1/l_z^2
    S lz, srho, sirho;          // l_z, rho, 1/rho in S
    const double* P;            // [T][nv] FP64 basis
    const double* Pdd;          // [T][nv]
    const double* PtP;          // [nv][nv]
    const double* PddtPdd;      // [nv][nv]
    const double* A;            // [6][nv] boundary rows
    const unsigned* pairs;      // [np] row p -> i | j << 16 (j >= n: obstacle j - n)
    const S* obs;               // [n_obs][kObs] obstacle table
    const double* smat;         // structured solve operands of the plan (nullptr: dense inverse)
    S* lam;                     // [T][3][np] multipliers
    S* ssum;                    // [T][3][n]  per-agent sums of b_fc (A_fc^T b before P^T); FP32: their corrections C
    S* X;                       // [T][3][n]  positions P c of the current coefficients
    unsigned* lflag;            // [T][ceil(np/64)] FP32: 0 when the 64-row group's multipliers are all +0
    double* c;                  // [3][ldc]   coefficients (agent-major per axis)
    double* ceq;                // [3][ldc]   c_eq = K12^{-1} b_eq (boundary part of the product)
    double* q;                  // [3][ldq]   [rho A_fc^T b_fc ; b_eq]  (eq. kkt_step_x)
    double* r;                  // [3][ldq]   refinement residual g - H c (first 11n entries)
    float* qf;                  // [3][ldq]   q rounded to FP32 (inverse-product operand)
    float* rf;                  // [3][ldq]   r rounded to FP32
    double* part;               // [nslab][4] residual partials: max|f|^2, sum|f|^2
    double* hist;               // [hist_cap][3] r_max, r_rms, cost
    int* ctrl;                  // kCtrl words, see above
    double tol;                 // convergence threshold on r_max (<= 0: none)
    int iter_cap;               // stop after this many iterations (<= 0: none)
    int shifted;                // 1: project delta + lambda/rho instead of delta
    int switch_at;              // > 0: iteration count at which the next rho stage starts
    double rho_next;            // rho of that stage (b_fc and g of the last iteration before it)
    S sirho_next;               // 1 / rho_next in S
    // optional parity outputs (nullptr = off)
    S* dbg_proj;                // [T][3][np] d e
    S* dbg_d;                   // [T][np]
    const S* proj_in;           // set-state input [T][3][np]
};

// Workgroups of a launch are dealt to the device's 8 accelerator dies (XCDs), each with
// its own L2, round-robin by workgroup index (blockIdx mod 8).  xcd_tile maps workgroup b
// to list entry start(b mod 8) + b / 8, so each die works through one contiguous run of
// the list (a bijection for any list length): neighbouring entries that read the same
// data fetch it into one L2 instead of eight.
constexpr int kXcds = 8;
__device__ inline int xcd_tile(int b, int ntiles) {
    const int q = ntiles / kXcds, r = ntiles % kXcds;
    const int x = b % kXcds, j = b / kXcds;
    return x * q + min(x, r) + j;
}

struct WorkItem {               // one pairwise workgroup: instants [t0, t0 + tc) of problem `prob`
    int prob, t0, tc, slab;
};

struct GemmTile {               // one 64-row output tile (64 or 48 columns) of one same-plan group
    int group, m0, col0, pad;
};

struct GemmGroup {              // problems sharing one plan: C[:, col] = c_eq + K11^{-1} B[:, col]
    const void* Ahi;            // [Mp][ldk] K11^{-1} (fp32 / bf16 hi / fp64), zero padded
    const void* Amid;           // bf16 middle term (BF16 split only)
    const void* Alo;            // bf16 low term (BF16 split only)
    int M, K, ldk;              // 11n, 11n, padded row stride of A (multiple of 32)
    int ncols;                  // 3 x members
    int first_col;              // offset into the column table
};

struct GemmCol {                // one right-hand side: problem axis
    const double* b;            // K entries (q or r), FP64
    const float* bf;            // the same rounded to FP32 (FP32 / BF16 products)
    double* c;                  // M entries
    const double* ceq;          // M entries, added when not accumulating
    const int* ctrl;            // problem control word (skip when converged / inactive)
};

enum PairMode { kModeIter = 0, kModeInit = 1, kModeSetState = 2 };

}  // namespace mato

// ------------------------------------------------------------------ handles ---
struct mato_plan_s {
    int n, T, nv, nb, precision, device;
    int n_obs = 0;
    double t_final, a, b, rho, cond;
    hipStream_t stream;
    std::vector<double> P, Pd, Pdd, PtP, PddtPdd, A, K0inv_c;   // host FP64
    double* dKinv = nullptr;     // (17n)^2 FP64 inverse
    double* dP = nullptr;        // [T][nv]
    double* dPdd = nullptr;
    double* dPtP = nullptr;
    double* dPddtPdd = nullptr;
    double* dA = nullptr;        // [6][nv]
    double* dK0c = nullptr;      // [nv][6] c-rows / b_eq-columns of the boundary-only inverse
    int solve = MATO_SOLVE_DENSE;
    std::vector<double> Ks0, Ksn;  // structured solve: inverses of K_0 and K_{rho n}, (nv+6)^2 FP64
    double* dS = nullptr;        // structured solve: [nv][nv] M1, [nv][nv] M2, [nv][6] E0, [nv][6] En
    unsigned* dPairs = nullptr;  // [n(n-1)/2 + n n_obs] internal row -> i | j << 16 (i < j)
    std::vector<unsigned> pairs; // host copy: the canonical row of internal row r is canonical_row(pairs[r])
    void* dAhi = nullptr;        // GEMM operand K11^{-1}: fp32, bf16 high term or fp64
    void* dAlo = nullptr;        // bf16 middle and low terms, one [Mp][ldk] plane each
    int ldk = 0;                 // padded row stride of the GEMM operand
    size_t bytes = 0;            // device bytes held
};

struct mato_batch_s {
    int precision = MATO_FP32;
    void* impl = nullptr;        // mato::Engine<float> or mato::Engine<double>
};
