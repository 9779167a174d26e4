// Internal declarations of libmato: device-side problem descriptors, work items,
// plan and batch handles, error plumbing.  Host and device code of every
// translation unit include this file; nothing here is part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

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

// Pair p = (i, j), i < j, in the row order of A_fc: p(i, j) = i n - i(i+1)/2 + j - i - 1.
__host__ __device__ inline int row_offset(int i, int n) { return i * n - i * (i + 1) / 2; }

// -------------------------------------------------------- device descriptors ---
// One problem as the kernels see it.  S is the pairwise-stage scalar (float or
// double); coefficients, linear term, residuals and the boundary data are FP64.
template <typename S>
struct ProblemDesc {
    int n, np, T, nv;           // agents, pairs, instants, coefficients per axis
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
    S* lam;                     // [T][3][np] multipliers
    S* ssum;                    // [T][3][n]  per-agent sums of b_fc (A_fc^T b before P^T)
    double* c;                  // [3][ldc]   coefficients (agent-major per axis)
    double* q;                  // [3][ldq]   [rho A_fc^T b_fc ; b_eq]  (eq. kkt_step_x)
    double* r;                  // [3][ldq]   refinement residual [g - H c ; b_eq - A c]
    double* part;               // [nslab][4] residual partials: max|f|^2, sum|f|^2, cost
    double* hist;               // [hist_cap][3] r_max, r_rms, cost
    int* ctrl;                  // [0] iterations, [1] converged, [2] non-finite, [3] active
    double tol;                 // convergence threshold on r_max (<= 0: none)
    // optional parity outputs (nullptr = off)
    S* dbg_proj;                // [T][3][np] d e
    S* dbg_d;                   // [T][np]
    S* dbg_X;                   // [T][3][n]
    const S* proj_in;           // set-state input [T][3][np]
};

struct WorkItem {               // one pairwise workgroup: instants [t0, t0 + tc) of problem `prob`
    int prob, t0, tc, slab;
};

struct GemmTile {               // one 64-row x 64-column output tile of one same-plan group
    int group, m0, col0, pad;
};

struct GemmGroup {              // problems sharing one plan: C[:, col] (+)= Kc x B[:, col]
    const void* Ahi;            // [M][ldk] c-rows [K11^{-1} | K12^{-1}] (fp32 / bf16 hi / fp64)
    const void* Alo;            // bf16 lo (BF16 split only)
    int M, K, ldk;              // 11n, 17n, padded row stride of A
    int ncols;                  // 3 x members
    int first_col;              // offset into the column table
};

struct GemmCol {                // one right-hand side: problem axis
    const double* b;            // K entries (q or r)
    double* c;                  // M entries
    const int* ctrl;            // problem control word (skip when converged / inactive)
};

enum PairMode { kModeIter = 0, kModeInit = 1, kModeSetState = 2 };

}  // namespace mato

// ------------------------------------------------------------------ handles ---
struct mato_plan_s {
    int n, T, nv, nb, precision, device;
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
    void* dAhi = nullptr;        // GEMM operand, c-rows of K^{-1}: fp32, bf16 hi or fp64
    void* dAlo = nullptr;        // bf16 lo part
    int ldk = 0;                 // padded row stride of the GEMM operand
    size_t bytes = 0;            // device bytes held
};

namespace mato {
template <typename S> struct BatchImpl;
}

struct mato_batch_s {
    int precision = MATO_FP32;
    void* impl = nullptr;        // BatchImpl<float> or BatchImpl<double>
};
