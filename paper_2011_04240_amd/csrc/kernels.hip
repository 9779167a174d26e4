// Per-iteration kernels of Algorithm 1 other than the inverse product.
//
//   pairwise_kernel  positions X = P c (eq. (param)) for a block of instants, then for
//                    every pair p = (i, j), i < j, at those instants: the difference
//                    delta = X_i - X_j, the alpha/beta projection of eq.
//                    (sphere_project), the clipped d step of eq. (step_d), the
//                    multiplier update of eq. (lag_update), b_fc of eq. (b_f) for the
//                    next x/y/z step, and the per-agent sums
//                    S_i(t) = sum_{j>i} b_ij(t) - sum_{j<i} b_ji(t)
//                    that A_fc^T b reduces to before the factor P^T.
//   qbuild_kernel    g = rho A_fc^T b_fc = rho P^T S_i (FP64), plus the iteration's
//                    residual record and the convergence test.
//   residual_kernel  FP64 refinement residual [g - H c ; b_eq - A c] of eq. (kkt_step_x),
//                    with H c = (I (x) Pdd^T Pdd) c + rho ((n I - 1 1^T) (x) P^T P) c.
//   init_kernel      boundary-only minimum-acceleration coefficients (initialisation).
//
// The alpha/beta/d step is evaluated without trigonometry.  With the scaled
// distance s = ||(dx/l_xy, dy/l_xy, dz/l_z)||, the direction of eq.
// (sphere_proposed) at the projected angles is e = delta / s, so
//     d* = e^T (delta + lambda/rho) / ||e||^2 = s (1 + delta^T lambda / (rho ||delta||^2)),
//     d e = w delta with w = d / s = max(1/s, 1 + delta^T lambda / (rho ||delta||^2)),
//     f_c = delta - d e.
// delta = 0 takes alpha = beta = 0, i.e. e = (0, 0, l_z).
#include "common.h"

namespace mato {

template <typename S>
__device__ inline S dev_sqrt(S x);
template <>
__device__ inline float dev_sqrt<float>(float x) { return sqrtf(x); }
template <>
__device__ inline double dev_sqrt<double>(double x) { return sqrt(x); }

// Decode the pair index p of an n-agent problem into (i, j), i < j.
__device__ inline void decode_pair(int p, int n, int& i, int& j) {
    const int a = 2 * n - 1;
    int ii = (int)(((float)a - sqrtf((float)(a * a - 8 * p))) * 0.5f);
    ii = ii < 0 ? 0 : (ii > n - 2 ? n - 2 : ii);
    if (row_offset(ii + 1, n) <= p) ++ii;
    if (row_offset(ii + 1, n) <= p) ++ii;
    if (row_offset(ii, n) > p) --ii;
    if (row_offset(ii, n) > p) --ii;
    i = ii;
    j = p - row_offset(ii, n) + ii + 1;
}

template <typename T, int BLOCK>
__device__ inline void block_reduce3(T& mx, T& s1, T& s2, T* sh /* 3 * BLOCK/64 */) {
    for (int off = 32; off > 0; off >>= 1) {
        mx = fmax(mx, __shfl_xor(mx, off));
        s1 += __shfl_xor(s1, off);
        s2 += __shfl_xor(s2, off);
    }
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    constexpr int NW = BLOCK / 64;
    if (lane == 0) {
        sh[w] = mx;
        sh[NW + w] = s1;
        sh[2 * NW + w] = s2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        T a = sh[0], b = sh[NW], c = sh[2 * NW];
        for (int k = 1; k < NW; ++k) {
            a = fmax(a, sh[k]);
            b += sh[NW + k];
            c += sh[2 * NW + k];
        }
        mx = a;
        s1 = b;
        s2 = c;
    }
}

// One workgroup per work item: instants [t0, t0 + tc) of one problem, all pairs.
// LDS: X [tc][3][n] then b_fc [tc][3][n_pairs] (scalar S).
template <typename S, int BLOCK>
__global__ __launch_bounds__(BLOCK) void pairwise_kernel(const WorkItem* __restrict__ items,
                                                         const ProblemDesc<S>* __restrict__ probs,
                                                         int mode) {
    const WorkItem it = items[blockIdx.x];
    const ProblemDesc<S>& D = probs[it.prob];
    if (!D.ctrl[3]) return;                          // inactive slot
    if (mode == kModeIter && D.ctrl[1]) return;      // converged
    extern __shared__ __align__(16) unsigned char smem_raw[];
    S* Xs = reinterpret_cast<S*>(smem_raw);
    const int n = D.n, np = D.np, nv = D.nv, t0 = it.t0, tc = it.tc;
    S* Bs = Xs + tc * 3 * n;
    const int tid = threadIdx.x;

    double cost = 0.0;
    if (mode != kModeSetState) {
        // positions X = P c at the block's instants (FP64 products, stored as S)
        const int nX = tc * 3 * n;
        for (int idx = tid; idx < nX; idx += BLOCK) {
            const int tl = idx / (3 * n);
            const int rem = idx - tl * 3 * n;
            const int a = rem / n, i = rem - a * n;
            const double* Pt = D.P + (size_t)(t0 + tl) * nv;
            const double* Pddt = D.Pdd + (size_t)(t0 + tl) * nv;
            const double* ci = D.c + (size_t)a * D.ldc + (size_t)i * nv;
            double x = 0.0, acc = 0.0;
            for (int k = 0; k < nv; ++k) {
                const double ck = ci[k];
                x += Pt[k] * ck;
                acc += Pddt[k] * ck;
            }
            Xs[idx] = (S)x;
            cost += acc * acc;
            if (D.dbg_X) D.dbg_X[((size_t)(t0 + tl) * 3 + a) * n + i] = (S)x;
        }
        __syncthreads();
    }

    const S ia2 = D.ia2, ib2 = D.ib2, rho = D.srho, irho = D.sirho, lzl = D.lz;
    S rmax = 0, rsum = 0;
    const int total = tc * np;
    constexpr int U = 4;
    for (int q0 = 0; q0 < total; q0 += BLOCK * U) {
        S L[U][3];
        S Pj[U][3];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int q = q0 + u * BLOCK + tid;
            L[u][0] = L[u][1] = L[u][2] = 0;
            Pj[u][0] = Pj[u][1] = Pj[u][2] = 0;
            if (q < total && mode != kModeInit) {
                const int tl = q / np, p = q - tl * np;
                const size_t base = (size_t)(t0 + tl) * 3 * np + p;
                L[u][0] = D.lam[base];
                L[u][1] = D.lam[base + np];
                L[u][2] = D.lam[base + 2 * (size_t)np];
                if (mode == kModeSetState) {
                    Pj[u][0] = D.proj_in[base];
                    Pj[u][1] = D.proj_in[base + np];
                    Pj[u][2] = D.proj_in[base + 2 * (size_t)np];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int q = q0 + u * BLOCK + tid;
            if (q >= total) continue;
            const int tl = q / np, p = q - tl * np;
            const size_t base = (size_t)(t0 + tl) * 3 * np + p;
            S* Bt = Bs + (size_t)tl * 3 * np;
            const S lx = L[u][0], ly = L[u][1], lzm = L[u][2];
            if (mode == kModeSetState) {
                Bt[p] = Pj[u][0] - lx * irho;
                Bt[np + p] = Pj[u][1] - ly * irho;
                Bt[2 * np + p] = Pj[u][2] - lzm * irho;
                continue;
            }
            int i, j;
            decode_pair(p, n, i, j);
            const S* X = Xs + tl * 3 * n;
            const S dx = X[i] - X[j];
            const S dy = X[n + i] - X[n + j];
            const S dz = X[2 * n + i] - X[2 * n + j];
            const S q2 = (dx * dx + dy * dy) * ia2 + dz * dz * ib2;   // s^2
            S px, py, pz, dd;
            if (q2 > 0) {
                const S D2 = dx * dx + dy * dy + dz * dz;
                const S s = dev_sqrt<S>(q2);
                const S dl = dx * lx + dy * ly + dz * lzm;
                const S w = fmax(S(1) / s, S(1) + dl * irho / D2);
                px = w * dx;
                py = w * dy;
                pz = w * dz;
                dd = w * s;
            } else {                                  // delta = 0: e = (0, 0, l_z)
                dd = fmax(S(1), lzm * irho / lzl);
                px = 0;
                py = 0;
                pz = dd * lzl;
            }
            const S fx = dx - px, fy = dy - py, fz = dz - pz;
            S nlx = 0, nly = 0, nlz = 0;
            if (mode == kModeIter) {
                nlx = lx + rho * fx;
                nly = ly + rho * fy;
                nlz = lzm + rho * fz;
                const S fn2 = fx * fx + fy * fy + fz * fz;
                rmax = fmax(rmax, fn2);
                rsum += fn2;
            }
            D.lam[base] = nlx;
            D.lam[base + np] = nly;
            D.lam[base + 2 * (size_t)np] = nlz;
            Bt[p] = px - nlx * irho;
            Bt[np + p] = py - nly * irho;
            Bt[2 * np + p] = pz - nlz * irho;
            if (D.dbg_proj) {
                D.dbg_proj[base] = px;
                D.dbg_proj[base + np] = py;
                D.dbg_proj[base + 2 * (size_t)np] = pz;
            }
            if (D.dbg_d) D.dbg_d[(size_t)(t0 + tl) * np + p] = dd;
        }
    }
    __syncthreads();

    // S_i(t) = sum_{j<i} (-b_ji) + sum_{j>i} b_ij, j ascending (fixed order)
    const int nS = tc * 3 * n;
    for (int o = tid; o < nS; o += BLOCK) {
        const int tl = o / (3 * n);
        const int rem = o - tl * 3 * n;
        const int a = rem / n, i = rem - a * n;
        const S* Bt = Bs + ((size_t)tl * 3 + a) * np;
        S acc = 0;
        int pj = i - 1;
        for (int j = 0; j < i; ++j) {
            acc -= Bt[pj];
            pj += n - j - 2;
        }
        const int base = row_offset(i, n) - i - 1;
        for (int j = i + 1; j < n; ++j) acc += Bt[base + j];
        D.ssum[((size_t)(t0 + tl) * 3 + a) * n + i] = acc;
    }

    if (mode == kModeIter) {
        __shared__ double red[3 * (BLOCK / 64)];
        double mx = (double)rmax, s1 = (double)rsum, s2 = cost;
        block_reduce3<double, BLOCK>(mx, s1, s2, red);
        if (tid == 0) {
            double* pp = D.part + (size_t)it.slab * 4;
            pp[0] = mx;
            pp[1] = s1;
            pp[2] = s2;
        }
    }
}

// One workgroup per problem: g = rho P^T S (FP64) into q[a][0 .. n*nv), then in
// iteration mode the residual record of this iteration and the convergence test.
template <typename S>
__global__ __launch_bounds__(256) void qbuild_kernel(const ProblemDesc<S>* __restrict__ probs, int mode) {
    const ProblemDesc<S>& D = probs[blockIdx.x];
    if (!D.ctrl[3]) return;
    if (mode == kModeIter && D.ctrl[1]) return;
    const int n = D.n, nv = D.nv, T = D.T;
    const int tot = 3 * n * nv;
    for (int o = threadIdx.x; o < tot; o += blockDim.x) {
        const int a = o / (n * nv);
        const int rem = o - a * n * nv;
        const int i = rem / nv, k = rem - i * nv;
        double acc = 0.0;
        const S* sp = D.ssum + (size_t)a * n + i;
        for (int t = 0; t < T; ++t) acc += D.P[(size_t)t * nv + k] * (double)sp[(size_t)t * 3 * n];
        D.q[(size_t)a * D.ldq + rem] = D.rho * acc;
    }
    if (mode == kModeIter && threadIdx.x == 0) {
        double mx = 0.0, s1 = 0.0, s2 = 0.0;
        for (int k = 0; k < D.nslab; ++k) {
            const double* pp = D.part + (size_t)k * 4;
            mx = fmax(mx, pp[0]);
            s1 += pp[1];
            s2 += pp[2];
        }
        const int it = D.ctrl[0];
        const double rmax = sqrt(mx);
        if (it < D.hist_cap) {
            D.hist[(size_t)it * 3 + 0] = rmax;
            D.hist[(size_t)it * 3 + 1] = sqrt(s1 / ((double)D.np * (double)T));
            D.hist[(size_t)it * 3 + 2] = s2;
        }
        D.ctrl[0] = it + 1;
        if (!isfinite(s1) || !isfinite(s2)) {
            D.ctrl[2] = 1;
            D.ctrl[1] = 1;
        } else if (D.tol > 0.0 && rmax < D.tol) {
            D.ctrl[1] = 1;
        }
    }
}

// grid (problems, 3 axes): r = [g - H c ; b_eq - A c] in FP64.
template <typename S>
__global__ __launch_bounds__(256) void residual_kernel(const ProblemDesc<S>* __restrict__ probs) {
    const ProblemDesc<S>& D = probs[blockIdx.x];
    if (!D.ctrl[3] || D.ctrl[1]) return;
    const int a = blockIdx.y;
    const int n = D.n, nv = D.nv;
    const double* c = D.c + (size_t)a * D.ldc;
    const double* q = D.q + (size_t)a * D.ldq;
    double* r = D.r + (size_t)a * D.ldq;
    __shared__ double csum[kMaxCoef];
    __shared__ double PtP[kMaxCoef * kMaxCoef], PddtPdd[kMaxCoef * kMaxCoef], A[kNb * kMaxCoef];
    for (int e = threadIdx.x; e < nv * nv; e += blockDim.x) {
        PtP[e] = D.PtP[e];
        PddtPdd[e] = D.PddtPdd[e];
    }
    for (int e = threadIdx.x; e < kNb * nv; e += blockDim.x) A[e] = D.A[e];
    if (threadIdx.x < nv) {
        double s = 0.0;
        for (int j = 0; j < n; ++j) s += c[(size_t)j * nv + threadIdx.x];
        csum[threadIdx.x] = s;
    }
    __syncthreads();
    const double nr = (double)n * D.rho;
    for (int o = threadIdx.x; o < n * nv; o += blockDim.x) {
        const int i = o / nv, k = o - i * nv;
        const double* ci = c + (size_t)i * nv;
        double h = 0.0;
        for (int l = 0; l < nv; ++l)
            h += PddtPdd[k * nv + l] * ci[l] + PtP[k * nv + l] * (nr * ci[l] - D.rho * csum[l]);
        r[o] = q[o] - h;
    }
    for (int o = threadIdx.x; o < n * kNb; o += blockDim.x) {
        const int i = o / kNb, bb = o - i * kNb;
        const double* ci = c + (size_t)i * nv;
        double h = 0.0;
        for (int l = 0; l < nv; ++l) h += A[bb * nv + l] * ci[l];
        r[n * nv + o] = q[n * nv + o] - h;
    }
}

// grid (problems): c_i = K0^{-1}[c rows, b_eq columns] b_eq,i for every agent and axis.
template <typename S>
__global__ __launch_bounds__(256) void init_kernel(const ProblemDesc<S>* __restrict__ probs,
                                                   const double* const* __restrict__ k0c) {
    const ProblemDesc<S>& D = probs[blockIdx.x];
    if (!D.ctrl[3]) return;
    const int n = D.n, nv = D.nv;
    const double* K0 = k0c[blockIdx.x];
    for (int o = threadIdx.x; o < 3 * n * nv; o += blockDim.x) {
        const int a = o / (n * nv);
        const int rem = o - a * n * nv;
        const int i = rem / nv, k = rem - i * nv;
        const double* beq = D.q + (size_t)a * D.ldq + (size_t)n * nv + (size_t)i * kNb;
        double v = 0.0;
        for (int bb = 0; bb < kNb; ++bb) v += K0[k * kNb + bb] * beq[bb];
        D.c[(size_t)a * D.ldc + rem] = v;
    }
}

// ------------------------------------------------------------- launchers ---
template <typename S>
hipError_t launch_pairwise(const WorkItem* items, int nitems, const ProblemDesc<S>* probs, int mode,
                           int threads, size_t lds, hipStream_t st) {
    if (nitems <= 0) return hipSuccess;
    switch (threads) {
        case 256:
            pairwise_kernel<S, 256><<<nitems, 256, lds, st>>>(items, probs, mode);
            break;
        case 512:
            pairwise_kernel<S, 512><<<nitems, 512, lds, st>>>(items, probs, mode);
            break;
        default:
            pairwise_kernel<S, 1024><<<nitems, 1024, lds, st>>>(items, probs, mode);
            break;
    }
    return hipGetLastError();
}

template <typename S>
hipError_t set_pairwise_lds_limit(size_t lds) {
    hipError_t e = hipFuncSetAttribute((const void*)pairwise_kernel<S, 256>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void*)pairwise_kernel<S, 512>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)pairwise_kernel<S, 1024>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <typename S>
hipError_t launch_qbuild(const ProblemDesc<S>* probs, int nprob, int mode, hipStream_t st) {
    if (nprob <= 0) return hipSuccess;
    qbuild_kernel<S><<<nprob, 256, 0, st>>>(probs, mode);
    return hipGetLastError();
}

template <typename S>
hipError_t launch_residual(const ProblemDesc<S>* probs, int nprob, hipStream_t st) {
    if (nprob <= 0) return hipSuccess;
    residual_kernel<S><<<dim3(nprob, 3), 256, 0, st>>>(probs);
    return hipGetLastError();
}

template <typename S>
hipError_t launch_init(const ProblemDesc<S>* probs, const double* const* k0c, int nprob, hipStream_t st) {
    if (nprob <= 0) return hipSuccess;
    init_kernel<S><<<nprob, 256, 0, st>>>(probs, k0c);
    return hipGetLastError();
}

template hipError_t launch_pairwise<float>(const WorkItem*, int, const ProblemDesc<float>*, int, int, size_t, hipStream_t);
template hipError_t launch_pairwise<double>(const WorkItem*, int, const ProblemDesc<double>*, int, int, size_t, hipStream_t);
template hipError_t set_pairwise_lds_limit<float>(size_t);
template hipError_t set_pairwise_lds_limit<double>(size_t);
template hipError_t launch_qbuild<float>(const ProblemDesc<float>*, int, int, hipStream_t);
template hipError_t launch_qbuild<double>(const ProblemDesc<double>*, int, int, hipStream_t);
template hipError_t launch_residual<float>(const ProblemDesc<float>*, int, hipStream_t);
template hipError_t launch_residual<double>(const ProblemDesc<double>*, int, hipStream_t);
template hipError_t launch_init<float>(const ProblemDesc<float>*, const double* const*, int, hipStream_t);
template hipError_t launch_init<double>(const ProblemDesc<double>*, const double* const*, int, hipStream_t);

}  // namespace mato
