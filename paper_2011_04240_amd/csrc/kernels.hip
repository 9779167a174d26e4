// Per-iteration kernels of Algorithm 1 other than the inverse product.
//
//   pairwise_kernel  for a block of instants and every pair p = (i, j), i < j: the difference
//                    delta = X_i - X_j, the alpha/beta projection of eq.
//                    (sphere_project), the clipped d step of eq. (step_d), the
//                    multiplier update of eq. (lag_update), b_fc of eq. (b_f) for the
//                    next x/y/z step, and the per-agent sums
//                    S_i(t) = sum_{j>i} b_ij(t) - sum_{j<i} b_ji(t)
//                    that A_fc^T b reduces to before the factor P^T.
//   positions_kernel X = P c at every instant, once per problem (FP64 problems and
//                    initialisation; the FP32 pairwise kernel forms X itself).
//   solve_positions_kernel  the x/y/z step from the two per-agent inverses of the
//                    structured solve, then (FP64) what positions_kernel does.
//   qbuild_kernel    g = rho A_fc^T b_fc = rho P^T S_i (FP64), plus the iteration's
//                    residual record (max ||f_c||, rms, smoothness cost) and the
//                    convergence test.
//   residual_kernel  FP64 refinement residual g - H c of eq. (kkt_step_x), with
//                    H c = (I (x) Pdd^T Pdd) c + rho (((n + n_obs) I - 1 1^T) (x) P^T P) c,
//                    stored as the correction's product reads it (FP64, or rounded to FP32).
//   ceq_kernel       c_eq = K12^{-1} b_eq, the boundary part of the inverse product.
//   init_kernel      boundary-only minimum-acceleration coefficients (initialisation).
//
// The alpha/beta/d step is evaluated without trigonometry.  With the scaled
// distance s = ||(dx/l_xy, dy/l_xy, dz/l_z)||, the direction of eq.
// (sphere_proposed) at the projected angles is e = delta / s, so
//     d* = e^T (delta + lambda/rho) / ||e||^2 = s (1 + delta^T lambda / (rho ||delta||^2)),
//     d e = w delta with w = d / s = max(1/s, 1 + delta^T lambda / (rho ||delta||^2)),
//     f_c = delta - d e.
// delta = 0 takes alpha = beta = 0, i.e. e = (0, 0, l_z).  A per-problem variant
// projects v = delta + lambda/rho instead (e = v / s_v, d = max(1, s_v)).
//
// Descriptor fields are read into registers once per workgroup and device
// pointers are used in the global address space, so that stores cannot force
// the descriptors to be re-read and LDS waits do not wait on global loads.
#include "common.h"

namespace mato {

template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
__device__ inline gptr<T> glob(T* p) {
    return (gptr<T>)p;
}
template <typename T>
__device__ inline gptr<const T> glob(const T* p) {
    return (gptr<const T>)p;
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

// Block maximum and FP64 sum, results in thread 0.  The maximum is taken in S within
// each wavefront (exact, so the same value as in FP64); the sum in the order of
// block_reduce3 (butterfly in each wavefront, then the wavefronts in order).
template <typename S, int BLOCK>
__device__ inline double block_reduce_max_sum(S mx, double& s1, double* sh /* 2 * BLOCK/64 */) {
    for (int off = 32; off > 0; off >>= 1) {
        mx = fmax(mx, __shfl_xor(mx, off));
        s1 += __shfl_xor(s1, off);
    }
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    constexpr int NW = BLOCK / 64;
    if (lane == 0) {
        sh[w] = (double)mx;
        sh[NW + w] = s1;
    }
    __syncthreads();
    double a = 0.0;
    if (threadIdx.x == 0) {
        double b = sh[NW];
        a = sh[0];
        for (int k = 1; k < NW; ++k) {
            a = fmax(a, sh[k]);
            b += sh[NW + k];
        }
        s1 = b;
    }
    return a;
}

// Fast reciprocal and reciprocal square root: the hardware approximations
// (about 1 ulp) in FP32, exact division and square root in FP64.
template <typename S>
struct Recip;
template <>
struct Recip<float> {
    static __device__ inline float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
    static __device__ inline float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
};
template <>
struct Recip<double> {
    static __device__ inline double rsq(double x) { return 1.0 / sqrt(x); }
    static __device__ inline double rcp(double x) { return 1.0 / x; }
};

// hi + lo += v with the rounding error of hi + v kept in lo (Knuth's TwoSum: error-free,
// and the same bits for either order of the two summands).
__device__ inline void two_sum_add(double& hi, double& lo, double v) {
    const double s = hi + v, bv = s - hi;
    lo += (hi - (s - bv)) + (v - bv);
    hi = s;
}

// Bit patterns, to tell an unchanged value (the sign of a zero included) from a changed one.
__device__ inline unsigned bits_of(float x) { return __float_as_uint(x); }
__device__ inline unsigned long long bits_of(double x) { return (unsigned long long)__double_as_longlong(x); }

// Multiplier access through a buffer resource: a wavefront-uniform base, a per-lane
// 32-bit offset and a uniform one; a lane whose offset is past the resource's size
// reads 0 and touches no memory.  Nontemporal (the multipliers are streamed once).
constexpr int kNt = 2;
template <typename S>
struct Buf;
template <>
struct Buf<float> {
    static __device__ inline float load(__amdgpu_buffer_rsrc_t r, unsigned vo, int so) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, kNt));
    }
    static __device__ inline void store(float v, __amdgpu_buffer_rsrc_t r, unsigned vo, int so) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, vo, so, kNt);
    }
};
template <>
struct Buf<double> {
    typedef unsigned u2 __attribute__((ext_vector_type(2)));
    static __device__ inline double load(__amdgpu_buffer_rsrc_t r, unsigned vo, int so) {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, kNt));
    }
    static __device__ inline void store(double v, __amdgpu_buffer_rsrc_t r, unsigned vo, int so) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, vo, so, kNt);
    }
};
constexpr unsigned kOutOfRange = 0x80000000u;   // above every resource size used here

// One workgroup per work item: instants [t0, t0 + tc) of one problem, all pairs.
// LDS: the FP64 agent sums of X [tc][3] (sum form), X [tc][3][n] (copied from the
// positions of the current coefficients), b_fc [tc][3][n_rows] (scalar S; in the sum
// form only the corrections of flagged pairs), the obstacle table, then the row- and
// column-ordered pair flags [tc][ceil(n_rows / 32)] each.  Rows after the agent pairs
// pair an agent with a static obstacle (fixed centre, own semi-axes).
// Threads form `tg` instant groups of `pw` pair lanes (pw = the smallest power of two
// >= n_pairs, between 64 and BLOCK).  A lane owns U pairs of a chunk and walks its
// group's instants; the multipliers of the next (chunk, instant) are loaded while the
// current one is computed, and the first ones before the positions are staged.
template <typename S, int BLOCK, int NV, int MODE, bool OBS>
__global__ __launch_bounds__(BLOCK) void pairwise_kernel(const WorkItem* __restrict__ items,
                                                         const ProblemDesc<S>* __restrict__ probs) {
    constexpr int U = 4;
    const WorkItem it = items[blockIdx.x];
    const ProblemDesc<S>* __restrict__ Dp = probs + it.prob;
    gptr<const int> ctrl = glob((const int*)Dp->ctrl);
    if (!ctrl[3]) return;                          // inactive slot
    if (MODE == kModeIter && ctrl[1]) return;      // converged
    const int n = Dp->n, np = Dp->np, n_obs = OBS ? Dp->n_obs : 0;   // OBS: some problem has obstacles
    const int t0 = it.t0, tc = it.tc;
    gptr<const S> Xm = glob((const S*)Dp->X);
    gptr<const unsigned> pairs = glob(Dp->pairs);
    gptr<S> lam = glob(Dp->lam);
    gptr<S> ssum = glob(Dp->ssum);
    gptr<const S> proj_in = glob(Dp->proj_in);
    S* const dbg_proj_p = Dp->dbg_proj;
    S* const dbg_d_p = Dp->dbg_d;
    const bool dbg_on = dbg_proj_p != nullptr || dbg_d_p != nullptr;
    gptr<double> part = glob(Dp->part);
    const S ia2 = Dp->ia2, ib2 = Dp->ib2, rho = Dp->srho, irho = Dp->sirho, lzl = Dp->lz;
    const bool shifted = Dp->shifted != 0;
    // b_fc feeds the next x-step, which uses the next stage's rho on a stage's last iteration
    const S irho_b = (MODE == kModeIter && Dp->switch_at > 0 && ctrl[0] + 1 == Dp->switch_at) ? Dp->sirho_next : irho;

    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* SXs = reinterpret_cast<double*>(smem_raw);   // [tc][3] sum over agents of X (sum form)
    S* Xs = reinterpret_cast<S*>(SXs + tc * 3);
    S* Bs = Xs + tc * 3 * n;
    S* Os = Bs + (size_t)tc * 3 * np;                // obstacle table [n_obs][kObs]
    // sum form of the per-agent sums (plain iteration without obstacles):
    //   S_i = n X_i - sum_j X_j + sum over pairs of i whose b_fc is not delta of (b_fc - delta),
    // the corrections in Bs, flagged by pair in row order (Mr) and in column order (Mc).  The
    // agent sum is compensated and S_i is formed in FP64 and rounded once: a rounding of
    // sum_j X_j shared by every agent would shift the agent mean of S, which the x-step's
    // mean block (no rho term) amplifies
    const bool sumform = (MODE == kModeIter || MODE == kModeSetState) && !shifted && n_obs == 0;
    const int nw = (np + 31) >> 5;
    unsigned* Mr = reinterpret_cast<unsigned*>(Os + (size_t)n_obs * kObs);   // [tc][nw]
    unsigned* Mc = Mr + tc * nw;                                              // [tc][nw]
    const int tid = threadIdx.x;

    int pw = 64;
    while (pw < np && pw < BLOCK) pw <<= 1;
    const int tg = BLOCK / pw;
    const int pl = tid & (pw - 1);
    // pw >= 64: a wavefront lies in one instant group, so the group index and everything
    // derived from it (instants, multiplier and LDS bases) are wavefront-uniform
    const int tgid = __builtin_amdgcn_readfirstlane(tid / pw);
    const int ntl = (tgid < tc) ? (tc - tgid + tg - 1) / tg : 0;   // instants of this lane's group
    const int npb = (np + pw * U - 1) / (pw * U);                   // pair chunks
    const int nit = npb * ntl;
    // multipliers of (chunk kc, instant ki) of this group start at element
    // first0 + kc cstride + ki istride; a buffer resource from there to the end of the
    // instant's three axes, lane offset pl sizeof(S), uniform offset (u pw + axis np) sizeof(S)
    const size_t first0 = (size_t)(t0 + tgid) * 3 * np;
    const size_t istride = (size_t)tg * 3 * np;
    const int cstride = pw * U;
    auto rsrc_at = [&](size_t first, int kc) {
        return __builtin_amdgcn_make_buffer_rsrc((void*)(S*)(lam + first), (short)0,
                                                 (3 * np - kc * cstride) * (int)sizeof(S), 0x00020000);
    };
    const int axis_bytes = np * (int)sizeof(S);
    const unsigned lane_bytes = (unsigned)pl * sizeof(S);

    // staged loads of one (chunk, instant): pair codes and multipliers (or d e in set-state)
    unsigned code[U];
    S L[U][3], Q[U][3];
    auto fetch = [&](int kc, int ki, size_t first) {
        const int pb = kc * cstride;
        const __amdgpu_buffer_rsrc_t rs = rsrc_at(first, kc);
        if (ki == 0) {                              // the same codes for every instant of the chunk
#pragma unroll
            for (int u = 0; u < U; ++u) code[u] = pairs[min(pb + u * pw + pl, np - 1)];   // past np: unused
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int p = pb + u * pw + pl;
            const bool ok = p < np;
            if (MODE != kModeInit) {
                const unsigned vo = ok ? lane_bytes : kOutOfRange;   // past the last pair: 0
                const int so = u * pw * (int)sizeof(S);
                L[u][0] = Buf<S>::load(rs, vo, so);
                L[u][1] = Buf<S>::load(rs, vo, so + axis_bytes);
                L[u][2] = Buf<S>::load(rs, vo, so + 2 * axis_bytes);
            } else {
                L[u][0] = L[u][1] = L[u][2] = 0;
            }
            if (MODE == kModeSetState) {
                Q[u][0] = Q[u][1] = Q[u][2] = 0;
                if (ok) {
                    const size_t e = first + (size_t)(u * pw + pl);
                    Q[u][0] = proj_in[e];
                    Q[u][1] = proj_in[e + np];
                    Q[u][2] = proj_in[e + 2 * (size_t)np];
                }
            }
        }
    };
    if (nit > 0) fetch(0, 0, first0);

    if (n_obs > 0) {
        gptr<const S> og = glob(Dp->obs);
        for (int idx = tid; idx < n_obs * kObs; idx += BLOCK) Os[idx] = og[idx];
    }
    if (MODE != kModeSetState || sumform) {
        // positions of the block's instants: one contiguous slab of X [t][3][n]
        const int nX = tc * 3 * n;
        gptr<const S> Xg = Xm + (size_t)t0 * 3 * n;
        for (int idx = tid; idx < nX; idx += BLOCK) Xs[idx] = Xg[idx];
        if (sumform)
            for (int idx = tid; idx < 2 * tc * nw; idx += BLOCK) Mr[idx] = 0u;
        __syncthreads();
        if (sumform) {                              // sum_j X_j of each (instant, axis) row:
            int G = 1;                              // G = min(64, 2^ceil(log2 n)) lanes per row (a
            while (G < n && G < 64) G <<= 1;        // function of n only), lane-strided double-double
            const int seg = tid / G, sl = tid & (G - 1);   // sums (TwoSum), then a butterfly within
            for (int r = seg; r < tc * 3; r += BLOCK / G) { // the segment: a fixed order
                double hi = 0.0, lo = 0.0;
                for (int j = sl; j < n; j += G) two_sum_add(hi, lo, (double)Xs[r * n + j]);
                for (int off = G >> 1; off > 0; off >>= 1) {
                    const double h2 = __shfl_xor(hi, off), l2 = __shfl_xor(lo, off);
                    two_sum_add(hi, lo, h2);        // exact and symmetric: every lane gets the same bits
                    lo += l2;
                }
                if (sl == 0) SXs[r] = (hi + lo) + 0.0;   // + 0.0: a -0 total as +0
            }
        }
    }

    S rmax = 0, rsum = 0;
    int kc = 0, ki = 0;                             // chunk and instant of step k (instants inner)
    size_t f_cur = first0, c_first = first0;        // first multiplier of (kc, ki) and of (kc, 0)
    for (int k = 0; k < nit; ++k) {
        unsigned cc[U];
        S Lc[U][3], Qc[U][3];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            cc[u] = code[u];
            Lc[u][0] = L[u][0]; Lc[u][1] = L[u][1]; Lc[u][2] = L[u][2];
            if (MODE == kModeSetState) { Qc[u][0] = Q[u][0]; Qc[u][1] = Q[u][1]; Qc[u][2] = Q[u][2]; }
        }
        int kc1 = kc, ki1 = ki + 1;
        size_t f_nxt = f_cur + istride, c_nxt = c_first;
        if (ki1 == ntl) {
            ki1 = 0;
            ++kc1;
            c_nxt = c_first + cstride;
            f_nxt = c_nxt;
        }
        if (k + 1 < nit) fetch(kc1, ki1, f_nxt);
        const int pb = kc * cstride;
        const int tl = tgid + ki * tg;
        const size_t fc = f_cur;                    // element (t0 + tl) 3 np + pb
        const __amdgpu_buffer_rsrc_t rs = rsrc_at(f_cur, kc);
        kc = kc1;
        ki = ki1;
        f_cur = f_nxt;
        c_first = c_nxt;
        S* Bt = Bs + tl * 3 * np;
        const S* X = Xs + tl * 3 * n;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int p = pb + u * pw + pl;
            if (p >= np) continue;
            const S lx = Lc[u][0], ly = Lc[u][1], lzm = Lc[u][2];
            const int i = (int)(cc[u] & 0xffffu), j = (int)(cc[u] >> 16);
            // sum form: a pair whose b_fc - delta is not +0 on every axis keeps it in Bt and is
            // flagged (the flags and values depend only on the state, in every mode)
            auto record = [&](S cx, S cy, S cz) {
                if ((bits_of(cx) | bits_of(cy) | bits_of(cz)) == 0) return;
                Bt[p] = cx;
                Bt[np + p] = cy;
                Bt[2 * np + p] = cz;
                const int c = j * (j - 1) / 2 + i;  // column order: pairs grouped by the larger agent
                atomicOr(&Mr[tl * nw + (p >> 5)], 1u << (p & 31));
                atomicOr(&Mc[tl * nw + (c >> 5)], 1u << (c & 31));
            };
            if (MODE == kModeSetState) {
                const S bx = Qc[u][0] - lx * irho, by = Qc[u][1] - ly * irho, bz = Qc[u][2] - lzm * irho;
                if (sumform) {
                    record(bx - (X[i] - X[j]), by - (X[n + i] - X[n + j]), bz - (X[2 * n + i] - X[2 * n + j]));
                } else {
                    Bt[p] = bx;
                    Bt[np + p] = by;
                    Bt[2 * np + p] = bz;
                }
                continue;
            }
            // partner: agent j, or (rows after the pairs) static obstacle j - n with its own axes
            S xj, yj, zj, ia2p = ia2, ib2p = ib2, lzp = lzl;
            if (!OBS || j < n) {
                xj = X[j];
                yj = X[n + j];
                zj = X[2 * n + j];
            } else {
                const S* ob = Os + (j - n) * kObs;
                xj = ob[0];
                yj = ob[1];
                zj = ob[2];
                ia2p = ob[3];
                ib2p = ob[4];
                lzp = ob[5];
            }
            const S dx = X[i] - xj;
            const S dy = X[n + i] - yj;
            const S dz = X[2 * n + i] - zj;
            const S q2 = (dx * dx + dy * dy) * ia2p + dz * dz * ib2p;   // s^2 (plain projection)
            // no multiplier (+0) and clear of the collision set by a margin: 1/s < 1 (also as the
            // FP32 approximation), so the general branch takes w = 1, d e = delta, f_c = +0,
            // lambda = +0 (unchanged, not stored), b_fc = delta and a zero residual (maximum and
            // sum unchanged), bit for bit; the shortcut below does just that
            // (bitwise and: one condition, not a chain of branches)
            const bool clear = (q2 > S(1.0001)) & ((bits_of(lx) | bits_of(ly) | bits_of(lzm)) == 0);
            const bool fast = (MODE == kModeIter) & !shifted & !dbg_on & clear;
            if (fast) {
                if (!sumform) {                     // the sum form needs no entry for b_fc = delta
                    Bt[p] = dx;
                    Bt[np + p] = dy;
                    Bt[2 * np + p] = dz;
                }
                continue;
            }
            S px, py, pz, dd;
            if (!shifted) {
                if (q2 > 0) {
                    const S D2 = dx * dx + dy * dy + dz * dz;
                    const S rs = Recip<S>::rsq(q2);                     // 1 / s
                    const S dl = dx * lx + dy * ly + dz * lzm;
                    const S w = fmax(rs, S(1) + dl * irho * Recip<S>::rcp(D2));
                    px = w * dx;
                    py = w * dy;
                    pz = w * dz;
                    dd = w * (q2 * rs);                                 // d = w s
                } else {                                                // delta = 0: e = (0, 0, l_z)
                    dd = fmax(S(1), lzm * irho / lzp);
                    px = 0;
                    py = 0;
                    pz = dd * lzp;
                }
            } else {
                // variant: project v = delta + lambda/rho; then d = max(1, s_v), d e = max(1/s_v, 1) v
                const S vx = dx + lx * irho, vy = dy + ly * irho, vz = dz + lzm * irho;
                const S q2 = (vx * vx + vy * vy) * ia2p + vz * vz * ib2p;
                if (q2 > 0) {
                    const S rs = Recip<S>::rsq(q2);
                    const S w = fmax(rs, S(1));
                    px = w * vx;
                    py = w * vy;
                    pz = w * vz;
                    dd = w * (q2 * rs);
                } else {                                                // v = 0: e = (0, 0, l_z), d = 1
                    dd = S(1);
                    px = 0;
                    py = 0;
                    pz = lzp;
                }
            }
            const S fx = dx - px, fy = dy - py, fz = dz - pz;
            S nlx = 0, nly = 0, nlz = 0;
            if (MODE == kModeIter) {
                nlx = lx + rho * fx;
                nly = ly + rho * fy;
                nlz = lzm + rho * fz;
                const S fn2 = fx * fx + fy * fy + fz * fz;
                rmax = fmax(rmax, fn2);
                rsum += fn2;
            }
            // an iteration stores only the multipliers whose bits change: lambda = 0 on a pair
            // that does not collide stays 0 exactly (w = 1, d e = delta, f_c = 0)
            const int so = u * pw * (int)sizeof(S);
            if (MODE != kModeIter || bits_of(nlx) != bits_of(lx)) Buf<S>::store(nlx, rs, lane_bytes, so);
            if (MODE != kModeIter || bits_of(nly) != bits_of(ly)) Buf<S>::store(nly, rs, lane_bytes, so + axis_bytes);
            if (MODE != kModeIter || bits_of(nlz) != bits_of(lzm))
                Buf<S>::store(nlz, rs, lane_bytes, so + 2 * axis_bytes);
            const S bx = px - nlx * irho_b, by = py - nly * irho_b, bz = pz - nlz * irho_b;
            if (!sumform) {
                Bt[p] = bx;
                Bt[np + p] = by;
                Bt[2 * np + p] = bz;
            } else {
                record(bx - dx, by - dy, bz - dz);   // +0 for a clear pair (b_fc = delta)
            }
            if (dbg_on) {
                const size_t e = fc + (size_t)(u * pw + pl);          // (t0 + tl) 3 np + p
                if (dbg_proj_p) {
                    gptr<S> dp = glob(dbg_proj_p);
                    dp[e] = px;
                    dp[e + np] = py;
                    dp[e + 2 * (size_t)np] = pz;
                }
                if (dbg_d_p) glob(dbg_d_p)[(size_t)(t0 + tl) * np + p] = dd;
            }
        }
    }
    __syncthreads();

    // S_i(t) = sum_{j<i} (-b_ji) + sum_{j>i} b_ij, j ascending (fixed order), then
    // sum_o (x_o + b_io) over static obstacles, o ascending.  Sum form: n X_i - sum_j X_j,
    // then the corrections of the flagged pairs (j, i), j < i ascending, and (i, j), j > i
    // ascending (b_fc = delta + correction, and sum_{j != i} (X_i - X_j) = n X_i - sum_j X_j)
    const int n3 = 3 * n;
    const int nS = tc * n3;
    for (int o = tid; o < nS; o += BLOCK) {
        const int tl = o / n3;
        const int rem = o - tl * n3;
        const int a = rem / n, i = rem - a * n;
        const S* Bt = Bs + ((size_t)tl * 3 + a) * np;
        if (sumform) {
            double acc = (double)n * (double)Xs[((size_t)tl * 3 + a) * n + i] - SXs[tl * 3 + a];
            // flagged bits of [lo, hi) in word w, ascending
            auto each_bit = [&](const unsigned* m, int lo, int hi, auto&& f) {
                for (int w = lo >> 5; lo < hi && w <= (hi - 1) >> 5; ++w) {
                    unsigned bits = m[w];
                    if (lo > 32 * w) bits &= ~0u << (lo - 32 * w);
                    if (hi - 32 * w < 32) bits &= (1u << (hi - 32 * w)) - 1u;
                    while (bits) {
                        f(32 * w + __builtin_ctz(bits));
                        bits &= bits - 1u;
                    }
                }
            };
            const int c0 = i * (i - 1) / 2;         // pairs (j, i), j < i: column bits c0 + j
            each_bit(Mc + tl * nw, c0, c0 + i, [&](int c) {
                const int j = c - c0;
                acc -= (double)Bt[row_offset(j, n) + i - j - 1];
            });
            const int r0 = row_offset(i, n);        // pairs (i, j), j > i: row bits r0 + j - i - 1
            each_bit(Mr + tl * nw, r0, r0 + n - i - 1, [&](int p) { acc += (double)Bt[p]; });
            ssum[((size_t)(t0 + tl) * 3 + a) * n + i] = (S)acc;
            continue;
        }
        S acc = 0;
        const S* col = Bt + i - 1;          // b_ji, j < i: column i of the pair triangle
        int off = 0;                        // row_offset(j, n) - j: the same for every lane
#pragma unroll 8
        for (int j = 0; j < i; ++j) {
            acc -= col[off];
            off += n - j - 2;
        }
        const S* row = Bt + row_offset(i, n) - i - 1;
#pragma unroll 8
        for (int j = i + 1; j < n; ++j) acc += row[j];
        if (n_obs > 0) {                    // agent-obstacle rows: target x_o + d e - lambda / rho
            const S* ro = Bt + n * (n - 1) / 2 + (size_t)i * n_obs;
            for (int o = 0; o < n_obs; ++o) acc += Os[o * kObs + a] + ro[o];
        }
        ssum[((size_t)(t0 + tl) * 3 + a) * n + i] = acc;
    }

    if (MODE == kModeIter) {
        __shared__ double red[2 * (BLOCK / 64)];
        double s1 = (double)rsum;
        const double mx = block_reduce_max_sum<S, BLOCK>(rmax, s1, red);
        if (tid == 0) {
            gptr<double> pp = part + (size_t)it.slab * 4;
            pp[0] = mx;
            pp[1] = s1;
        }
    }
}

// ----------------------------------------------------------------------------------
// The pairwise stage of FP32 problems, with the per-agent sums in fixed point.
//
// S_i(t) = sum_{j>i} b_ij - sum_{j<i} b_ji + sum_o (x_o + b_io).  With every b written as
// delta + corr (delta = X_i - X_j, or X_i - x_o on an obstacle row; corr = b - delta):
//     S_i = (n + n_obs) X_i - sum_j X_j + C_i,  C_i = sum over the rows of agent i of (+-corr),
// + where i is the row's first member, - where it is the second.  This kernel forms C_i; the
// positions' part enters the linear term as P^T of it, (n + n_obs) P^T P c_i -
// P^T P sum_j c_j, in FP64 from the coefficients (no rounding of the positions).  The
// corrections enter C_i in fixed point with kFx fractional bits (int64): those sums are
// exact, so the rows' corrections can be added with LDS atomics in whatever order the lanes
// reach them and C_i does not depend on the tile shape or the batch.  C_i is rounded to FP32
// once.  A row whose corr is +0 on every axis (b = delta: the usual case away from
// collisions) adds nothing.  The rows come in the plan's tournament order, so the lanes
// of a wavefront touch different agents and the atomics rarely collide.
//
// The positions of the work item's instants are formed here from the current
// coefficients (X = P c in FP64, eq. (param)), so an FP32 iteration has no positions
// launch and no positions traffic; the X buffer is filled only when it is read back.
//
// LDS per instant of the work item: the positions [n] (x, y, z, 0) and the corrections
// [3][n] (int64), 40 n bytes (at least 16 n + 8 n_v: the corrections' area holds the
// basis rows first); then the obstacle table.  Thread layout, multiplier
// loads and the far-pair shortcut are those of pairwise_kernel.
constexpr int kFx = 40;

// round(v 2^kFx) as an int64 (|v| < 2^22): the double y is exact, hi and lo are its
// upper and lower 32 bits.
__device__ inline long long fx_of(float v) {
    const double y = rint(ldexp((double)v, kFx));
    const double hi = floor(y * 0x1p-32);
    const double lo = fma(hi, -0x1p32, y);
    const unsigned long long u = ((unsigned long long)(unsigned)(int)hi << 32) | (unsigned long long)(unsigned)lo;
    return (long long)u;
}

// Per-pair-instant arithmetic of the FP32 kernel.  Every rounding step is written out
// (fused where fmaf says so, nothing else contracted), so that the two row orders of the
// kernel and its broad phase evaluate the same operations bit for bit wherever they are
// inlined.
//
// s^2 = (dx^2 + dy^2) / l_xy^2 + dz^2 / l_z^2: nondecreasing in |dx|, |dy|, |dz|.
__device__ inline float scaled_sq(float dx, float dy, float dz, float ia2p, float ib2p) {
#pragma clang fp contract(off)
    return fmaf(fmaf(dx, dx, dy * dy), ia2p, (dz * dz) * ib2p);
}

// The plain projection of eqs. (sphere_project), (step_d) for one pair-instant past the
// far-pair shortcut, trig-free (see the top of this file): d e = (px, py, pz) and d, from
// delta, s^2 = q2 and the multiplier.
__device__ inline void project_plain(float dx, float dy, float dz, float q2, float lx, float ly, float lzm,
                                     float irho, float lzp, float& px, float& py, float& pz, float& dd) {
#pragma clang fp contract(off)
    if (q2 > 0) {
        const float D2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
        const float rs_ = Recip<float>::rsq(q2);                        // 1 / s
        const float dl = fmaf(dx, lx, fmaf(dy, ly, dz * lzm));
        const float w = fmaxf(rs_, fmaf(dl * irho, Recip<float>::rcp(D2), 1.f));
        px = w * dx;
        py = w * dy;
        pz = w * dz;
        dd = w * (q2 * rs_);                                            // d = w s
    } else {                                                            // delta = 0: e = (0, 0, l_z)
        dd = fmaxf(1.f, (lzm * irho) / lzp);
        px = 0;
        py = 0;
        pz = dd * lzp;
    }
}

// The multiplier step of eq. (lag_update) with f_c = delta - d e, the row's |f_c|^2, and
// b_fc - delta = d e - lambda_new / rho - delta (the row's correction of the agent sums).
__device__ inline void row_update(float dx, float dy, float dz, float px, float py, float pz, float lx, float ly,
                                  float lzm, float rho, float& nlx, float& nly, float& nlz, float& fn2) {
#pragma clang fp contract(off)
    const float fx = dx - px, fy = dy - py, fz = dz - pz;
    nlx = fmaf(rho, fx, lx);
    nly = fmaf(rho, fy, ly);
    nlz = fmaf(rho, fz, lzm);
    fn2 = fmaf(fx, fx, fmaf(fy, fy, fz * fz));
}
__device__ inline float row_correction(float p, float nl, float irho_b, float d) {
#pragma clang fp contract(off)
    return fmaf(-nl, irho_b, p) - d;
}

// s^2 of a pair at least this far apart (from bounding boxes) at every instant of a work
// item is above the shortcut's 1.0001 at each of them: the margin covers the rounding of
// the two evaluations of the same expression.
constexpr float kBroadClear = 1.0002f;

template <int BLOCK, int NV, int MODE, bool OBS>
__global__ __launch_bounds__(BLOCK) void pairwise_fx_kernel(const WorkItem* __restrict__ items,
                                                            const ProblemDesc<float>* __restrict__ probs) {
    using S = float;
    constexpr int U = 4;
    // a problem's items are consecutive in the list: through xcd_tile they run on one die,
    // whose L2 then holds the problem's coefficients for all of them
    const WorkItem it = items[xcd_tile(blockIdx.x, gridDim.x)];
    const ProblemDesc<S>* __restrict__ Dp = probs + it.prob;
    gptr<const int> ctrl = glob((const int*)Dp->ctrl);
    const int n = Dp->n, np = Dp->np, n_obs = OBS ? Dp->n_obs : 0;
    const int t0 = it.t0, tc = it.tc;
    const int nv = NV > 0 ? NV : Dp->nv;
    const int ngr = (np + 63) >> 6;                                      // 64-row multiplier groups
    // The first basis entry and group flag of each thread are requested before the activity
    // test, so that their latency overlaps it (dropped if the slot is idle).
    const int tid = threadIdx.x;
    gptr<const double> Pm = glob(Dp->P);
    gptr<unsigned> lflag = glob(Dp->lflag);
    const double p_first = tid < tc * nv ? Pm[(size_t)t0 * nv + tid] : 0.0;
    const unsigned f_first = (MODE == kModeIter && tid < tc * ngr) ? lflag[(size_t)t0 * ngr + tid] : 0u;
    if (!ctrl[3]) return;                          // inactive slot
    if (MODE == kModeIter && ctrl[1]) return;      // converged
    gptr<const unsigned> pairs = glob(Dp->pairs);
    gptr<S> lam = glob(Dp->lam);
    gptr<S> ssum = glob(Dp->ssum);
    gptr<const S> proj_in = glob(Dp->proj_in);
    S* const dbg_proj_p = Dp->dbg_proj;
    S* const dbg_d_p = Dp->dbg_d;
    const bool dbg_on = dbg_proj_p != nullptr || dbg_d_p != nullptr;
    gptr<double> part = glob(Dp->part);
    const S ia2 = Dp->ia2, ib2 = Dp->ib2, rho = Dp->srho, irho = Dp->sirho, lzl = Dp->lz;
    const bool shifted = Dp->shifted != 0;
    // b_fc feeds the next x-step, which uses the next stage's rho on a stage's last iteration
    const S irho_b = (MODE == kModeIter && Dp->switch_at > 0 && ctrl[0] + 1 == Dp->switch_at) ? Dp->sirho_next : irho;

    extern __shared__ __align__(16) unsigned char smem_raw[];
    float4* Xs = reinterpret_cast<float4*>(smem_raw);                     // [tc][n]
    long long* Acc = reinterpret_cast<long long*>(Xs + (size_t)tc * n);  // [tc][3][n], first [tc][nv] doubles
    unsigned long long* Fb = reinterpret_cast<unsigned long long*>(Acc + (size_t)tc * max(3 * n, nv));  // [ngr]
    unsigned* Fs = reinterpret_cast<unsigned*>(Fb + ngr);               // [tc][ngr] group flags
    unsigned* NFs = Fs + (size_t)tc * ngr;                               // [tc][ngr] flags after the pass
    unsigned* Gf = NFs + (size_t)tc * ngr;                               // [ngr] some instant flagged
    S* Os = reinterpret_cast<S*>(Gf + ngr);                              // [n_obs][kObs]
    S* Bs = Os + (size_t)n_obs * kObs;                                   // [n][6] boxes over the item
    unsigned* Lq = reinterpret_cast<unsigned*>(Bs + (size_t)n * 6);     // [BLOCK/64][64][2] row lists
    __shared__ int any_general;                    // some row took the general branch (iteration)
    __shared__ int wcnt[BLOCK / 64];
    const int wv = tid >> 6, lane = tid & 63;

    int pw = 64;
    while (pw < np && pw < BLOCK) pw <<= 1;
    const int tg = BLOCK / pw;
    const int pl = tid & (pw - 1);
    const int tgid = __builtin_amdgcn_readfirstlane(tid / pw);          // wavefront-uniform
    const int ntl = (tgid < tc) ? (tc - tgid + tg - 1) / tg : 0;
    const int npb = (np + pw * U - 1) / (pw * U);
    const int nit = npb * ntl;
    const size_t first0 = (size_t)(t0 + tgid) * 3 * np;
    const size_t istride = (size_t)tg * 3 * np;
    const int cstride = pw * U;
    auto rsrc_at = [&](size_t first, int kc) {
        return __builtin_amdgcn_make_buffer_rsrc((void*)(S*)(lam + first), (short)0,
                                                 (3 * np - kc * cstride) * (int)sizeof(S), 0x00020000);
    };
    const int axis_bytes = np * (int)sizeof(S);
    const unsigned lane_bytes = (unsigned)pl * sizeof(S);
    // The rows of a wavefront for one u are 64 consecutive rows from a multiple of 64: one
    // multiplier group, whose flag (0: every multiplier of the group is +0 on every axis)
    // decides whether its multipliers are read.  A group read as 0 takes out-of-range buffer
    // offsets, which return +0 without a memory access.
    const int wrow = __builtin_amdgcn_readfirstlane(pl & ~63);

    unsigned code[U], Fl[U] = {0u, 0u, 0u, 0u};
    S L[U][3], Q[U][3];
    auto fetch = [&](int kc, int ki, size_t first) {
        const int pb = kc * cstride;
        const __amdgpu_buffer_rsrc_t rs = rsrc_at(first, kc);
        if (MODE == kModeIter) {
            const unsigned* fr = Fs + (size_t)(tgid + ki * tg) * ngr;
#pragma unroll
            for (int u = 0; u < U; ++u) Fl[u] = fr[min((pb + u * pw + wrow) >> 6, ngr - 1)];
        }
        if (ki == 0) {
#pragma unroll
            for (int u = 0; u < U; ++u) code[u] = pairs[min(pb + u * pw + pl, np - 1)];   // past np: unused
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int p = pb + u * pw + pl;
            const bool ok = p < np;
            if (MODE != kModeInit) {
                // past the last row, or a group flagged all +0: 0
                const unsigned vo = (ok && (MODE != kModeIter || Fl[u] != 0)) ? lane_bytes : kOutOfRange;
                const int so = u * pw * (int)sizeof(S);
                L[u][0] = Buf<S>::load(rs, vo, so);
                L[u][1] = Buf<S>::load(rs, vo, so + axis_bytes);
                L[u][2] = Buf<S>::load(rs, vo, so + 2 * axis_bytes);
            } else {
                L[u][0] = L[u][1] = L[u][2] = 0;
            }
            if (MODE == kModeSetState) {
                Q[u][0] = Q[u][1] = Q[u][2] = 0;
                if (ok) {
                    const size_t e = first + (size_t)(u * pw + pl);
                    Q[u][0] = proj_in[e];
                    Q[u][1] = proj_in[e + np];
                    Q[u][2] = proj_in[e + 2 * (size_t)np];
                }
            }
        }
    };
    if (n_obs > 0) {
        gptr<const S> og = glob(Dp->obs);
        for (int idx = tid; idx < n_obs * kObs; idx += BLOCK) Os[idx] = og[idx];
    }
    {
        // positions of the work item's instants from the current coefficients, eq. (param):
        // X = P c in FP64 per (axis, agent) column (coefficients ascending), rounded to FP32,
        // into LDS as (x, y, z, .) (not stored: a readback forms them anew).  The basis rows of the
        // item's instants are staged in the correction area (zeroed afterwards); a column's
        // coefficients sit in registers and G = BLOCK / 3n thread groups take every G-th
        // instant, two instants' products in flight at a time.
        gptr<const double> cm = glob((const double*)Dp->c);
        const int ldc = Dp->ldc;
        double* Pl = reinterpret_cast<double*>(Acc);                    // [tc][nv]
        if (tid < tc * nv) Pl[tid] = p_first;
        for (int idx = tid + BLOCK; idx < tc * nv; idx += BLOCK) Pl[idx] = Pm[(size_t)t0 * nv + idx];
        if (MODE == kModeIter) {
            if (tid < tc * ngr) Fs[tid] = f_first;
            for (int idx = tid + BLOCK; idx < tc * ngr; idx += BLOCK) Fs[idx] = lflag[(size_t)t0 * ngr + idx];
        }
        __syncthreads();
        if (nit > 0) fetch(0, 0, first0);
        float* Xf = reinterpret_cast<float*>(Xs);
        const int n3 = 3 * n;
        const int G = max(1, BLOCK / n3);
        for (int w = tid; w < n3 * G; w += BLOCK) {
            const int g = w / n3, col = w - g * n3;
            const int a = col / n, i = col - a * n;
            gptr<const double> ci = cm + (size_t)a * ldc + (size_t)i * nv;
            auto put = [&](int tl, double x) { Xf[((size_t)tl * n + i) * 4 + a] = (S)x; };
            if constexpr (NV > 0) {
                double cv[NV];
#pragma unroll
                for (int k = 0; k < NV; ++k) cv[k] = ci[k];
                for (int tl = g; tl < tc; tl += 2 * G) {
                    int tu[2];
#pragma unroll
                    for (int u = 0; u < 2; ++u) tu[u] = min(tl + u * G, tc - 1);   // past tc: not stored
                    double x[2] = {0.0, 0.0};
#pragma unroll
                    for (int k = 0; k < NV; ++k)
#pragma unroll
                        for (int u = 0; u < 2; ++u) x[u] += Pl[tu[u] * NV + k] * cv[k];
#pragma unroll
                    for (int u = 0; u < 2; ++u)
                        if (tl + u * G < tc) put(tl + u * G, x[u]);
                }
            } else {
                for (int tl = g; tl < tc; tl += G) {
                    double x = 0.0;
                    for (int k = 0; k < nv; ++k) x += Pl[tl * nv + k] * ci[k];
                    put(tl, x);
                }
            }
        }
        __syncthreads();                                               // Pl is read before Acc is zeroed
        for (int idx = tid; idx < tc * 3 * n; idx += BLOCK) Acc[idx] = 0;
        if (tid == 0) any_general = 0;
        if (MODE == kModeIter) {
            for (int idx = tid; idx < tc * ngr; idx += BLOCK) NFs[idx] = 0u;
            for (int g = tid; g < ngr; g += BLOCK) {
                unsigned f = 0u;
                for (int tl = 0; tl < tc; ++tl) f |= Fs[tl * ngr + g];
                Gf[g] = f;
            }
            // every agent's bounding box over the item's instants (unbounded if a position is NaN)
            for (int col = tid; col < n3; col += BLOCK) {
                const int a = col / n, i = col - a * n;
                float lo = Xf[(size_t)i * 4 + a], hi = lo;
                bool bad = lo != lo;
                for (int tl = 1; tl < tc; ++tl) {
                    const float x = Xf[((size_t)tl * n + i) * 4 + a];
                    lo = fminf(lo, x);
                    hi = fmaxf(hi, x);
                    bad |= x != x;
                }
                Bs[i * 6 + 2 * a] = bad ? -INFINITY : lo;
                Bs[i * 6 + 2 * a + 1] = bad ? INFINITY : hi;
            }
        }
    }
    __syncthreads();

    // Broad phase (iterations with the plain projection and no parity outputs): a row whose
    // group has no multiplier flagged at any instant of the item and whose agents' boxes keep
    // s^2 above kBroadClear takes the far-pair shortcut at every instant, so nothing is done
    // for it.  The other rows' bits (Fb) are kept; when they are at most half the rows, only
    // they are worked through, instant by instant (the row list), else every row is, in the
    // streaming order below.
    bool use_list = false;
    if (MODE == kModeIter && !shifted && !dbg_on) {
        constexpr int nw = BLOCK / 64;
        constexpr int kPre = 8;                        // groups whose pair codes are loaded together
        int cntw = 0;
        for (int g0 = wv; g0 < ngr; g0 += nw * kPre) {
          unsigned cds[kPre];
#pragma unroll
          for (int k = 0; k < kPre; ++k) cds[k] = pairs[min(((g0 + k * nw) << 6) + lane, np - 1)];   // past np: unused
#pragma unroll
          for (int k = 0; k < kPre; ++k) {
            const int g = g0 + k * nw;
            if (g >= ngr) break;                       // uniform
            const int p = (g << 6) + lane;
            bool fail = false;
            if (p < np) {
                const unsigned cd = cds[k];
                const int i = (int)(cd & 0xffffu), j = (int)(cd >> 16);
                const S* bi = Bs + i * 6;
                S gx, gy, gz, ia2p = ia2, ib2p = ib2;
                if (!OBS || j < n) {
                    const S* bj = Bs + j * 6;
                    gx = fmaxf(0.f, fmaxf(bi[0] - bj[1], bj[0] - bi[1]));
                    gy = fmaxf(0.f, fmaxf(bi[2] - bj[3], bj[2] - bi[3]));
                    gz = fmaxf(0.f, fmaxf(bi[4] - bj[5], bj[4] - bi[5]));
                } else {
                    const S* ob = Os + (j - n) * kObs;
                    gx = fmaxf(0.f, fmaxf(bi[0] - ob[0], ob[0] - bi[1]));
                    gy = fmaxf(0.f, fmaxf(bi[2] - ob[1], ob[1] - bi[3]));
                    gz = fmaxf(0.f, fmaxf(bi[4] - ob[2], ob[2] - bi[5]));
                    ia2p = ob[3];
                    ib2p = ob[4];
                }
                const S q2g = scaled_sq(gx, gy, gz, ia2p, ib2p);
                fail = !(q2g > kBroadClear) || Gf[g] != 0u;
            }
            const unsigned long long b = __ballot(fail);
            if (lane == 0) Fb[g] = b;
            cntw += __popcll(b);
          }
        }
        if (lane == 0) wcnt[wv] = cntw;
        __syncthreads();
        int tot = 0;
        for (int w = 0; w < nw; ++w) tot += wcnt[w];
        use_list = 2 * tot <= np;
    }

    S rmax = 0, rsum = 0;
    bool general = false;
    int kc = 0, ki = 0;
    size_t f_cur = first0, c_first = first0;
    const int nit_stream = use_list ? 0 : nit;
    for (int k = 0; k < nit_stream; ++k) {
        unsigned cc[U], Flc[U];
        bool nzl[U];                                   // the row's multiplier after this pass is not +0
        S Lc[U][3], Qc[U][3];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            cc[u] = code[u];
            Flc[u] = Fl[u];
            nzl[u] = false;
            Lc[u][0] = L[u][0]; Lc[u][1] = L[u][1]; Lc[u][2] = L[u][2];
            if (MODE == kModeSetState) { Qc[u][0] = Q[u][0]; Qc[u][1] = Q[u][1]; Qc[u][2] = Q[u][2]; }
        }
        int kc1 = kc, ki1 = ki + 1;
        size_t f_nxt = f_cur + istride, c_nxt = c_first;
        if (ki1 == ntl) {
            ki1 = 0;
            ++kc1;
            c_nxt = c_first + cstride;
            f_nxt = c_nxt;
        }
        if (k + 1 < nit) fetch(kc1, ki1, f_nxt);
        const int pb = kc * cstride;
        const int tl = tgid + ki * tg;
        const size_t fc = f_cur;
        const __amdgpu_buffer_rsrc_t rs = rsrc_at(f_cur, kc);
        kc = kc1;
        ki = ki1;
        f_cur = f_nxt;
        c_first = c_nxt;
        const float4* X = Xs + (size_t)tl * n;
        long long* A = Acc + (size_t)tl * 3 * n;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int p = pb + u * pw + pl;
            if (p >= np) continue;
            const S lx = Lc[u][0], ly = Lc[u][1], lzm = Lc[u][2];
            const int i = (int)(cc[u] & 0xffffu), j = (int)(cc[u] >> 16);
            const float4 xi = X[i];
            S xj, yj, zj, ia2p = ia2, ib2p = ib2, lzp = lzl;
            if (!OBS || j < n) {
                const float4 xv = X[j];
                xj = xv.x;
                yj = xv.y;
                zj = xv.z;
            } else {
                const S* ob = Os + (j - n) * kObs;
                xj = ob[0];
                yj = ob[1];
                zj = ob[2];
                ia2p = ob[3];
                ib2p = ob[4];
                lzp = ob[5];
            }
            const S dx = xi.x - xj;
            const S dy = xi.y - yj;
            const S dz = xi.z - zj;
            // b_fc - delta of this row into the agent sums (+ for i, - for an agent j)
            auto record = [&](S cx, S cy, S cz) {
                if ((bits_of(cx) | bits_of(cy) | bits_of(cz)) == 0) return;
                const long long fx = fx_of(cx), fy = fx_of(cy), fz = fx_of(cz);
                atomicAdd((unsigned long long*)&A[i], (unsigned long long)fx);
                atomicAdd((unsigned long long*)&A[n + i], (unsigned long long)fy);
                atomicAdd((unsigned long long*)&A[2 * n + i], (unsigned long long)fz);
                if (!OBS || j < n) {
                    atomicAdd((unsigned long long*)&A[j], (unsigned long long)(-fx));
                    atomicAdd((unsigned long long*)&A[n + j], (unsigned long long)(-fy));
                    atomicAdd((unsigned long long*)&A[2 * n + j], (unsigned long long)(-fz));
                }
            };
            if (MODE == kModeSetState) {
                record(Qc[u][0] - lx * irho - dx, Qc[u][1] - ly * irho - dy, Qc[u][2] - lzm * irho - dz);
                nzl[u] = (bits_of(lx) | bits_of(ly) | bits_of(lzm)) != 0;
                continue;
            }
            const S q2 = scaled_sq(dx, dy, dz, ia2p, ib2p);              // s^2 (plain projection)
            // no multiplier (+0) and clear of the collision set by a margin: the general branch
            // gives w = 1, d e = delta, f_c = +0, lambda = +0 (not stored), b_fc = delta (no
            // correction) and a zero residual, bit for bit
            const bool clear = (q2 > S(1.0001)) & ((bits_of(lx) | bits_of(ly) | bits_of(lzm)) == 0);
            const bool fast = (MODE == kModeIter) & !shifted & !dbg_on & clear;
            if (fast) continue;
            S px, py, pz, dd;
            if (!shifted) {
                project_plain(dx, dy, dz, q2, lx, ly, lzm, irho, lzp, px, py, pz, dd);
            } else {
                // variant: project v = delta + lambda/rho; then d = max(1, s_v), d e = max(1/s_v, 1) v
                const S vx = dx + lx * irho, vy = dy + ly * irho, vz = dz + lzm * irho;
                const S q2v = (vx * vx + vy * vy) * ia2p + vz * vz * ib2p;
                if (q2v > 0) {
                    const S rs_ = Recip<S>::rsq(q2v);
                    const S w = fmax(rs_, S(1));
                    px = w * vx;
                    py = w * vy;
                    pz = w * vz;
                    dd = w * (q2v * rs_);
                } else {                                                // v = 0: e = (0, 0, l_z), d = 1
                    dd = S(1);
                    px = 0;
                    py = 0;
                    pz = lzp;
                }
            }
            S nlx = 0, nly = 0, nlz = 0;
            if (MODE == kModeIter) {
                S fn2;
                row_update(dx, dy, dz, px, py, pz, lx, ly, lzm, rho, nlx, nly, nlz, fn2);
                rmax = fmax(rmax, fn2);
                rsum += fn2;
                general = true;
                nzl[u] = (bits_of(nlx) | bits_of(nly) | bits_of(nlz)) != 0;
            }
            // an iteration stores only the multipliers whose bits change
            const int so = u * pw * (int)sizeof(S);
            if (MODE != kModeIter || bits_of(nlx) != bits_of(lx)) Buf<S>::store(nlx, rs, lane_bytes, so);
            if (MODE != kModeIter || bits_of(nly) != bits_of(ly)) Buf<S>::store(nly, rs, lane_bytes, so + axis_bytes);
            if (MODE != kModeIter || bits_of(nlz) != bits_of(lzm))
                Buf<S>::store(nlz, rs, lane_bytes, so + 2 * axis_bytes);
            record(row_correction(px, nlx, irho_b, dx), row_correction(py, nly, irho_b, dy),
                   row_correction(pz, nlz, irho_b, dz));
            if (dbg_on) {
                const size_t e = fc + (size_t)(u * pw + pl);          // (t0 + tl) 3 np + p
                if (dbg_proj_p) {
                    gptr<S> dp = glob(dbg_proj_p);
                    dp[e] = px;
                    dp[e + np] = py;
                    dp[e + 2 * (size_t)np] = pz;
                }
                if (dbg_d_p) glob(dbg_d_p)[(size_t)(t0 + tl) * np + p] = dd;
            }
        }
        // group flags after this pass: stored where they change (every group outside iterations)
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int g = (pb + u * pw + wrow) >> 6;
            const unsigned any = __ballot(nzl[u]) != 0ull ? 1u : 0u;
            if (g < ngr && (tid & 63) == 0 && (MODE != kModeIter || any != (Flc[u] != 0 ? 1u : 0u)))
                lflag[(size_t)(t0 + tl) * ngr + g] = any;
        }
    }
    if (MODE == kModeIter && use_list) {
        // The row list: a wavefront collects its groups' kept rows (row, code) in LDS, in
        // batches of at most 64 rows, and spreads each batch's rows times tc instants over
        // its lanes (instants padded to a power of two, tcp).
        constexpr int nw = BLOCK / 64;
        volatile unsigned* lq = Lq + (size_t)wv * 128;
        const int lt = tc > 1 ? 32 - __clz(tc - 1) : 0, tcp = 1 << lt;
        int R = 0;
        auto run_batch = [&]() {
            __builtin_amdgcn_wave_barrier();
            for (int e = lane; e < (R << lt); e += 64) {
                const int r = e >> lt, tl = e & (tcp - 1);
                if (tl >= tc) continue;
                const int p = (int)lq[2 * r];
                const unsigned cd = lq[2 * r + 1];
                const int g = p >> 6;
                const int i = (int)(cd & 0xffffu), j = (int)(cd >> 16);
                S xj, yj, zj, ia2p = ia2, ib2p = ib2, lzp = lzl;
                const float4 xi = Xs[(size_t)tl * n + i];
                if (!OBS || j < n) {
                    const float4 xv = Xs[(size_t)tl * n + j];
                    xj = xv.x;
                    yj = xv.y;
                    zj = xv.z;
                } else {
                    const S* ob = Os + (j - n) * kObs;
                    xj = ob[0];
                    yj = ob[1];
                    zj = ob[2];
                    ia2p = ob[3];
                    ib2p = ob[4];
                    lzp = ob[5];
                }
                const S dx = xi.x - xj;
                const S dy = xi.y - yj;
                const S dz = xi.z - zj;
                const size_t el = (size_t)(t0 + tl) * 3 * np + p;
                S lx = 0, ly = 0, lzm = 0;
                if (Fs[tl * ngr + g] != 0u) {
                    lx = lam[el];
                    ly = lam[el + np];
                    lzm = lam[el + 2 * (size_t)np];
                }
                const S q2 = scaled_sq(dx, dy, dz, ia2p, ib2p);          // s^2 (plain projection)
                if ((q2 > S(1.0001)) & ((bits_of(lx) | bits_of(ly) | bits_of(lzm)) == 0)) continue;
                S px, py, pz, dd, nlx, nly, nlz, fn2;
                project_plain(dx, dy, dz, q2, lx, ly, lzm, irho, lzp, px, py, pz, dd);
                row_update(dx, dy, dz, px, py, pz, lx, ly, lzm, rho, nlx, nly, nlz, fn2);
                rmax = fmax(rmax, fn2);
                rsum += fn2;
                general = true;
                if (bits_of(nlx) != bits_of(lx)) lam[el] = nlx;
                if (bits_of(nly) != bits_of(ly)) lam[el + np] = nly;
                if (bits_of(nlz) != bits_of(lzm)) lam[el + 2 * (size_t)np] = nlz;
                if ((bits_of(nlx) | bits_of(nly) | bits_of(nlz)) != 0) atomicOr(&NFs[tl * ngr + g], 1u);
                const S cx = row_correction(px, nlx, irho_b, dx), cy = row_correction(py, nly, irho_b, dy),
                        cz = row_correction(pz, nlz, irho_b, dz);
                if ((bits_of(cx) | bits_of(cy) | bits_of(cz)) != 0) {
                    long long* A = Acc + (size_t)tl * 3 * n;
                    const long long fx = fx_of(cx), fy = fx_of(cy), fz = fx_of(cz);
                    atomicAdd((unsigned long long*)&A[i], (unsigned long long)fx);
                    atomicAdd((unsigned long long*)&A[n + i], (unsigned long long)fy);
                    atomicAdd((unsigned long long*)&A[2 * n + i], (unsigned long long)fz);
                    if (!OBS || j < n) {
                        atomicAdd((unsigned long long*)&A[j], (unsigned long long)(-fx));
                        atomicAdd((unsigned long long*)&A[n + j], (unsigned long long)(-fy));
                        atomicAdd((unsigned long long*)&A[2 * n + j], (unsigned long long)(-fz));
                    }
                }
            }
            __builtin_amdgcn_wave_barrier();
            R = 0;
        };
        constexpr int kPre = 8;                        // groups whose pair codes are loaded together
        for (int g0 = wv; g0 < ngr; g0 += nw * kPre) {
            unsigned cds[kPre];
#pragma unroll
            for (int k = 0; k < kPre; ++k) cds[k] = pairs[min(((g0 + k * nw) << 6) + lane, np - 1)];   // past np: unused
#pragma unroll
            for (int k = 0; k < kPre; ++k) {
                const int g = g0 + k * nw;
                const unsigned long long mask = g < ngr ? Fb[g] : 0ull;
                if (mask == 0ull) continue;                             // uniform
                const int m = __popcll(mask);
                if (R + m > 64) run_batch();
                if ((mask >> lane) & 1ull) {
                    const int pos = R + __popcll(mask & ((1ull << lane) - 1ull));
                    lq[2 * pos] = (unsigned)((g << 6) + lane);
                    lq[2 * pos + 1] = cds[k];
                }
                R += m;
            }
        }
        if (R > 0) run_batch();
    }
    if (MODE == kModeIter && general) any_general = 1;
    __syncthreads();
    if (MODE == kModeIter && use_list)                   // the row list's group flags where they change
        for (int idx = tid; idx < tc * ngr; idx += BLOCK)
            if (NFs[idx] != Fs[idx]) lflag[(size_t)t0 * ngr + idx] = NFs[idx];

    // The rows' corrections of the agent sums, C_i = S_i - ((n + n_obs) X_i - sum_j X_j), of
    // the item's instants, rounded once to FP32: the linear-term kernel adds the positions'
    // part from the coefficients.  [tc][3][n] is one contiguous run of [T][3][n].
    {
        gptr<S> out = ssum + (size_t)t0 * 3 * n;
        for (int idx = tid; idx < tc * 3 * n; idx += BLOCK) out[idx] = (S)ldexp((double)Acc[idx], -kFx);
    }

    if (MODE == kModeIter) {
        __shared__ double red[2 * (BLOCK / 64)];
        if (any_general) {                          // uniform: read after the barrier
            double s1 = (double)rsum;
            const double mx = block_reduce_max_sum<S, BLOCK>(rmax, s1, red);
            if (tid == 0) {
                gptr<double> pp = part + (size_t)it.slab * 4;
                pp[0] = mx;
                pp[1] = s1;
            }
        } else if (tid == 0) {                      // every row took the shortcut: zero residual
            gptr<double> pp = part + (size_t)it.slab * 4;
            pp[0] = 0.0;
            pp[1] = 0.0;
        }
    }
}

// One workgroup per problem: X = P c (eq. (param)) at every instant, in FP64 products
// stored as S (FP64 problems; the FP32 pairwise kernel forms its own instants' positions).
// A thread owns (axis, agent) columns; the basis rows are staged in LDS in chunks.
template <typename S, int NV>
__device__ inline void positions_body(const ProblemDesc<S>* __restrict__ Dp) {
    const int n = Dp->n, nv = NV > 0 ? NV : Dp->nv, T = Dp->T, ldc = Dp->ldc;
    gptr<const double> Pm = glob(Dp->P);
    gptr<const double> cm = glob((const double*)Dp->c);
    gptr<S> Xm = glob(Dp->X);
    constexpr int kRows = 3072;                    // basis entries staged per chunk (24 KB)
    __shared__ double Ps[kRows];
    const int n3 = 3 * n;
    const int TC = kRows / nv;                     // instants per chunk (279 for 11 coefficients)
    for (int tb = 0; tb < T; tb += TC) {
        const int tn = min(TC, T - tb);
        __syncthreads();
        for (int e = threadIdx.x; e < tn * nv; e += blockDim.x) Ps[e] = Pm[(size_t)tb * nv + e];
        __syncthreads();
        for (int col = threadIdx.x; col < n3; col += blockDim.x) {
            const int a = col / n, i = col - a * n;
            gptr<const double> ci = cm + (size_t)a * ldc + (size_t)i * nv;
            if constexpr (NV > 0) {
                double cv[NV];
#pragma unroll
                for (int k = 0; k < NV; ++k) cv[k] = ci[k];
                int t = 0;
                // four instants at a time: four independent FMA chains and their LDS reads
                // in flight together
                for (; t + 4 <= tn; t += 4) {
                    double x[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int k = 0; k < NV; ++k)
#pragma unroll
                        for (int u = 0; u < 4; ++u) x[u] += Ps[(t + u) * NV + k] * cv[k];
#pragma unroll
                    for (int u = 0; u < 4; ++u) Xm[(size_t)(tb + t + u) * n3 + col] = (S)x[u];
                }
                for (; t < tn; ++t) {
                    double x = 0.0;
#pragma unroll
                    for (int k = 0; k < NV; ++k) x += Ps[t * NV + k] * cv[k];
                    Xm[(size_t)(tb + t) * n3 + col] = (S)x;
                }
            } else {
                for (int t = 0; t < tn; ++t) {
                    double x = 0.0;
                    for (int k = 0; k < nv; ++k) x += Ps[t * nv + k] * ci[k];
                    Xm[(size_t)(tb + t) * n3 + col] = (S)x;
                }
            }
        }
    }
}

template <typename S, int NV>
__global__ __launch_bounds__(256) void positions_kernel(const ProblemDesc<S>* __restrict__ probs, int mode) {
    const ProblemDesc<S>* __restrict__ Dp = probs + blockIdx.x;
    gptr<const int> ctrl = glob((const int*)Dp->ctrl);
    if (!ctrl[3]) return;
    if (mode == kModeIter && ctrl[1]) return;
    positions_body<S, NV>(Dp);
}

// One workgroup per problem: the x/y/z step of eq. (kkt_step_x) by the block structure
// of K (structured solve), then X = P c and the cost.  With the agent mean g_mean,
//     c_i = c_eq,i + M1 g_i + M2 g_mean,   M1 = K_{rho n}^{-1}, M2 = K_0^{-1} - K_{rho n}^{-1}
// (coefficient rows and columns of the per-agent inverses), all in FP64; the mean is
// summed over agents in ascending order.
template <typename S, int NV>
__global__ __launch_bounds__(256) void solve_positions_kernel(const ProblemDesc<S>* __restrict__ probs) {
    const ProblemDesc<S>* __restrict__ Dp = probs + blockIdx.x;
    gptr<const int> ctrl = glob((const int*)Dp->ctrl);
    if (!ctrl[3] || ctrl[1]) return;
    const int n = Dp->n, nv = NV > 0 ? NV : Dp->nv, ldq = Dp->ldq, ldc = Dp->ldc;
    constexpr int kGroups = 8;                      // agent groups of the partial sums of g
    __shared__ double M[2 * kMaxCoef * kMaxCoef];
    __shared__ double part[kGroups * kAxes * kMaxCoef];
    __shared__ double gm[kAxes * kMaxCoef], h[kAxes * kMaxCoef];
    gptr<const double> Sm = glob(Dp->smat);
    for (int e = threadIdx.x; e < 2 * nv * nv; e += blockDim.x) M[e] = Sm[e];
    gptr<const double> q = glob((const double*)Dp->q);
    const int m3 = kAxes * nv;
    const int ng = max(1, min(kGroups, (int)blockDim.x / m3));
    // g_mean: agents i = grp, grp + ng, ... summed per group, then the groups in order
    for (int o = threadIdx.x; o < ng * m3; o += blockDim.x) {
        const int grp = o / m3, ak = o - grp * m3;
        const int a = ak / nv, k = ak - a * nv;
        gptr<const double> qa = q + (size_t)a * ldq + k;
        double sacc = 0.0;
#pragma unroll 4
        for (int i = grp; i < n; i += ng) sacc += qa[(size_t)i * nv];
        part[grp * m3 + ak] = sacc;
    }
    __syncthreads();
    const double inv_n = 1.0 / (double)n;
    for (int o = threadIdx.x; o < m3; o += blockDim.x) {
        double sacc = 0.0;
        for (int grp = 0; grp < ng; ++grp) sacc += part[grp * m3 + o];
        gm[o] = sacc * inv_n;
    }
    __syncthreads();
    for (int o = threadIdx.x; o < m3; o += blockDim.x) {
        const int a = o / nv, k = o - a * nv;
        double v = 0.0;
        for (int l = 0; l < nv; ++l) v += M[nv * nv + k * nv + l] * gm[a * nv + l];
        h[o] = v;
    }
    __syncthreads();
    gptr<double> c = glob(Dp->c);
    gptr<const double> ceq = glob((const double*)Dp->ceq);
    const int nc = n * nv;
    for (int o = threadIdx.x; o < kAxes * nc; o += blockDim.x) {      // one output coefficient each
        const int a = o / nc, rem = o - a * nc;
        const int i = rem / nv, k = rem - i * nv;
        gptr<const double> gi = q + (size_t)a * ldq + (size_t)i * nv;
        double v = 0.0;
        if constexpr (NV > 0) {
#pragma unroll
            for (int l = 0; l < NV; ++l) v += M[k * NV + l] * gi[l];
        } else {
            for (int l = 0; l < nv; ++l) v += M[k * nv + l] * gi[l];
        }
        const size_t oc = (size_t)a * ldc + rem;
        c[oc] = ceq[oc] + h[a * nv + k] + v;
    }
    if constexpr (!std::is_same<S, float>::value) {
        __syncthreads();                   // c is read back by other threads of this workgroup
        positions_body<S, NV>(Dp);
    }
}

// One workgroup per problem: g = rho P^T S (FP64) into q[a][0 .. n*nv) (and its FP32
// copy), then in iteration mode the residual record of this iteration and the
// convergence test.  A thread owns one (axis, agent) column of S and produces its
// nv coefficients.  FP32 problems hold only the corrections C of S: their P^T S_i is
// P^T C_i + P^T P ((n + n_obs) c_i - sum_j c_j), the second part from the coefficients.
template <typename S, int NV>
__global__ __launch_bounds__(256) void qbuild_kernel(const ProblemDesc<S>* __restrict__ probs, int mode) {
    const ProblemDesc<S>* __restrict__ Dp = probs + blockIdx.x;
    gptr<int> ctrl = glob(Dp->ctrl);
    if (!ctrl[3]) return;
    if (mode == kModeIter && ctrl[1]) return;
    const int n = Dp->n, nv = NV > 0 ? NV : Dp->nv, T = Dp->T, ldq = Dp->ldq;
    // the linear term of the next x-step: the next stage's rho on a stage's last iteration
    const double rho = (mode == kModeIter && Dp->switch_at > 0 && ctrl[0] + 1 == Dp->switch_at) ? Dp->rho_next : Dp->rho;
    gptr<const double> Pm = glob(Dp->P);
    gptr<const S> ss = glob((const S*)Dp->ssum);
    gptr<double> q = glob(Dp->q);
    gptr<float> qf = glob(Dp->qf);
    const int n3 = 3 * n;
    constexpr bool kCorr = std::is_same<S, float>::value;   // ssum holds C, not S
    // FP32 problems: the positions' part P^T P ((n + n_obs) c_i - sum_j c_j) per column, from the
    // columns' coefficients staged in LDS (dynamic, [3n][nv]), which then hold the part itself
    extern __shared__ double cxs[];
    __shared__ double PtPs[kCorr ? kMaxCoef * kMaxCoef : 1], csum[kCorr ? kAxes * kMaxCoef : 1];
    if constexpr (kCorr) {
        gptr<const double> cm = glob((const double*)Dp->c);
        gptr<const double> Gm = glob(Dp->PtP);
        const int ldc = Dp->ldc;
        const double nn = (double)(n + Dp->n_obs);
        for (int e = threadIdx.x; e < nv * nv; e += blockDim.x) PtPs[e] = Gm[e];
        for (int e = threadIdx.x; e < n3 * nv; e += blockDim.x) {
            const int col = e / nv, l = e - col * nv, a = col / n, i = col - a * n;
            cxs[e] = cm[(size_t)a * ldc + (size_t)i * nv + l];
        }
        __syncthreads();
        // sum over agents: groups of agents g, g + 7, ... first, then the groups in order
        constexpr int kGroups = 7;
        __shared__ double cpart[kGroups * kAxes * kMaxCoef];
        const int m3 = kAxes * nv;
        for (int o = threadIdx.x; o < kGroups * m3; o += blockDim.x) {
            const int grp = o / m3, al = o - grp * m3;
            const int a = al / nv, l = al - a * nv;
            double sacc = 0.0;
            for (int i = grp; i < n; i += kGroups) sacc += cxs[((size_t)a * n + i) * nv + l];
            cpart[o] = sacc;
        }
        __syncthreads();
        for (int o = threadIdx.x; o < m3; o += blockDim.x) {
            double sacc = cpart[o];
            for (int grp = 1; grp < kGroups; ++grp) sacc += cpart[grp * m3 + o];
            csum[o] = sacc;
        }
        __syncthreads();
        constexpr int NVC = NV > 0 ? NV : kMaxCoef;
        for (int col = threadIdx.x; col < n3; col += blockDim.x) {
            const int a = col / n;
            double* cc = cxs + (size_t)col * nv;
            double v[NVC];
#pragma unroll
            for (int l = 0; l < NVC; ++l) v[l] = (NV > 0 || l < nv) ? nn * cc[l] - csum[a * nv + l] : 0.0;
#pragma unroll 1
            for (int k = 0; k < nv; ++k) {
                double x = 0.0;
#pragma unroll
                for (int l = 0; l < NVC; ++l)
                    if (NV > 0 || l < nv) x += PtPs[k * nv + l] * v[l];
                cc[k] = x;                               // own column only: no other thread reads it
            }
        }
    }
    if constexpr (NV > 0) {
        // A thread owns columns tid and tid + 256 (3n <= 480); the basis rows are staged in
        // LDS in chunks and each column's S values are loaded 8 instants at a time.
        static_assert(3 * MATO_MAX_AGENTS <= 512, "two columns per thread of a 256-thread workgroup");
        constexpr int kRows = 2048;
        constexpr int TC = kRows / NV;
        __shared__ double Ps[kRows];
        double acc[2][NV];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int k = 0; k < NV; ++k) acc[h][k] = 0.0;
        for (int tb = 0; tb < T; tb += TC) {
            const int tn = min(TC, T - tb);
            __syncthreads();
            for (int e = threadIdx.x; e < tn * NV; e += blockDim.x) Ps[e] = Pm[(size_t)tb * NV + e];
            __syncthreads();
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int col = threadIdx.x + h * 256;
                if (col >= n3) continue;
                gptr<const S> sp = ss + (size_t)tb * n3 + col;     // [(t*3 + a)*n + i] = t*3n + col
                int t = 0;
                // 8 instants per step, the next 8 loaded while these are multiplied out
                S sv[8], sn[8];
                if (tn >= 8) {
#pragma unroll
                    for (int u = 0; u < 8; ++u) sv[u] = sp[(size_t)u * n3];
                }
                for (; t + 8 <= tn; t += 8) {
                    const bool more = t + 16 <= tn;
                    if (more) {
#pragma unroll
                        for (int u = 0; u < 8; ++u) sn[u] = sp[(size_t)(t + 8 + u) * n3];
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const double su = (double)sv[u];
#pragma unroll
                        for (int k = 0; k < NV; ++k) acc[h][k] += Ps[(t + u) * NV + k] * su;
                    }
                    if (more) {
#pragma unroll
                        for (int u = 0; u < 8; ++u) sv[u] = sn[u];
                    }
                }
                for (; t < tn; ++t) {
                    const double sv = (double)sp[(size_t)t * n3];
#pragma unroll
                    for (int k = 0; k < NV; ++k) acc[h][k] += Ps[t * NV + k] * sv;
                }
            }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int col = threadIdx.x + h * 256;
            if (col >= n3) continue;
            const int a = col / n, i = col - a * n;
            const size_t o = (size_t)a * ldq + (size_t)i * nv;
#pragma unroll
            for (int k = 0; k < NV; ++k) {
                const double gk = kCorr ? rho * (cxs[(size_t)col * NV + k] + acc[h][k]) : rho * acc[h][k];
                q[o + k] = gk;
                qf[o + k] = (float)gk;
            }
        }
    } else {
      for (int col = threadIdx.x; col < n3; col += blockDim.x) {
        const int a = col / n, i = col - a * n;
        gptr<const S> sp = ss + col;                 // [(t*3 + a)*n + i] = t*3n + col
        const size_t o = (size_t)a * ldq + (size_t)i * nv;
        {
            for (int k = 0; k < nv; ++k) {
                double acc = 0.0;
                if constexpr (kCorr) acc = cxs[(size_t)col * nv + k];
                for (int t = 0; t < T; ++t) acc += Pm[(size_t)t * nv + k] * (double)sp[(size_t)t * n3];
                q[o + k] = rho * acc;
                qf[o + k] = (float)(rho * acc);
            }
        }
      }
    }
    if (mode == kModeIter) {
        // The smoothness cost of eq. (cost_proposed) of the current coefficients:
        // sum_t (Pddot c)^2 of a column is the quadratic form c^T (Pddot^T Pddot) c, n_v^2
        // products per column instead of T n_v; columns strided per thread, then the tree.
        __shared__ double G[kMaxCoef * kMaxCoef];
        gptr<const double> Gm = glob(Dp->PddtPdd);
        gptr<const double> cm = glob((const double*)Dp->c);
        const int ldc = Dp->ldc;
        for (int e = threadIdx.x; e < nv * nv; e += blockDim.x) G[e] = Gm[e];
        __syncthreads();
        double z = 0.0;
        for (int col = threadIdx.x; col < n3; col += blockDim.x) {
            const int a = col / n, i = col - a * n;
            gptr<const double> ci = cm + (size_t)a * ldc + (size_t)i * nv;
            if constexpr (NV > 0) {
                double cv[NV];
#pragma unroll
                for (int k = 0; k < NV; ++k) cv[k] = ci[k];
                // FP32 problems: the column's own copy in LDS (its slot of the staged positions
                // part, no longer read) for the loop over k (not unrolled), an LDS read per k
                // instead of a global one
                double* cl = kCorr ? cxs + (size_t)col * NV : nullptr;
                if constexpr (kCorr) {
#pragma unroll
                    for (int k = 0; k < NV; ++k) cl[k] = cv[k];
                }
#pragma unroll 1
                for (int k = 0; k < NV; ++k) {
                    double gk = 0.0;
#pragma unroll
                    for (int l = 0; l < NV; ++l) gk += G[k * NV + l] * cv[l];
                    z += (kCorr ? cl[k] : (double)ci[k]) * gk;    // == cv[k]
                }
            } else {
                for (int k = 0; k < nv; ++k) {
                    double gk = 0.0;
                    for (int l = 0; l < nv; ++l) gk += G[k * nv + l] * ci[l];
                    z += ci[k] * gk;
                }
            }
        }
        // residual partials of the pairwise work items: strided per thread, then a fixed tree
        gptr<const double> part = glob((const double*)Dp->part);
        const int nslab = Dp->nslab;
        double mx = 0.0, s1 = 0.0;
        for (int k = threadIdx.x; k < nslab; k += blockDim.x) {
            mx = fmax(mx, part[(size_t)k * 4 + 0]);
            s1 += part[(size_t)k * 4 + 1];
        }
        __shared__ double red[3 * 4];
        block_reduce3<double, 256>(mx, s1, z, red);
        if (threadIdx.x != 0) return;
        gptr<double> hist = glob(Dp->hist);
        const double s2 = z;
        const int itn = ctrl[0];
        const double rmax = sqrt(mx);
        {
            // the first hist_cap - 1 iterations, then the last entry follows the latest one
            const size_t h = (size_t)min(itn, Dp->hist_cap - 1) * 3;
            hist[h + 0] = rmax;
            hist[h + 1] = sqrt(s1 / ((double)Dp->np * (double)T));
            hist[h + 2] = s2;
        }
        ctrl[0] = itn + 1;
        if (!isfinite(s1) || !isfinite(s2)) {
            ctrl[2] = 1;
            ctrl[1] = 1;
        } else if (Dp->tol > 0.0 && rmax < Dp->tol) {
            ctrl[4] = 1;
            ctrl[1] = 1;
        } else if (Dp->iter_cap > 0 && itn + 1 >= Dp->iter_cap) {
            ctrl[1] = 1;
        }
    }
}

// grid (problems, 3 axes): r = g - H c in FP64 (and its FP32 copy).  The boundary
// rows of the correction are not formed: K11^{-1} A^T = 0, and the boundary
// coefficients of c come from c_eq exactly.
template <typename S>
__global__ __launch_bounds__(256) void residual_kernel(const ProblemDesc<S>* __restrict__ probs) {
    const ProblemDesc<S>* __restrict__ Dp = probs + blockIdx.x;
    gptr<const int> ctrl = glob((const int*)Dp->ctrl);
    if (!ctrl[3] || ctrl[1]) return;
    const int a = blockIdx.y;
    const int n = Dp->n, nv = Dp->nv, ldq = Dp->ldq;
    const double rho = Dp->rho;
    gptr<const double> c = glob((const double*)Dp->c) + (size_t)a * Dp->ldc;
    gptr<const double> q = glob((const double*)Dp->q) + (size_t)a * ldq;
    gptr<double> r = glob(Dp->r) + (size_t)a * ldq;
    gptr<float> rf = glob(Dp->rf) + (size_t)a * ldq;
    __shared__ double csum[kMaxCoef];
    __shared__ double PtP[kMaxCoef * kMaxCoef], PddtPdd[kMaxCoef * kMaxCoef];
    __shared__ double cs[kMaxCoef * MATO_MAX_AGENTS];
    gptr<const double> gPtP = glob(Dp->PtP), gPddtPdd = glob(Dp->PddtPdd);
    for (int e = threadIdx.x; e < nv * nv; e += blockDim.x) {
        PtP[e] = gPtP[e];
        PddtPdd[e] = gPddtPdd[e];
    }
    for (int e = threadIdx.x; e < n * nv; e += blockDim.x) cs[e] = c[e];
    __syncthreads();
    if (threadIdx.x < nv) {
        double s = 0.0;
        for (int j = 0; j < n; ++j) s += cs[j * nv + threadIdx.x];
        csum[threadIdx.x] = s;
    }
    __syncthreads();
    const double nr = (double)(n + Dp->n_obs) * rho;        // diagonal weight: agent pairs and obstacles
    for (int o = threadIdx.x; o < n * nv; o += blockDim.x) {
        const int i = o / nv, k = o - i * nv;
        const double* ci = cs + i * nv;
        double h = 0.0;
        for (int l = 0; l < nv; ++l)
            h += PddtPdd[k * nv + l] * ci[l] + PtP[k * nv + l] * (nr * ci[l] - rho * csum[l]);
        const double v = q[o] - h;
        if constexpr (std::is_same<S, double>::value) r[o] = v;    // the FP64 product's operand
        else rf[o] = (float)v;                                     // the MFMA products' operand
    }
}

// grid (problems, 3 axes): c_eq = K12^{-1} b_eq in FP64 (b_eq has the start in row 0
// and the goal in row 3 of each agent's six boundary rows, zeros elsewhere).
template <typename S>
__global__ __launch_bounds__(256) void ceq_kernel(const ProblemDesc<S>* __restrict__ probs,
                                                  const double* const* __restrict__ kinv) {
    const ProblemDesc<S>* __restrict__ Dp = probs + blockIdx.x;
    gptr<const int> ctrl = glob((const int*)Dp->ctrl);
    if (!ctrl[3]) return;
    const int a = blockIdx.y;
    const int n = Dp->n, nv = Dp->nv, M = n * nv, N = n * (nv + kNb);
    gptr<const double> beq = glob((const double*)Dp->q) + (size_t)a * Dp->ldq + M;
    gptr<double> ceq = glob(Dp->ceq) + (size_t)a * Dp->ldc;
    if (Dp->smat) {
        // structured: c_eq,i = E0 b_mean + En (b_i - b_mean), the b_eq columns of K_0^{-1}, K_{rho n}^{-1}
        __shared__ double bm[kNb];
        if (threadIdx.x < kNb) {
            double s = 0.0;
            for (int i = 0; i < n; ++i) s += beq[(size_t)i * kNb + threadIdx.x];
            bm[threadIdx.x] = s / (double)n;
        }
        __syncthreads();
        gptr<const double> E0 = glob(Dp->smat) + 2 * nv * nv;
        gptr<const double> En = E0 + nv * kNb;
        for (int m = threadIdx.x; m < M; m += blockDim.x) {
            const int i = m / nv, k = m - i * nv;
            double v = 0.0;
            for (int r = 0; r < kNb; ++r)
                v += E0[k * kNb + r] * bm[r] + En[k * kNb + r] * (beq[(size_t)i * kNb + r] - bm[r]);
            ceq[m] = v;
        }
        return;
    }
    gptr<const double> K = glob(kinv[blockIdx.x]);
    for (int m = threadIdx.x; m < M; m += blockDim.x) {
        gptr<const double> row = K + (size_t)m * N + M;
        double v = 0.0;
        for (int i = 0; i < n; ++i) v += row[i * kNb + 0] * beq[i * kNb + 0] + row[i * kNb + 3] * beq[i * kNb + 3];
        ceq[m] = v;
    }
}

// grid (problems): c_i = K0^{-1}[c rows, b_eq columns] b_eq,i for every agent and axis.
template <typename S>
__global__ __launch_bounds__(256) void init_kernel(const ProblemDesc<S>* __restrict__ probs,
                                                   const double* const* __restrict__ k0c) {
    const ProblemDesc<S>* __restrict__ Dp = probs + blockIdx.x;
    gptr<const int> ctrl = glob((const int*)Dp->ctrl);
    if (!ctrl[3]) return;
    const int n = Dp->n, nv = Dp->nv, ldq = Dp->ldq, ldc = Dp->ldc;
    gptr<const double> K0 = glob(k0c[blockIdx.x]);
    gptr<const double> q = glob((const double*)Dp->q);
    gptr<double> c = glob(Dp->c);
    for (int o = threadIdx.x; o < 3 * n * nv; o += blockDim.x) {
        const int a = o / (n * nv);
        const int rem = o - a * n * nv;
        const int i = rem / nv, k = rem - i * nv;
        gptr<const double> beq = q + (size_t)a * ldq + (size_t)n * nv + (size_t)i * kNb;
        double v = 0.0;
        for (int bb = 0; bb < kNb; ++bb) v += K0[k * kNb + bb] * beq[bb];
        c[(size_t)a * ldc + rem] = v;
    }
}

// ------------------------------------------------------------- launchers ---
template <typename S, int NV, int MODE, bool OBS>
static hipError_t launch_pw(const WorkItem* items, int nitems, const ProblemDesc<S>* probs, int threads,
                            size_t lds, hipStream_t st) {
    switch (threads) {
        case 256:
            pairwise_kernel<S, 256, NV, MODE, OBS><<<nitems, 256, lds, st>>>(items, probs);
            break;
        case 512:
            pairwise_kernel<S, 512, NV, MODE, OBS><<<nitems, 512, lds, st>>>(items, probs);
            break;
        default:
            pairwise_kernel<S, 1024, NV, MODE, OBS><<<nitems, 1024, lds, st>>>(items, probs);
            break;
    }
    return hipGetLastError();
}

template <typename S, int NV>
static hipError_t launch_pw_mode(const WorkItem* items, int nitems, const ProblemDesc<S>* probs, int mode, bool obs,
                                 int threads, size_t lds, hipStream_t st) {
    if (mode == kModeIter)
        return obs ? launch_pw<S, NV, kModeIter, true>(items, nitems, probs, threads, lds, st)
                   : launch_pw<S, NV, kModeIter, false>(items, nitems, probs, threads, lds, st);
    if (mode == kModeInit) return launch_pw<S, NV, kModeInit, true>(items, nitems, probs, threads, lds, st);
    return launch_pw<S, NV, kModeSetState, true>(items, nitems, probs, threads, lds, st);
}

template <int NV, int MODE, bool OBS>
static hipError_t launch_fx(const WorkItem* items, int nitems, const ProblemDesc<float>* probs, int threads,
                            size_t lds, hipStream_t st) {
    switch (threads) {
        case 256:
            pairwise_fx_kernel<256, NV, MODE, OBS><<<nitems, 256, lds, st>>>(items, probs);
            break;
        case 512:
            pairwise_fx_kernel<512, NV, MODE, OBS><<<nitems, 512, lds, st>>>(items, probs);
            break;
        default:
            pairwise_fx_kernel<1024, NV, MODE, OBS><<<nitems, 1024, lds, st>>>(items, probs);
            break;
    }
    return hipGetLastError();
}

template <int NV>
static hipError_t launch_fx_mode(const WorkItem* items, int nitems, const ProblemDesc<float>* probs, int mode, bool obs,
                                 int threads, size_t lds, hipStream_t st) {
    if (mode == kModeIter)
        return obs ? launch_fx<NV, kModeIter, true>(items, nitems, probs, threads, lds, st)
                   : launch_fx<NV, kModeIter, false>(items, nitems, probs, threads, lds, st);
    if (mode == kModeInit) return launch_fx<NV, kModeInit, true>(items, nitems, probs, threads, lds, st);
    return launch_fx<NV, kModeSetState, true>(items, nitems, probs, threads, lds, st);
}

// nv: the (common) number of basis coefficients of the launch's problems, or 0 if they differ.
// FP32 problems take the fixed-point kernel, FP64 problems the direct one.
template <typename S>
hipError_t launch_pairwise(const WorkItem* items, int nitems, const ProblemDesc<S>* probs, int mode,
                           int threads, size_t lds, int nv, bool obs, hipStream_t st) {
    if (nitems <= 0) return hipSuccess;
    if constexpr (std::is_same<S, float>::value) {
        if (nv == 11) return launch_fx_mode<11>(items, nitems, probs, mode, obs, threads, lds, st);
        return launch_fx_mode<0>(items, nitems, probs, mode, obs, threads, lds, st);
    } else {
        if (nv == 11) return launch_pw_mode<S, 11>(items, nitems, probs, mode, obs, threads, lds, st);
        return launch_pw_mode<S, 0>(items, nitems, probs, mode, obs, threads, lds, st);
    }
}

template <typename S, int NV, int MODE, bool OBS>
static hipError_t set_lds_one(size_t lds) {
    hipError_t e = hipFuncSetAttribute((const void*)pairwise_kernel<S, 256, NV, MODE, OBS>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void*)pairwise_kernel<S, 512, NV, MODE, OBS>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)pairwise_kernel<S, 1024, NV, MODE, OBS>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <typename S, int NV>
static hipError_t set_lds_nv(size_t lds) {
    hipError_t e = set_lds_one<S, NV, kModeIter, false>(lds);
    if (e != hipSuccess) return e;
    e = set_lds_one<S, NV, kModeIter, true>(lds);
    if (e != hipSuccess) return e;
    e = set_lds_one<S, NV, kModeInit, true>(lds);
    if (e != hipSuccess) return e;
    return set_lds_one<S, NV, kModeSetState, true>(lds);
}

template <int NV, int MODE, bool OBS>
static hipError_t set_lds_fx1(size_t lds) {
    hipError_t e = hipFuncSetAttribute((const void*)pairwise_fx_kernel<256, NV, MODE, OBS>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void*)pairwise_fx_kernel<512, NV, MODE, OBS>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)pairwise_fx_kernel<1024, NV, MODE, OBS>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <int MODE, bool OBS>
static hipError_t set_lds_fx(size_t lds) {
    hipError_t e = set_lds_fx1<11, MODE, OBS>(lds);
    if (e != hipSuccess) return e;
    return set_lds_fx1<0, MODE, OBS>(lds);
}

template <typename S>
hipError_t set_pairwise_lds_limit(size_t lds) {
    if constexpr (std::is_same<S, float>::value) {
        hipError_t e = set_lds_fx<kModeIter, false>(lds);
        if (e != hipSuccess) return e;
        e = set_lds_fx<kModeIter, true>(lds);
        if (e != hipSuccess) return e;
        e = set_lds_fx<kModeInit, true>(lds);
        if (e != hipSuccess) return e;
        return set_lds_fx<kModeSetState, true>(lds);
    } else {
        hipError_t e = set_lds_nv<S, 11>(lds);
        if (e != hipSuccess) return e;
        return set_lds_nv<S, 0>(lds);
    }
}

template <typename S>
hipError_t launch_qbuild(const ProblemDesc<S>* probs, int nprob, int mode, int nv, int nmax, hipStream_t st) {
    if (nprob <= 0) return hipSuccess;
    // FP32: the coefficients of every (axis, agent) column of the largest problem in LDS
    const size_t lds = std::is_same<S, float>::value ? sizeof(double) * 3 * (size_t)nmax * (nv > 0 ? nv : kMaxCoef) : 0;
    if (nv == 11)
        qbuild_kernel<S, 11><<<nprob, 256, lds, st>>>(probs, mode);
    else
        qbuild_kernel<S, 0><<<nprob, 256, lds, st>>>(probs, mode);
    return hipGetLastError();
}

template <typename S>
hipError_t launch_positions(const ProblemDesc<S>* probs, int nprob, int mode, int nv, hipStream_t st) {
    if (nprob <= 0) return hipSuccess;
    if (nv == 11)
        positions_kernel<S, 11><<<nprob, 256, 0, st>>>(probs, mode);
    else
        positions_kernel<S, 0><<<nprob, 256, 0, st>>>(probs, mode);
    return hipGetLastError();
}

template <typename S>
hipError_t launch_residual(const ProblemDesc<S>* probs, int nprob, hipStream_t st) {
    if (nprob <= 0) return hipSuccess;
    residual_kernel<S><<<dim3(nprob, 3), 256, 0, st>>>(probs);
    return hipGetLastError();
}

template <typename S>
hipError_t launch_ceq(const ProblemDesc<S>* probs, const double* const* kinv, int nprob, hipStream_t st) {
    if (nprob <= 0) return hipSuccess;
    ceq_kernel<S><<<dim3(nprob, 3), 256, 0, st>>>(probs, kinv);
    return hipGetLastError();
}

template <typename S>
hipError_t launch_solve_positions(const ProblemDesc<S>* probs, int nprob, int nv, hipStream_t st) {
    if (nprob <= 0) return hipSuccess;
    if (nv == 11)
        solve_positions_kernel<S, 11><<<nprob, 256, 0, st>>>(probs);
    else
        solve_positions_kernel<S, 0><<<nprob, 256, 0, st>>>(probs);
    return hipGetLastError();
}

template <typename S>
hipError_t launch_init(const ProblemDesc<S>* probs, const double* const* k0c, int nprob, hipStream_t st) {
    if (nprob <= 0) return hipSuccess;
    init_kernel<S><<<nprob, 256, 0, st>>>(probs, k0c);
    return hipGetLastError();
}

template hipError_t launch_pairwise<float>(const WorkItem*, int, const ProblemDesc<float>*, int, int, size_t, int, bool,
                                          hipStream_t);
template hipError_t launch_pairwise<double>(const WorkItem*, int, const ProblemDesc<double>*, int, int, size_t, int, bool,
                                           hipStream_t);
template hipError_t set_pairwise_lds_limit<float>(size_t);
template hipError_t set_pairwise_lds_limit<double>(size_t);
template hipError_t launch_qbuild<float>(const ProblemDesc<float>*, int, int, int, int, hipStream_t);
template hipError_t launch_qbuild<double>(const ProblemDesc<double>*, int, int, int, int, hipStream_t);
template hipError_t launch_positions<float>(const ProblemDesc<float>*, int, int, int, hipStream_t);
template hipError_t launch_positions<double>(const ProblemDesc<double>*, int, int, int, hipStream_t);
template hipError_t launch_residual<float>(const ProblemDesc<float>*, int, hipStream_t);
template hipError_t launch_residual<double>(const ProblemDesc<double>*, int, hipStream_t);
template hipError_t launch_ceq<float>(const ProblemDesc<float>*, const double* const*, int, hipStream_t);
template hipError_t launch_ceq<double>(const ProblemDesc<double>*, const double* const*, int, hipStream_t);
template hipError_t launch_solve_positions<float>(const ProblemDesc<float>*, int, int, hipStream_t);
template hipError_t launch_solve_positions<double>(const ProblemDesc<double>*, int, int, hipStream_t);
template hipError_t launch_init<float>(const ProblemDesc<float>*, const double* const*, int, hipStream_t);
template hipError_t launch_init<double>(const ProblemDesc<double>*, const double* const*, int, hipStream_t);

}  // namespace mato
