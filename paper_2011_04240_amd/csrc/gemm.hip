// The x/y/z QP step through the precomputed inverse, eq. (kkt_step_x) and
// Remarks 1-2: for every right-hand side (problem, axis) of a same-plan group
//     c = c_eq + K11^{-1} g,     c_eq = K12^{-1} b_eq       (c-rows of K^{-1} q~),
// one dense (11n x 11n) x (11n x 3B) product per iteration for B problems; c_eq
// is formed once per problem in FP64.  With accumulate = 1 the same product is
// applied to the FP64 refinement residual g - H c and added to c (K11^{-1} A^T = 0,
// so the boundary multipliers nu are not needed for the correction).
//
// Tiles are 64 rows x 64 (or 48) right-hand sides, computed as 16 x 16 MFMA output blocks.
//   gemm_f32_tile  v_mfma_f32_16x16x4_f32, FP32 operands, FP32 accumulation.
//   gemm_bf16  v_mfma_f32_16x16x32_bf16 over three-term BF16 splits of both
//              operands (the six products down to 2^-16 relative), FP32 accumulation.
//   gemm_f64   FP64 FMA (the reference-precision path).
// The MFMA kernels read the FP32 copy of the right-hand sides (the BF16 kernel
// splits it on the way into LDS); the product is added to the FP64
// coefficients in the epilogue.
#include "common.h"

namespace mato {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short ushortx8 __attribute__((ext_vector_type(8)));

__device__ inline unsigned short f2bf_rne(float x) {
    unsigned int u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ inline float bf2f(unsigned short h) { return __uint_as_float(((unsigned int)h) << 16); }

// The tile list holds the 64-row tiles of one 64-column block consecutively and workgroups
// take tiles through xcd_tile: the right-hand sides of a column block are fetched into one
// L2 instead of eight.

struct TileCols {
    const double* bptr;
    const float* bfptr;
    bool active;
};

__device__ inline TileCols load_col(const GemmGroup& G, const GemmCol* __restrict__ cols, int col) {
    TileCols r{nullptr, nullptr, false};
    if (col < G.ncols) {
        const GemmCol cc = cols[G.first_col + col];
        r.bptr = cc.b;
        r.bfptr = cc.bf;
        r.active = cc.ctrl[3] && !cc.ctrl[1];
    }
    return r;
}

__device__ inline void store_out(const GemmGroup& G, const GemmCol* __restrict__ cols, int row, int col,
                                 double v, int accumulate) {
    if (row >= G.M || col >= G.ncols) return;
    const GemmCol cc = cols[G.first_col + col];
    if (!cc.ctrl[3] || cc.ctrl[1]) return;
    double* c = cc.c + row;
    *c = (accumulate ? *c : cc.ceq[row]) + v;
}

// Both MFMA kernels use 512 threads: two groups of four wavefronts walk the even and
// the odd 32-wide K steps of the same 64 x 64 output tile (each group with its own
// LDS stage), and the two partial tiles are added in a fixed order at the end.
// In a group, lane `lr` (0..63) of wavefront w loads row m0 + lr of K11^{-1} and
// right-hand side col0 + lr, k-slice [8w, 8w + 8) of the step; the next step is
// fetched into registers while the current one is multiplied out of LDS.  Right-hand
// sides past the group's last column alias column 0 (their results are discarded).
__device__ inline const float* col_ptr(const GemmGroup& G, const GemmCol* __restrict__ cols, int col,
                                       bool& active) {
    const int cidx = col < G.ncols ? col : 0;
    const GemmCol cc = cols[G.first_col + cidx];
    active = col < G.ncols && cc.ctrl[3] && !cc.ctrl[1];
    return cc.bf;
}

// Epilogue: group 1 hands its partial tile to group 0 through LDS, group 0 adds it
// and writes c (+)= result for the active right-hand sides.
__device__ inline void finish_tile(const GemmTile& t, const GemmGroup& G, const GemmCol* __restrict__ cols,
                                   floatx4 (&acc)[2][2], float* red, int grp, int wq, int lane, int accumulate) {
    const int wm = wq >> 1, wn = wq & 1;
    __syncthreads();
    if (grp == 1) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) red[((wq * 4 + i * 2 + j) * 4 + r) * 64 + lane] = acc[i][j][r];
    }
    __syncthreads();
    if (grp != 0) return;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int col = t.col0 + wn * 32 + j * 16 + (lane & 15);
        if (col >= G.ncols) continue;
        const GemmCol cc = cols[G.first_col + col];
        if (!cc.ctrl[3] || cc.ctrl[1]) continue;
        double old[2][4];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = t.m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + r;
                old[i][r] = row < G.M ? (accumulate ? cc.c[row] : cc.ceq[row]) : 0.0;
            }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = t.m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + r;
                const float v = acc[i][j][r] + red[((wq * 4 + i * 2 + j) * 4 + r) * 64 + lane];
                if (row < G.M) cc.c[row] = old[i][r] + (double)v;
            }
    }
}

// FP32 product over tiles of 64 rows x 16 NB right-hand sides (NB = 4: 64, NB = 3: 48,
// the width chosen when it balances the tiles over the compute units better, e.g. 704
// instead of 528 tiles at n = 64 and 1024 problems).  Wavefront wq of a group of four owns
// rows 16 wq .. 16 wq + 15 and all NB blocks of 16 x 16 MFMA outputs.  The 32-wide K steps
// go through two LDS stages: the next step is stored while the current one is multiplied,
// one barrier per step, and the step after next is already being loaded.  The even and
// the odd K steps accumulate apart and are added at the end, so that NG = 2 groups of
// four wavefronts (512 threads, one group per parity: half the chain of steps, for
// launches with fewer tiles than compute units) and NG = 1 give the same bits.
// Staging: thread (wq, lr) loads row m0 + lr of K11^{-1} and right-hand side col0 + lr
// at k-slice [8 wq, 8 wq + 8) of the step and stores each as two 16-byte words into the
// [row][k] stage (k stride kLDK: the 16 lanes of a read hit disjoint banks).  MFMA kk
// (0..7) of a step takes k = 8 g + kk in lane group g = lane / 16, so a lane reads its
// eight k of a row as two 16-byte words.  Every output takes the same MFMA sequence at
// either width, so both widths give the same bits.
constexpr int kW48 = 48;
constexpr int kLDK = 36;
// operands are read through the global address space, so that the loads are global (not
// flat) loads and waiting for LDS does not also wait for them
typedef __attribute__((address_space(1))) const float* gcfloat;
typedef __attribute__((address_space(1))) const floatx4* gcfloat4;

template <int NB, int NG>
__global__ __launch_bounds__(256 * NG) void gemm_f32_tile(const GemmTile* __restrict__ tiles,
                                                          const GemmGroup* __restrict__ groups,
                                                          const GemmCol* __restrict__ cols, int accumulate) {
    constexpr int NC = 16 * NB;                         // right-hand sides per tile
    constexpr int STAGE = (64 + NC) * kLDK;             // floats per stage: A [64][kLDK], B [NC][kLDK]
    constexpr int NA = 3 - NG;                          // accumulator sets per wavefront: 2 (NG = 1) or 1
    const GemmTile t = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    const GemmGroup G = groups[t.group];
    __shared__ __align__(16) float smem[NG * 2 * STAGE];
    const int tid = threadIdx.x, grp = NG == 2 ? tid >> 8 : 0, gt = tid & 255;
    const int lane = gt & 63, wq = gt >> 6;
    const int lr = lane, kq = wq * 8;
    float* stg = smem + grp * 2 * STAGE;
    bool act;
    const gcfloat brow = (gcfloat)col_ptr(G, cols, t.col0 + lr, act) + kq;
    if (!__syncthreads_or(act && lr < NC)) return;      // every right-hand side of the tile converged
    const gcfloat arow = (gcfloat)G.Ahi + (size_t)(t.m0 + lr) * G.ldk + kq;
    const int nk = G.ldk / 32;
    const int nsteps = (nk + NG - 1) / NG;              // steps per group (group 1 may idle on the last)
    floatx4 acc[NA][NB];
#pragma unroll
    for (int h = 0; h < NA; ++h)
#pragma unroll
        for (int j = 0; j < NB; ++j) acc[h][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    floatx4 ra0, ra1, rb0, rb1;
    auto fetch = [&](int s) {                            // group step s is K step NG s + grp
        const int k0 = min(NG * s + grp, nk - 1) * 32;   // past the last: reload it (unused)
        ra0 = *(gcfloat4)(arow + k0);
        ra1 = *(gcfloat4)(arow + k0 + 4);
        rb0 = *(gcfloat4)(brow + k0);
        rb1 = *(gcfloat4)(brow + k0 + 4);
    };
    auto store = [&](int s) {
        float* As = stg + (s & 1) * STAGE;
        float* Bs = As + 64 * kLDK;
        *(floatx4*)(As + lr * kLDK + kq) = ra0;
        *(floatx4*)(As + lr * kLDK + kq + 4) = ra1;
        if (lr < NC) {
            *(floatx4*)(Bs + lr * kLDK + kq) = rb0;
            *(floatx4*)(Bs + lr * kLDK + kq + 4) = rb1;
        }
    };
    auto mult = [&](int s, floatx4 (&ac)[NB]) {
        const float* As = stg + (s & 1) * STAGE;
        const float* Bs = As + 64 * kLDK;
        const int m = lane & 15, g8 = (lane >> 4) * 8;
        const floatx4 a0 = *(const floatx4*)(As + (wq * 16 + m) * kLDK + g8);
        const floatx4 a1 = *(const floatx4*)(As + (wq * 16 + m) * kLDK + g8 + 4);
        const float av[8] = {a0[0], a0[1], a0[2], a0[3], a1[0], a1[1], a1[2], a1[3]};
        float bv[NB][8];
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const floatx4 b0 = *(const floatx4*)(Bs + (j * 16 + m) * kLDK + g8);
            const floatx4 b1 = *(const floatx4*)(Bs + (j * 16 + m) * kLDK + g8 + 4);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                bv[j][e] = b0[e];
                bv[j][e + 4] = b1[e];
            }
        }
        // the NB accumulators interleaved: independent MFMAs back to back
#pragma unroll
        for (int kk = 0; kk < 8; ++kk)
#pragma unroll
            for (int j = 0; j < NB; ++j)
                ac[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[kk], bv[j][kk], ac[j], 0, 0, 0);
    };
    fetch(0);
    store(0);
    if (nsteps > 1) fetch(1);
    __syncthreads();
    for (int s = 0; s < nsteps; ++s) {
        if (NG == 1 || NG * s + grp < nk) {
            if (NA == 2 && (s & 1)) mult(s, acc[NA - 1]);
            else mult(s, acc[0]);
        }
        if (s + 1 < nsteps) store(s + 1);
        if (s + 2 < nsteps) fetch(s + 2);
        __syncthreads();
    }
    // the odd steps' partial tile: the second accumulator set, or group 1's through LDS (the
    // stages are free after the last barrier); even + odd, then c (+)= result
    float* red = smem;
    if (NG == 2) {
        if (grp == 1) {
#pragma unroll
            for (int j = 0; j < NB; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) red[((wq * NB + j) * 4 + r) * 64 + lane] = acc[0][j][r];
        }
        __syncthreads();
        if (grp != 0) return;
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const int col = t.col0 + j * 16 + (lane & 15);
        if (col >= G.ncols) continue;
        const GemmCol cc = cols[G.first_col + col];
        if (!cc.ctrl[3] || cc.ctrl[1]) continue;
        double old[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = t.m0 + wq * 16 + 4 * (lane >> 4) + r;
            old[r] = row < G.M ? (accumulate ? cc.c[row] : cc.ceq[row]) : 0.0;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = t.m0 + wq * 16 + 4 * (lane >> 4) + r;
            const float odd = NG == 2 ? red[((wq * NB + j) * 4 + r) * 64 + lane] : acc[NA - 1][j][r];
            const float v = acc[0][j][r] + odd;
            if (row < G.M) cc.c[row] = old[r] + (double)v;
        }
    }
}

// An FP32 value as the sum of three bf16 terms, hi = bf16(x), mid = bf16(x - hi),
// lo = bf16(x - hi - mid): exact (8 + 8 + 8 significant bits), each difference exact in FP32.
__device__ inline void split8x3(const float4& x0, const float4& x1, ushortx8& hi, ushortx8& mid, ushortx8& lo) {
    const float v[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const unsigned short h = f2bf_rne(v[e]);
        const float r1 = v[e] - bf2f(h);
        const unsigned short m = f2bf_rne(r1);
        hi[e] = h;
        mid[e] = m;
        lo[e] = f2bf_rne(r1 - bf2f(m));
    }
}

// Three-term BF16 split of both operands, A = Ah + Am + Al (from the FP64 inverse) and
// B = Bh + Bm + Bl (exact for the FP32 right-hand side): six v_mfma_f32_16x16x32_bf16
// per block and step (hh, hm, mh, hl, lh, mm); the dropped terms (ml, lm, ll) are below
// 2^-23 of |A||B|, so the product carries FP32's precision at BF16 MFMA rates.
__global__ __launch_bounds__(512) void gemm_bf16(const GemmTile* __restrict__ tiles,
                                                 const GemmGroup* __restrict__ groups,
                                                 const GemmCol* __restrict__ cols, int accumulate) {
    const GemmTile t = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    const GemmGroup G = groups[t.group];
    constexpr int LDH = 40;                                   // [row][k] stride in bf16 elements
    constexpr int PL = 64 * LDH;                              // one staged plane
    __shared__ __align__(16) unsigned short smem[2 * 6 * PL];
    const int tid = threadIdx.x, grp = tid >> 8, gt = tid & 255;
    const int lane = gt & 63, wq = gt >> 6;
    const int wm = wq >> 1, wn = wq & 1;
    const int lr = gt & 63, kq = (gt >> 6) * 8;
    unsigned short* As = smem + grp * 6 * PL;                 // Ah, Am, Al, Bh, Bm, Bl
    unsigned short* Bs = As + 3 * PL;
    bool act;
    const float* brow = col_ptr(G, cols, t.col0 + lr, act) + kq;
    if (!__syncthreads_or(act)) return;
    const size_t aoff = (size_t)(t.m0 + lr) * G.ldk + kq;
    const unsigned short* ahi = (const unsigned short*)G.Ahi + aoff;
    const unsigned short* amd = (const unsigned short*)G.Amid + aoff;
    const unsigned short* alo = (const unsigned short*)G.Alo + aoff;
    const int nk = G.ldk / 32;
    const int nsteps = (nk + 1) / 2;
    floatx4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    ushortx8 vh, vm, vl;
    float4 rb0, rb1;
    auto fetch = [&](int s) {
        const int k0 = (2 * s + grp) * 32;
        if (k0 < G.ldk) {
            vh = *(const ushortx8*)(ahi + k0);
            vm = *(const ushortx8*)(amd + k0);
            vl = *(const ushortx8*)(alo + k0);
            rb0 = *(const float4*)(brow + k0);
            rb1 = *(const float4*)(brow + k0 + 4);
        }
    };
    fetch(0);
    for (int s = 0; s < nsteps; ++s) {
        const bool valid = (2 * s + grp) < nk;
        ushortx8 bh, bm, bl;
        if (valid) split8x3(rb0, rb1, bh, bm, bl);
        __syncthreads();
        if (valid) {
            *(ushortx8*)&As[lr * LDH + kq] = vh;
            *(ushortx8*)&As[PL + lr * LDH + kq] = vm;
            *(ushortx8*)&As[2 * PL + lr * LDH + kq] = vl;
            *(ushortx8*)&Bs[lr * LDH + kq] = bh;
            *(ushortx8*)&Bs[PL + lr * LDH + kq] = bm;
            *(ushortx8*)&Bs[2 * PL + lr * LDH + kq] = bl;
        }
        __syncthreads();
        if (s + 1 < nsteps) fetch(s + 1);
        if (valid) {
            const int kb = 8 * (lane >> 4);
            bf16x8 a[3][2], b[3][2];
#pragma unroll
            for (int p = 0; p < 3; ++p) {
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    const int m = wm * 32 + i * 16 + (lane & 15);
                    a[p][i] = __builtin_bit_cast(bf16x8, *(const ushortx8*)&As[p * PL + m * LDH + kb]);
                }
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const int c = wn * 32 + j * 16 + (lane & 15);
                    b[p][j] = __builtin_bit_cast(bf16x8, *(const ushortx8*)&Bs[p * PL + c * LDH + kb]);
                }
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    floatx4 x = acc[i][j];
                    x = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][i], b[0][j], x, 0, 0, 0);
                    x = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][i], b[1][j], x, 0, 0, 0);
                    x = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][i], b[0][j], x, 0, 0, 0);
                    x = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][i], b[2][j], x, 0, 0, 0);
                    x = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2][i], b[0][j], x, 0, 0, 0);
                    x = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][i], b[1][j], x, 0, 0, 0);
                    acc[i][j] = x;
                }
        }
    }
    finish_tile(t, G, cols, acc, reinterpret_cast<float*>(smem), grp, wq, lane, accumulate);
}

__global__ __launch_bounds__(256) void gemm_f64(const GemmTile* __restrict__ tiles,
                                                const GemmGroup* __restrict__ groups,
                                                const GemmCol* __restrict__ cols, int accumulate) {
    const GemmTile t = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    const GemmGroup G = groups[t.group];
    __shared__ double As[16][65];   // [k][m]
    __shared__ double Bs[16][65];   // [k][rhs]
    const int tid = threadIdx.x;
    const int lr = tid >> 2, kc = (tid & 3) * 4;
    const TileCols bc = load_col(G, cols, t.col0 + lr);
    if (!__syncthreads_or(bc.active)) return;
    const double* arow = (const double*)G.Ahi + (size_t)(t.m0 + lr) * G.ldk + kc;
    const int tr = (tid >> 4) * 4, tcol = (tid & 15) * 4;
    double acc[4][4] = {};
    for (int k0 = 0; k0 < G.ldk; k0 += 16) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            As[kc + e][lr] = arow[k0 + e];
            Bs[kc + e][lr] = bc.active ? bc.bptr[k0 + kc + e] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            double a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[k][tr + i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Bs[k][tcol + j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) store_out(G, cols, t.m0 + tr + i, t.col0 + tcol + j, acc[i][j], accumulate);
}

static int device_cus() {
    static int cus = 0;
    if (cus == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
    }
    return cus;
}

hipError_t launch_gemm(int precision, int width, const GemmTile* tiles, int ntiles, const GemmGroup* groups,
                       const GemmCol* cols, int accumulate, hipStream_t st) {
    if (ntiles <= 0) return hipSuccess;
    // fewer tiles than compute units: two groups of wavefronts per tile, one per K parity
    const bool split = ntiles < device_cus();
    if (precision == MATO_FP32 && width == kW48) {
        if (split) gemm_f32_tile<3, 2><<<ntiles, 512, 0, st>>>(tiles, groups, cols, accumulate);
        else gemm_f32_tile<3, 1><<<ntiles, 256, 0, st>>>(tiles, groups, cols, accumulate);
    } else if (precision == MATO_FP32) {
        if (split) gemm_f32_tile<4, 2><<<ntiles, 512, 0, st>>>(tiles, groups, cols, accumulate);
        else gemm_f32_tile<4, 1><<<ntiles, 256, 0, st>>>(tiles, groups, cols, accumulate);
    }
    else if (precision == MATO_BF16_REFINED)
        gemm_bf16<<<ntiles, 512, 0, st>>>(tiles, groups, cols, accumulate);
    else
        gemm_f64<<<ntiles, 256, 0, st>>>(tiles, groups, cols, accumulate);
    return hipGetLastError();
}

}  // namespace mato
