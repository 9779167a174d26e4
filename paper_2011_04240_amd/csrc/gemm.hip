// The x/y/z QP step through the precomputed inverse, eq. (kkt_step_x) and
// Remarks 1-2: for every right-hand side (problem, axis) of a same-plan group
//     c = c_eq + K11^{-1} g,     c_eq = K12^{-1} b_eq       (c-rows of K^{-1} q~),
// one dense (11n x 11n) x (11n x 3B) product per iteration for B problems; c_eq
// is formed once per problem in FP64.  With accumulate = 1 the same product is
// applied to the FP64 refinement residual g - H c and added to c (K11^{-1} A^T = 0,
// so the boundary multipliers nu are not needed for the correction).
//
// Tiles are 64 rows x 64 (or 48) right-hand sides, computed as 16 x 16 MFMA output blocks.
//   gemm_f32_tile   v_mfma_f32_16x16x4_f32, FP32 operands, FP32 accumulation.
//   gemm_bf16_tile  v_mfma_f32_16x16x32_bf16 over three-term BF16 splits of both
//                   operands (the six products down to 2^-16 relative), FP32 accumulation.
//   gemm_f64        FP64 FMA (the reference-precision path).
// The MFMA kernels read the FP32 copy of the right-hand sides (the BF16 kernel
// splits it on the way into LDS); the product is added to the FP64
// coefficients in the epilogue.
#include "common.h"

namespace mato {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short ushortx8 __attribute__((ext_vector_type(8)));

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

// What the tile kernels keep of right-hand side col0 + lane from the prologue: its FP32
// operand, its destination c, the value the product is added to (c when accumulating,
// c_eq otherwise) and whether it is still iterating.  Columns past the group alias column 0.
struct ColRef {
    const float* bf;
    double* c;
    const double* src;
    int live;
};

__device__ inline ColRef col_ref(const GemmGroup& G, const GemmCol* __restrict__ cols, int col, int accumulate) {
    const int cidx = col < G.ncols ? col : 0;
    const GemmCol cc = cols[G.first_col + cidx];
    return ColRef{cc.bf, cc.c, accumulate ? cc.c : cc.ceq, (col < G.ncols && cc.ctrl[3] && !cc.ctrl[1]) ? 1 : 0};
}

__device__ inline unsigned long long shfl_u64(unsigned long long x, int from) {
    const int lo = __shfl((int)(unsigned)x, from), hi = __shfl((int)(unsigned)(x >> 32), from);
    return ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
}

// The output of wavefront wq is NB 16 x 16 blocks: lane (m, g) holds rows
// m0 + 16 wq + 4 g + r (r = 0..3) of right-hand side col0 + 16 j + m.  A column's pointers
// come from lane 16 j + m, which loaded them in the prologue.  load_old requests the values
// the product is added to for all blocks together (rows past M clamped, their results
// dropped) at the start of the last K step, so that they arrive while it runs; store_tile
// writes c = old + v.
template <int NB>
__device__ inline void load_old(const GemmTile& t, const GemmGroup& G, const ColRef& me, int wq, int lane,
                                double (&old)[NB][4]) {
    const int m = lane & 15, g = lane >> 4;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const double* src = (const double*)shfl_u64((unsigned long long)me.src, j * 16 + m);
#pragma unroll
        for (int r = 0; r < 4; ++r) old[j][r] = src[min(t.m0 + wq * 16 + 4 * g + r, G.M - 1)];
    }
}

template <int NB>
__device__ inline void store_tile(const GemmTile& t, const GemmGroup& G, const ColRef& me, int wq, int lane,
                                  const double (&old)[NB][4], const float (&v)[NB][4]) {
    const int m = lane & 15, g = lane >> 4;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        double* dst = (double*)shfl_u64((unsigned long long)me.c, j * 16 + m);
        const int live = __shfl(me.live, j * 16 + m);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = t.m0 + wq * 16 + 4 * g + r;
            if (live && row < G.M) dst[row] = old[j][r] + (double)v[j][r];
        }
    }
}

// FP32 product over tiles of 64 rows x 16 NB right-hand sides (NB = 4: 64, NB = 3: 48,
// the width chosen when it balances the tiles over the compute units better, e.g. 704
// instead of 528 tiles at n = 64 and 1024 problems).  Wavefront wq of a group of four owns
// rows 16 wq .. 16 wq + 15 and all NB blocks of 16 x 16 MFMA outputs, so the rows of
// K11^{-1} go straight from global memory into the lanes that multiply them: lane (m, g)
// loads row m0 + 16 wq + m at k = 8 g .. 8 g + 7 of the 32-wide K step, one step ahead.
// The right-hand sides are shared by the four wavefronts and go through two LDS stages:
// thread (wq, lr) loads right-hand side col0 + lr at k-slice [8 wq, 8 wq + 8) two steps
// ahead and stores it into the [column][k] stage (k stride kLDK: the 16 lanes of a read
// hit disjoint banks) one step ahead, one barrier per step.  MFMA kk (0..7) of a step
// takes k = 8 g + kk in lane group g.  The even and the odd K steps accumulate apart and
// are added at the end, so that NG = 2 groups of four wavefronts (512 threads, one group
// per parity: half the chain of steps, for launches with fewer tiles than compute units)
// and NG = 1 give the same bits.  Every output takes the same MFMA sequence at either
// width, so both widths give the same bits.
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
    constexpr int STAGE = NC * kLDK;                    // floats per stage: B [NC][kLDK]
    constexpr int NA = 3 - NG;                          // accumulator sets per wavefront: 2 (NG = 1) or 1
    const GemmTile t = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    const GemmGroup G = groups[t.group];
    __shared__ __align__(16) float smem[NG * 2 * STAGE];
    const int tid = threadIdx.x, grp = NG == 2 ? tid >> 8 : 0, gt = tid & 255;
    const int lane = gt & 63, wq = gt >> 6;
    const int lr = lane, kq = wq * 8;
    float* stg = smem + grp * 2 * STAGE;
    const ColRef me = col_ref(G, cols, t.col0 + lr, accumulate);
    const gcfloat brow = (gcfloat)me.bf + kq;
    if (!__syncthreads_or(me.live && lr < NC)) return;  // every right-hand side of the tile converged
    const int m = lane & 15, g8 = (lane >> 4) * 8;
    const gcfloat arow = (gcfloat)G.Ahi + (size_t)(t.m0 + wq * 16 + m) * G.ldk + g8;
    const int nk = G.ldk / 32;
    const int nsteps = (nk + NG - 1) / NG;              // steps per group (group 1 may idle on the last)
    floatx4 acc[NA][NB];
#pragma unroll
    for (int h = 0; h < NA; ++h)
#pragma unroll
        for (int j = 0; j < NB; ++j) acc[h][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    // two register sets each for A (the step's, the next step's in flight) and B (in
    // flight to the next stage, being fetched), named statically in a loop of two steps per
    // trip, so that no loaded register is copied (a copy waits for its load)
    floatx4 a0[2], a1[2], b0[2], b1[2];
    auto kstep = [&](int s) { return min(NG * s + grp, nk - 1) * 32; };   // past the last: reload it (unused)
    auto fetchA = [&](int s, floatx4 (&a)[2]) {          // group step s is K step NG s + grp
        a[0] = *(gcfloat4)(arow + kstep(s));
        a[1] = *(gcfloat4)(arow + kstep(s) + 4);
    };
    auto fetchB = [&](int s, floatx4 (&b)[2]) {
        b[0] = *(gcfloat4)(brow + kstep(s));
        b[1] = *(gcfloat4)(brow + kstep(s) + 4);
    };
    auto store = [&](int s, const floatx4 (&b)[2]) {
        float* Bs = stg + (s & 1) * STAGE;
        if (lr < NC) {
            *(floatx4*)(Bs + lr * kLDK + kq) = b[0];
            *(floatx4*)(Bs + lr * kLDK + kq + 4) = b[1];
        }
    };
    auto mult = [&](int s, floatx4 (&ac)[NB], const floatx4 (&a)[2]) {
        const float* Bs = stg + (s & 1) * STAGE;
        const float av[8] = {a[0][0], a[0][1], a[0][2], a[0][3], a[1][0], a[1][1], a[1][2], a[1][3]};
        float bv[NB][8];
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const floatx4 c0 = *(const floatx4*)(Bs + (j * 16 + m) * kLDK + g8);
            const floatx4 c1 = *(const floatx4*)(Bs + (j * 16 + m) * kLDK + g8 + 4);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                bv[j][e] = c0[e];
                bv[j][e + 4] = c1[e];
            }
        }
        // the NB accumulators interleaved: independent MFMAs back to back
#pragma unroll
        for (int kk = 0; kk < 8; ++kk)
#pragma unroll
            for (int j = 0; j < NB; ++j)
                ac[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[kk], bv[j][kk], ac[j], 0, 0, 0);
    };
    auto step = [&](int s, floatx4 (&ac)[NB], const floatx4 (&acur)[2], floatx4 (&anext)[2],
                    const floatx4 (&bstore)[2], floatx4 (&bfetch)[2]) {
        fetchA(s + 1, anext);                            // unconditional: past the end it reloads
        if (NG == 1 || NG * s + grp < nk) mult(s, ac, acur);    // the last step, so that the
        if (s + 1 < nsteps) store(s + 1, bstore);              // count of loads in flight is the
        fetchB(s + 2, bfetch);                                 // same on every path
        __syncthreads();
    };
    fetchA(0, a0);
    fetchB(0, b0);
    store(0, b0);
    fetchB(1, b1);
    __syncthreads();
    // the last step is taken after the addends of the epilogue are requested (48-column
    // tiles; at 64 columns their registers would cost a wavefront per SIMD)
    double old[NB][4];
    int s = 0;
    if constexpr (NB == 3) {
        for (; s + 2 < nsteps; s += 2) {
            step(s, acc[0], a0, a1, b1, b0);
            step(s + 1, acc[NA - 1], a1, a0, b0, b1);
        }
        if (s + 1 < nsteps) {
            step(s, acc[0], a0, a1, b1, b0);
            load_old<NB>(t, G, me, wq, lane, old);
            step(s + 1, acc[NA - 1], a1, a0, b0, b1);
        } else {
            load_old<NB>(t, G, me, wq, lane, old);
            step(s, acc[0], a0, a1, b1, b0);
        }
    } else {
        for (; s + 1 < nsteps; s += 2) {
            step(s, acc[0], a0, a1, b1, b0);
            step(s + 1, acc[NA - 1], a1, a0, b0, b1);
        }
        if (s < nsteps) step(s, acc[0], a0, a1, b1, b0);
        load_old<NB>(t, G, me, wq, lane, old);
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
    float v[NB][4];
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            v[j][r] = acc[0][j][r] + (NG == 2 ? red[((wq * NB + j) * 4 + r) * 64 + lane] : acc[NA - 1][j][r]);
    store_tile<NB>(t, G, me, wq, lane, old, v);
}

// The three BF16 terms of eight FP32 values, hi = bf16(x), mid = bf16(x - hi),
// lo = bf16(x - hi - mid), with the device's round-to-nearest-even conversion: exact
// (8 + 8 + 8 significant bits), every difference exact in FP32.
__device__ inline void split8x3(const floatx4& x0, const floatx4& x1, ushortx8& hi, ushortx8& mid, ushortx8& lo) {
    const float v[8] = {x0[0], x0[1], x0[2], x0[3], x1[0], x1[1], x1[2], x1[3]};
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const __bf16 h = (__bf16)v[e];
        const float r1 = v[e] - (float)h;
        const __bf16 m = (__bf16)r1;
        hi[e] = __builtin_bit_cast(unsigned short, h);
        mid[e] = __builtin_bit_cast(unsigned short, m);
        lo[e] = __builtin_bit_cast(unsigned short, (__bf16)(r1 - (float)m));
    }
}

// Three-term BF16 split of both operands, A = Ah + Am + Al (from the FP64 inverse) and
// B = Bh + Bm + Bl (exact for the FP32 right-hand side): six v_mfma_f32_16x16x32_bf16
// per 16 x 16 block and K step (hh, hm, mh, hl, lh, mm); the dropped terms (ml, lm, ll)
// are below 2^-23 of |A||B|, so the product carries FP32's precision at BF16 MFMA rates.
// Tiles, stages and accumulation as in gemm_f32_tile: 64 rows x 16 NB right-hand sides,
// wavefront wq owns rows 16 wq .. 16 wq + 15 and loads the three terms of its rows straight
// into the MFMA lanes (lane (m, g): row m0 + 16 wq + m, k = 8 g .. 8 g + 7 of the step, one
// step ahead); the right-hand sides go through two LDS stages with one barrier per 32-wide
// K step, split into their three terms on the way in (thread (wq, lr): right-hand side
// col0 + lr, k-slice [8 wq, 8 wq + 8)); the even and the odd steps accumulate apart
// (NG = 2: one group of four wavefronts per parity, same bits).  Each staged column holds
// 32 bf16 (64 bytes, no padding) as four 16-byte chunks; chunk c of column r sits at
// position c ^ ((r >> 2) & 3), so the 16 columns x 4 chunks a wavefront reads for one MFMA
// operand fall on distinct banks in every group of 16 lanes.
template <int NB, int NG>
__global__ __launch_bounds__(256 * NG) void gemm_bf16_tile(const GemmTile* __restrict__ tiles,
                                                           const GemmGroup* __restrict__ groups,
                                                           const GemmCol* __restrict__ cols, int accumulate) {
    constexpr int NC = 16 * NB;
    constexpr int RW = 32;                              // bf16 per staged column
    constexpr int PB = NC * RW;                         // one term's plane
    constexpr int STAGE = 3 * PB;                       // bf16 per stage: Bh Bm Bl
    constexpr int NA = 3 - NG;
    const GemmTile t = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    const GemmGroup G = groups[t.group];
    __shared__ __align__(16) unsigned short smem[NG * 2 * STAGE];
    const int tid = threadIdx.x, grp = NG == 2 ? tid >> 8 : 0, gt = tid & 255;
    const int lane = gt & 63, wq = gt >> 6;
    const int lr = lane, kq = wq * 8;
    unsigned short* stg = smem + grp * 2 * STAGE;
    const ColRef me = col_ref(G, cols, t.col0 + lr, accumulate);
    const gcfloat brow = (gcfloat)me.bf + kq;
    if (!__syncthreads_or(me.live && lr < NC)) return;  // every right-hand side of the tile converged
    const int m = lane & 15;
    const size_t aoff = (size_t)(t.m0 + wq * 16 + m) * G.ldk + (lane >> 4) * 8;
    typedef __attribute__((address_space(1))) const ushortx8* gcush8;
    typedef __attribute__((address_space(1))) const unsigned short* gcush;
    const gcush ah = (gcush)G.Ahi + aoff, am = (gcush)G.Amid + aoff, al = (gcush)G.Alo + aoff;
    const int nk = G.ldk / 32;
    const int nsteps = (nk + NG - 1) / NG;
    const int wslot = (wq ^ ((lr >> 2) & 3)) * 8;       // this thread's chunk in its staged column
    floatx4 acc[NA][NB];
#pragma unroll
    for (int h = 0; h < NA; ++h)
#pragma unroll
        for (int j = 0; j < NB; ++j) acc[h][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    // register sets named statically in a loop of two steps per trip, as in gemm_f32_tile
    ushortx8 a0[3], a1[3];                              // A terms: the step's, the next step's
    floatx4 b0[2], b1[2];                               // B: to the next stage, being fetched
    auto kstep = [&](int s) { return min(NG * s + grp, nk - 1) * 32; };   // past the last: reload it (unused)
    auto fetchA = [&](int s, ushortx8 (&a)[3]) {
        a[0] = *(gcush8)(ah + kstep(s));
        a[1] = *(gcush8)(am + kstep(s));
        a[2] = *(gcush8)(al + kstep(s));
    };
    auto fetchB = [&](int s, floatx4 (&b)[2]) {
        b[0] = *(gcfloat4)(brow + kstep(s));
        b[1] = *(gcfloat4)(brow + kstep(s) + 4);
    };
    auto store = [&](int s, const floatx4 (&b)[2]) {
        unsigned short* Bs = stg + (s & 1) * STAGE;
        if (lr < NC) {
            ushortx8 t3[3];
            split8x3(b[0], b[1], t3[0], t3[1], t3[2]);
#pragma unroll
            for (int p = 0; p < 3; ++p) *(ushortx8*)(Bs + p * PB + lr * RW + wslot) = t3[p];
        }
    };
    auto mult = [&](int s, floatx4 (&ac)[NB], const ushortx8 (&ca)[3]) {
        const unsigned short* Bs = stg + (s & 1) * STAGE;
        const int rslot = ((lane >> 4) ^ ((m >> 2) & 3)) * 8;
        bf16x8 a[3], b[3][NB];
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            a[p] = __builtin_bit_cast(bf16x8, ca[p]);
#pragma unroll
            for (int j = 0; j < NB; ++j)
                b[p][j] = __builtin_bit_cast(bf16x8, *(const ushortx8*)(Bs + p * PB + (j * 16 + m) * RW + rslot));
        }
        // products in the order hh, hm, mh, hl, lh, mm; the NB blocks interleaved
        constexpr int pa[6] = {0, 0, 1, 0, 2, 1}, pb[6] = {0, 1, 0, 2, 0, 1};
#pragma unroll
        for (int q = 0; q < 6; ++q)
#pragma unroll
            for (int j = 0; j < NB; ++j)
                ac[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[pa[q]], b[pb[q]][j], ac[j], 0, 0, 0);
    };
    auto step = [&](int s, floatx4 (&ac)[NB], const ushortx8 (&acur)[3], ushortx8 (&anext)[3],
                    const floatx4 (&bstore)[2], floatx4 (&bfetch)[2]) {
        fetchA(s + 1, anext);                            // unconditional: past the end it reloads
        if (NG == 1 || NG * s + grp < nk) mult(s, ac, acur);    // the last step, so that the
        if (s + 1 < nsteps) store(s + 1, bstore);              // count of loads in flight is the
        fetchB(s + 2, bfetch);                                 // same on every path
        __syncthreads();
    };
    fetchA(0, a0);
    fetchB(0, b0);
    store(0, b0);
    fetchB(1, b1);
    __syncthreads();
    // the last step is taken after the addends of the epilogue are requested (48-column
    // tiles; at 64 columns their registers would cost a wavefront per SIMD)
    double old[NB][4];
    int s = 0;
    if constexpr (NB == 3) {
        for (; s + 2 < nsteps; s += 2) {
            step(s, acc[0], a0, a1, b1, b0);
            step(s + 1, acc[NA - 1], a1, a0, b0, b1);
        }
        if (s + 1 < nsteps) {
            step(s, acc[0], a0, a1, b1, b0);
            load_old<NB>(t, G, me, wq, lane, old);
            step(s + 1, acc[NA - 1], a1, a0, b0, b1);
        } else {
            load_old<NB>(t, G, me, wq, lane, old);
            step(s, acc[0], a0, a1, b1, b0);
        }
    } else {
        for (; s + 1 < nsteps; s += 2) {
            step(s, acc[0], a0, a1, b1, b0);
            step(s + 1, acc[NA - 1], a1, a0, b0, b1);
        }
        if (s < nsteps) step(s, acc[0], a0, a1, b1, b0);
        load_old<NB>(t, G, me, wq, lane, old);
    }
    float* red = reinterpret_cast<float*>(smem);
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
    float v[NB][4];
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            v[j][r] = acc[0][j][r] + (NG == 2 ? red[((wq * NB + j) * 4 + r) * 64 + lane] : acc[NA - 1][j][r]);
    store_tile<NB>(t, G, me, wq, lane, old, v);
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
    else if (precision == MATO_BF16_REFINED) {
        if (width == kW48) {
            if (split) gemm_bf16_tile<3, 2><<<ntiles, 512, 0, st>>>(tiles, groups, cols, accumulate);
            else gemm_bf16_tile<3, 1><<<ntiles, 256, 0, st>>>(tiles, groups, cols, accumulate);
        } else {
            if (split) gemm_bf16_tile<4, 2><<<ntiles, 512, 0, st>>>(tiles, groups, cols, accumulate);
            else gemm_bf16_tile<4, 1><<<ntiles, 256, 0, st>>>(tiles, groups, cols, accumulate);
        }
    }
    else
        gemm_f64<<<ntiles, 256, 0, st>>>(tiles, groups, cols, accumulate);
    return hipGetLastError();
}

}  // namespace mato
