// The x/y/z QP step through the precomputed inverse, eq. (kkt_step_x) and
// Remarks 1-2: for every right-hand side (problem, axis) of a same-plan group
//     c (+)= [K11^{-1} | K12^{-1}] [g ; b_eq]           (c-rows of K^{-1} q~),
// one dense (11n x 17n) x (17n x 3B) product per iteration for B problems.
// With accumulate = 1 the same product is applied to the FP64 refinement
// residual [g - H c ; b_eq - A c] and added to c (K11^{-1} A^T = 0, so the
// boundary multipliers nu are not needed for the correction).
//
// Tiles are 64 rows x 64 right-hand sides; 256 threads = 4 wavefronts, each
// owning a 32 x 32 quadrant computed as 2 x 2 blocks of 16 x 16 MFMA outputs.
//   gemm_f32   v_mfma_f32_16x16x4_f32, FP32 operands, FP32 accumulation.
//   gemm_bf16  v_mfma_f32_16x16x32_bf16 over two-term BF16 splits of both
//              operands (hi*hi + hi*lo + lo*hi), FP32 accumulation.
//   gemm_f64   FP64 FMA (the reference-precision path).
// Right-hand sides are FP64 in memory and rounded on the way into LDS; the
// product is added to the FP64 coefficients in the epilogue.
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

struct TileCols {
    const double* bptr;
    bool active;
};

__device__ inline TileCols load_col(const GemmGroup& G, const GemmCol* __restrict__ cols, int col) {
    TileCols r{nullptr, false};
    if (col < G.ncols) {
        const GemmCol cc = cols[G.first_col + col];
        r.bptr = cc.b;
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
    *c = accumulate ? *c + v : v;
}

__global__ __launch_bounds__(256) void gemm_f32(const GemmTile* __restrict__ tiles,
                                                const GemmGroup* __restrict__ groups,
                                                const GemmCol* __restrict__ cols, int accumulate) {
    const GemmTile t = tiles[blockIdx.x];
    const GemmGroup G = groups[t.group];
    __shared__ float As[32][68];   // [k][m]
    __shared__ float Bs[32][68];   // [k][rhs]
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w >> 1, wn = w & 1;
    const int lr = tid >> 2, kc = (tid & 3) * 8;     // loader: row / rhs lr, k-chunk kc
    const TileCols bc = load_col(G, cols, t.col0 + lr);
    if (!__syncthreads_or(bc.active)) return;        // every right-hand side converged
    const float* arow = (const float*)G.Ahi + (size_t)(t.m0 + lr) * G.ldk + kc;
    floatx4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

    for (int k0 = 0; k0 < G.ldk; k0 += 32) {
        const float4 a0 = *(const float4*)(arow + k0);
        const float4 a1 = *(const float4*)(arow + k0 + 4);
        double bv[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) bv[e] = bc.active ? bc.bptr[k0 + kc + e] : 0.0;
        As[kc + 0][lr] = a0.x; As[kc + 1][lr] = a0.y; As[kc + 2][lr] = a0.z; As[kc + 3][lr] = a0.w;
        As[kc + 4][lr] = a1.x; As[kc + 5][lr] = a1.y; As[kc + 6][lr] = a1.z; As[kc + 7][lr] = a1.w;
#pragma unroll
        for (int e = 0; e < 8; ++e) Bs[kc + e][lr] = (float)bv[e];
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 32; kk += 4) {
            const int kr = kk + (lane >> 4);
            float af[2], bf[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) af[i] = As[kr][wm * 32 + i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < 2; ++j) bf[j] = Bs[kr][wn * 32 + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i], bf[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = t.m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + r;
                const int col = t.col0 + wn * 32 + j * 16 + (lane & 15);
                store_out(G, cols, row, col, (double)acc[i][j][r], accumulate);
            }
}

__global__ __launch_bounds__(256) void gemm_bf16(const GemmTile* __restrict__ tiles,
                                                 const GemmGroup* __restrict__ groups,
                                                 const GemmCol* __restrict__ cols, int accumulate) {
    const GemmTile t = tiles[blockIdx.x];
    const GemmGroup G = groups[t.group];
    __shared__ __align__(16) unsigned short Ah[64][40], Al[64][40];   // [m][k]
    __shared__ __align__(16) unsigned short Bh[64][40], Bl[64][40];   // [rhs][k]
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w >> 1, wn = w & 1;
    const int lr = tid >> 2, kc = (tid & 3) * 8;
    const TileCols bc = load_col(G, cols, t.col0 + lr);
    if (!__syncthreads_or(bc.active)) return;
    const unsigned short* ahi = (const unsigned short*)G.Ahi + (size_t)(t.m0 + lr) * G.ldk + kc;
    const unsigned short* alo = (const unsigned short*)G.Alo + (size_t)(t.m0 + lr) * G.ldk + kc;
    floatx4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

    for (int k0 = 0; k0 < G.ldk; k0 += 32) {
        const ushortx8 vh = *(const ushortx8*)(ahi + k0);
        const ushortx8 vl = *(const ushortx8*)(alo + k0);
        double bv[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) bv[e] = bc.active ? bc.bptr[k0 + kc + e] : 0.0;
        *(ushortx8*)&Ah[lr][kc] = vh;
        *(ushortx8*)&Al[lr][kc] = vl;
        ushortx8 bh, bl;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const float x = (float)bv[e];
            const unsigned short h = f2bf_rne(x);
            bh[e] = h;
            bl[e] = f2bf_rne(x - bf2f(h));
        }
        *(ushortx8*)&Bh[lr][kc] = bh;
        *(ushortx8*)&Bl[lr][kc] = bl;
        __syncthreads();
        const int kq = 8 * (lane >> 4);
        bf16x8 a_h[2], a_l[2], b_h[2], b_l[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int m = wm * 32 + i * 16 + (lane & 15);
            a_h[i] = __builtin_bit_cast(bf16x8, *(const ushortx8*)&Ah[m][kq]);
            a_l[i] = __builtin_bit_cast(bf16x8, *(const ushortx8*)&Al[m][kq]);
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int c = wn * 32 + j * 16 + (lane & 15);
            b_h[j] = __builtin_bit_cast(bf16x8, *(const ushortx8*)&Bh[c][kq]);
            b_l[j] = __builtin_bit_cast(bf16x8, *(const ushortx8*)&Bl[c][kq]);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_h[i], b_h[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_h[i], b_l[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_l[i], b_h[j], acc[i][j], 0, 0, 0);
            }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = t.m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + r;
                const int col = t.col0 + wn * 32 + j * 16 + (lane & 15);
                store_out(G, cols, row, col, (double)acc[i][j][r], accumulate);
            }
}

__global__ __launch_bounds__(256) void gemm_f64(const GemmTile* __restrict__ tiles,
                                                const GemmGroup* __restrict__ groups,
                                                const GemmCol* __restrict__ cols, int accumulate) {
    const GemmTile t = tiles[blockIdx.x];
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

hipError_t launch_gemm(int precision, const GemmTile* tiles, int ntiles, const GemmGroup* groups,
                       const GemmCol* cols, int accumulate, hipStream_t st) {
    if (ntiles <= 0) return hipSuccess;
    if (precision == MATO_FP32)
        gemm_f32<<<ntiles, 256, 0, st>>>(tiles, groups, cols, accumulate);
    else if (precision == MATO_BF16_REFINED)
        gemm_bf16<<<ntiles, 256, 0, st>>>(tiles, groups, cols, accumulate);
    else
        gemm_f64<<<ntiles, 256, 0, st>>>(tiles, groups, cols, accumulate);
    return hipGetLastError();
}

}  // namespace mato
