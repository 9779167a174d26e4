// Measurement utilities of libmato: a streaming copy, a streaming in-place update
// (equal HBM reads and writes) and a streaming read (16-byte nontemporal accesses,
// grid-stride), the practical ceilings against which the pairwise stage's multiplier
// stream (12 bytes read per pair-instant; written back only where a multiplier changes)
// is compared.  Not part of the method.
#include "common.h"

#include <algorithm>

namespace mato {

typedef float v4f __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void stream_copy_kernel(const v4f* __restrict__ src, v4f* __restrict__ dst,
                                                          size_t n4) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n4; i += (size_t)gridDim.x * blockDim.x)
        __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

// x <- x / 2 + 1 in place (x / 2 is exact, so the value after k launches is the same
// on the host in FP32)
__global__ __launch_bounds__(256) void stream_update_kernel(v4f* __restrict__ x, size_t n4) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n4; i += (size_t)gridDim.x * blockDim.x)
        __builtin_nontemporal_store(__builtin_nontemporal_load(x + i) * 0.5f + 1.0f, x + i);
}

// Sum of the floats each workgroup reads (one partial per workgroup, so that the loads
// stay); with every float 1.0 and at most 2^24 per workgroup the sums are exact.
__global__ __launch_bounds__(256) void stream_read_kernel(const v4f* __restrict__ src, size_t n4,
                                                          float* __restrict__ part) {
    __shared__ float red[256];
    float acc = 0.0f;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n4; i += (size_t)gridDim.x * blockDim.x) {
        const v4f v = __builtin_nontemporal_load(src + i);
        acc += (v.x + v.y) + (v.z + v.w);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

}  // namespace mato

using namespace mato;

extern "C" mato_status mato_stream_copy(int64_t bytes, int32_t grid, int32_t iters, void* hip_stream,
                                        double* ms_per_copy) {
    if (!ms_per_copy || bytes < 16 || bytes % 16 != 0 || grid < 1 || iters < 1) {
        set_error("stream copy: bytes a positive multiple of 16, grid and iters >= 1");
        return MATO_ERR_INVALID_ARG;
    }
    hipStream_t st = (hipStream_t)hip_stream;
    const size_t n4 = (size_t)bytes / 16;
    void *src = nullptr, *dst = nullptr;
    if (hipMalloc(&src, (size_t)bytes) != hipSuccess || hipMalloc(&dst, (size_t)bytes) != hipSuccess) {
        (void)hipGetLastError();
        dfree(src);
        set_error("device allocation of 2 x %lld bytes failed", (long long)bytes);
        return MATO_ERR_OUT_OF_MEMORY;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    mato_status status = MATO_OK;
    float ms = 0.0f;
    std::vector<unsigned char> head(std::min<size_t>((size_t)bytes, 65536)), tail(head.size());
    auto run = [&]() -> mato_status {
        MATO_HIP(hipMemsetAsync(src, 0x5a, (size_t)bytes, st));
        MATO_HIP(hipMemsetAsync(dst, 0, (size_t)bytes, st));
        MATO_HIP(hipEventCreate(&e0));
        MATO_HIP(hipEventCreate(&e1));
        stream_copy_kernel<<<grid, 256, 0, st>>>((const v4f*)src, (v4f*)dst, n4);   // warm-up
        MATO_HIP(hipEventRecord(e0, st));
        for (int r = 0; r < iters; ++r) stream_copy_kernel<<<grid, 256, 0, st>>>((const v4f*)src, (v4f*)dst, n4);
        MATO_HIP(hipEventRecord(e1, st));
        MATO_HIP(hipEventSynchronize(e1));
        MATO_HIP(hipEventElapsedTime(&ms, e0, e1));
        MATO_HIP(hipMemcpy(head.data(), dst, head.size(), hipMemcpyDeviceToHost));
        MATO_HIP(hipMemcpy(tail.data(), (char*)dst + (bytes - (int64_t)tail.size()), tail.size(), hipMemcpyDeviceToHost));
        for (size_t k = 0; k < head.size(); ++k)
            if (head[k] != 0x5a || tail[k] != 0x5a) {
                set_error("stream copy: destination differs from the source");
                return MATO_ERR_HIP;
            }
        return MATO_OK;
    };
    status = run();
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    dfree(src);
    dfree(dst);
    if (status == MATO_OK) *ms_per_copy = (double)ms / iters;
    return status;
}

extern "C" mato_status mato_stream_update(int64_t bytes, int32_t grid, int32_t iters, void* hip_stream,
                                          double* ms_per_update) {
    if (!ms_per_update || bytes < 16 || bytes % 16 != 0 || grid < 1 || iters < 1) {
        set_error("stream update: bytes a positive multiple of 16, grid and iters >= 1");
        return MATO_ERR_INVALID_ARG;
    }
    hipStream_t st = (hipStream_t)hip_stream;
    const size_t n4 = (size_t)bytes / 16;
    void* x = nullptr;
    if (hipMalloc(&x, (size_t)bytes) != hipSuccess) {
        (void)hipGetLastError();
        set_error("device allocation of %lld bytes failed", (long long)bytes);
        return MATO_ERR_OUT_OF_MEMORY;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float ms = 0.0f;
    std::vector<float> head(std::min<size_t>((size_t)bytes, 65536) / 4), tail(head.size());
    auto run = [&]() -> mato_status {
        MATO_HIP(hipMemsetAsync(x, 0, (size_t)bytes, st));
        MATO_HIP(hipEventCreate(&e0));
        MATO_HIP(hipEventCreate(&e1));
        stream_update_kernel<<<grid, 256, 0, st>>>((v4f*)x, n4);                      // warm-up
        MATO_HIP(hipEventRecord(e0, st));
        for (int r = 0; r < iters; ++r) stream_update_kernel<<<grid, 256, 0, st>>>((v4f*)x, n4);
        MATO_HIP(hipEventRecord(e1, st));
        MATO_HIP(hipEventSynchronize(e1));
        MATO_HIP(hipEventElapsedTime(&ms, e0, e1));
        MATO_HIP(hipMemcpy(head.data(), x, head.size() * 4, hipMemcpyDeviceToHost));
        MATO_HIP(hipMemcpy(tail.data(), (char*)x + (bytes - (int64_t)tail.size() * 4), tail.size() * 4,
                           hipMemcpyDeviceToHost));
        float want = 0.0f;
        for (int r = 0; r <= iters; ++r) want = want * 0.5f + 1.0f;
        for (size_t k = 0; k < head.size(); ++k)
            if (head[k] != want || tail[k] != want) {
                set_error("stream update: unexpected value after %d launches", iters + 1);
                return MATO_ERR_HIP;
            }
        return MATO_OK;
    };
    const mato_status status = run();
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    dfree(x);
    if (status == MATO_OK) *ms_per_update = (double)ms / iters;
    return status;
}

extern "C" mato_status mato_stream_read(int64_t bytes, int32_t grid, int32_t iters, void* hip_stream,
                                        double* ms_per_read) {
    if (!ms_per_read || bytes < 16 || bytes % 16 != 0 || grid < 1 || iters < 1) {
        set_error("stream read: bytes a positive multiple of 16, grid and iters >= 1");
        return MATO_ERR_INVALID_ARG;
    }
    const size_t n4 = (size_t)bytes / 16;
    if (n4 > ((size_t)grid << 22)) {                // at most 2^24 floats per workgroup: exact sums
        set_error("stream read: more than 2^24 floats per workgroup; use a larger grid");
        return MATO_ERR_INVALID_ARG;
    }
    hipStream_t st = (hipStream_t)hip_stream;
    void* src = nullptr;
    float* part = nullptr;
    if (hipMalloc(&src, (size_t)bytes) != hipSuccess || hipMalloc(&part, sizeof(float) * grid) != hipSuccess) {
        (void)hipGetLastError();
        dfree(src);
        set_error("device allocation of %lld bytes failed", (long long)bytes);
        return MATO_ERR_OUT_OF_MEMORY;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float ms = 0.0f;
    std::vector<float> hp(grid);
    auto run = [&]() -> mato_status {
        MATO_HIP(hipMemsetD32Async((hipDeviceptr_t)src, 0x3f800000, n4 * 4, st));   // every float 1.0
        MATO_HIP(hipEventCreate(&e0));
        MATO_HIP(hipEventCreate(&e1));
        stream_read_kernel<<<grid, 256, 0, st>>>((const v4f*)src, n4, part);   // warm-up
        MATO_HIP(hipEventRecord(e0, st));
        for (int r = 0; r < iters; ++r) stream_read_kernel<<<grid, 256, 0, st>>>((const v4f*)src, n4, part);
        MATO_HIP(hipEventRecord(e1, st));
        MATO_HIP(hipEventSynchronize(e1));
        MATO_HIP(hipEventElapsedTime(&ms, e0, e1));
        MATO_HIP(hipMemcpy(hp.data(), part, sizeof(float) * grid, hipMemcpyDeviceToHost));
        double total = 0.0;
        for (float v : hp) total += v;
        if (total != (double)n4 * 4) {
            set_error("stream read: read %.0f floats of 1.0, expected %zu", total, n4 * 4);
            return MATO_ERR_HIP;
        }
        return MATO_OK;
    };
    const mato_status status = run();
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    dfree(src);
    dfree(part);
    if (status == MATO_OK) *ms_per_read = (double)ms / iters;
    return status;
}
