// Yardsticks the render's measurements are compared with: a plain
// device-to-device streaming copy (the achievable HBM bandwidth; 16-byte
// loads and stores, one read and one write of every byte) and a stream of
// independent FP32 FMAs (the achievable vector FMA rate, with all or only
// some lanes of each wavefront live).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "../../include/lf.h"
#include "lf_internal.h"

namespace lf {

__global__ __launch_bounds__(256) void k_stream_copy(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                     int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

// Eight independent FMA chains per lane, `iters` steps each, on the first
// `active` lanes of every wavefront; every thread writes the sum of its
// chains (the other lanes leave their start values untouched).
__global__ __launch_bounds__(256) void k_fma_rate(float *__restrict__ out, int32_t iters, int32_t active, float a,
                                                  float b) {
    const int lane = threadIdx.x & 63;
    float x0 = lane, x1 = lane + 1, x2 = lane + 2, x3 = lane + 3;
    float x4 = lane + 4, x5 = lane + 5, x6 = lane + 6, x7 = lane + 7;
    if (lane < active) {
#pragma unroll 8
        for (int i = 0; i < iters; ++i) {
            x0 = fmaf(x0, a, b);
            x1 = fmaf(x1, a, b);
            x2 = fmaf(x2, a, b);
            x3 = fmaf(x3, a, b);
            x4 = fmaf(x4, a, b);
            x5 = fmaf(x5, a, b);
            x6 = fmaf(x6, a, b);
            x7 = fmaf(x7, a, b);
        }
    }
    out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = ((x0 + x1) + (x2 + x3)) + ((x4 + x5) + (x6 + x7));
}

}  // namespace lf

extern "C" int lf_fma_rate(float *out, int32_t blocks, int32_t iters, int32_t active, void *hip_stream) {
    if (!out) return lf::fail_msg(LF_EINVAL, "out must not be NULL");
    if (blocks < 1 || iters < 1 || active < 1 || active > 64)
        return lf::fail_msg(LF_EINVAL, "need blocks >= 1, iters >= 1 and active in [1, 64]");
    hipLaunchKernelGGL(lf::k_fma_rate, dim3(blocks), dim3(256), 0, (hipStream_t)hip_stream, out, iters, active,
                       0.999f, 0.001f);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return lf::fail_msg(LF_EHIP, hipGetErrorString(e));
    return LF_OK;
}

extern "C" int lf_stream_copy(const void *src, void *dst, int64_t bytes, void *hip_stream) {
    if (!src || !dst) return lf::fail_msg(LF_EINVAL, "src and dst must not be NULL");
    if (bytes <= 0 || bytes % 16 || ((uintptr_t)src & 15) || ((uintptr_t)dst & 15))
        return lf::fail_msg(LF_EINVAL, "bytes must be a positive multiple of 16 and both buffers 16-byte aligned");
    const int64_t n = bytes / 16;
    // one 16-byte element per thread over the whole buffer (grid-stride only
    // past 2^30 workgroups): on MI355X a 2 GiB copy runs at 6.1 TB/s this way
    // against 4.5-4.7 TB/s with a persistent grid of 8-64 workgroups per CU
    const int grid = (int)std::min<int64_t>((n + 255) / 256, (int64_t)1 << 30);
    hipLaunchKernelGGL(lf::k_stream_copy, dim3(grid), dim3(256), 0, (hipStream_t)hip_stream, (const uint4 *)src,
                       (uint4 *)dst, n);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return lf::fail_msg(LF_EHIP, hipGetErrorString(e));
    return LF_OK;
}
