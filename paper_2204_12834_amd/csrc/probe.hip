// Stream probes: the achievable HBM bandwidth of plain streaming kernels on
// the device (the reference the series kernels are compared with) and a copy
// of known size for calibrating hardware byte counters.
#include "common.hpp"

namespace poba {

__global__ __launch_bounds__(kBlock) void k_probe_read(const f4v* __restrict__ src, int64_t n4, float* sink) {
    f4v acc = {0.f, 0.f, 0.f, 0.f};
    const int64_t stride = int64_t(gridDim.x) * kBlock;
    int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    for (; i + 3 * stride < n4; i += 4 * stride) {
        const f4v a = __builtin_nontemporal_load(src + i);
        const f4v b = __builtin_nontemporal_load(src + i + stride);
        const f4v c = __builtin_nontemporal_load(src + i + 2 * stride);
        const f4v d = __builtin_nontemporal_load(src + i + 3 * stride);
        acc += (a + b) + (c + d);
    }
    for (; i < n4; i += stride) acc += __builtin_nontemporal_load(src + i);
    const float t = acc.x + acc.y + acc.z + acc.w;
    if (t == 1234.5f) sink[blockIdx.x] = t;  // keeps the loads alive
}

__global__ __launch_bounds__(kBlock) void k_probe_copy(const f4v* __restrict__ src, f4v* __restrict__ dst, int64_t n4) {
    const int64_t stride = int64_t(gridDim.x) * kBlock;
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n4; i += stride)
        __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

__global__ __launch_bounds__(kBlock) void k_probe_write(f4v* __restrict__ dst, int64_t n4) {
    const int64_t stride = int64_t(gridDim.x) * kBlock;
    const f4v z = {0.f, 0.f, 0.f, 0.f};
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n4; i += stride) __builtin_nontemporal_store(z, dst + i);
}

}  // namespace poba

using namespace poba;

extern "C" poba_status poba_probe(int32_t kind, const void* src, void* dst, size_t bytes, int32_t blocks,
                                  poba_stream stream) {
    (void)hipGetLastError();  // report only this call's launch errors
    if (!src || (bytes & 15) || (reinterpret_cast<uintptr_t>(src) & 15)) return POBA_ERR_INVALID_ARG;
    if ((kind == 1 || kind == 2) && (!dst || (reinterpret_cast<uintptr_t>(dst) & 15))) return POBA_ERR_INVALID_ARG;
    if (kind < 0 || kind > 2) return POBA_ERR_INVALID_ARG;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int64_t n4 = int64_t(bytes / 16);
    const unsigned g = unsigned(blocks > 0 ? blocks : 256 * 16);
    if (kind == 0)
        hipLaunchKernelGGL(k_probe_read, dim3(g), dim3(kBlock), 0, s, reinterpret_cast<const f4v*>(src), n4,
                           reinterpret_cast<float*>(dst));
    else if (kind == 1)
        hipLaunchKernelGGL(k_probe_copy, dim3(g), dim3(kBlock), 0, s, reinterpret_cast<const f4v*>(src),
                           reinterpret_cast<f4v*>(dst), n4);
    else
        hipLaunchKernelGGL(k_probe_write, dim3(g), dim3(kBlock), 0, s, reinterpret_cast<f4v*>(dst), n4);
    return hipGetLastError() == hipSuccess ? POBA_OK : POBA_ERR_HIP;
}
