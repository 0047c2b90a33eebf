// Streaming copy used as the practical HBM bandwidth reference and as the
// known-traffic kernel for calibrating byte counters: every byte read once
// and written once.
#include "common.hpp"
#include "internal.hpp"

namespace mwd {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Each workgroup copies runs of 4 x 256 16-byte vectors: four loads in flight
// per lane, then four stores, all non-temporal (the data are not reused).
__global__ void __launch_bounds__(256)
stream_copy_kernel(u32x4* __restrict__ dst, const u32x4* __restrict__ src, long long n)
{
    constexpr int UN = 4;
    const long long step = (long long)gridDim.x * UN * 256;
    for (long long base = (long long)blockIdx.x * UN * 256 + threadIdx.x; base < n; base += step) {
        u32x4 v[UN];
#pragma unroll
        for (int k = 0; k < UN; ++k) {
            const long long i = base + k * 256;
            if (i < n) v[k] = __builtin_nontemporal_load(&src[i]);
        }
#pragma unroll
        for (int k = 0; k < UN; ++k) {
            const long long i = base + k * 256;
            if (i < n) __builtin_nontemporal_store(v[k], &dst[i]);
        }
    }
}

hipError_t stream_copy(void* dst, const void* src, long long bytes, hipStream_t stream)
{
    const long long n = bytes / 16;
    if (n == 0) return hipSuccess;
    long long blocks = (n + 4 * 256 - 1) / (4 * 256);
    if (blocks > 256 * 64) blocks = 256 * 64;  // 64 workgroups per CU, then grid-stride
    hipLaunchKernelGGL(stream_copy_kernel, dim3((unsigned)blocks), dim3(256), 0, stream,
                       static_cast<u32x4*>(dst), static_cast<const u32x4*>(src), n);
    return hipGetLastError();
}

}  // namespace mwd
