// Streaming copy used as the practical HBM bandwidth reference and as the
// known-traffic kernel for calibrating byte counters: 16-byte vectors,
// grid-stride, every byte read once and written once.
#include "common.hpp"
#include "internal.hpp"

namespace mwd {

__global__ void __launch_bounds__(256)
stream_copy_kernel(uint4* __restrict__ dst, const uint4* __restrict__ src, long long n)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        dst[i] = src[i];
}

hipError_t stream_copy(void* dst, const void* src, long long bytes, hipStream_t stream)
{
    const long long n = bytes / 16;
    if (n == 0) return hipSuccess;
    long long blocks = (n + 255) / 256;
    if (blocks > 256 * 64) blocks = 256 * 64;  // 64 workgroups per CU, then grid-stride
    hipLaunchKernelGGL(stream_copy_kernel, dim3((unsigned)blocks), dim3(256), 0, stream,
                       static_cast<uint4*>(dst), static_cast<const uint4*>(src), n);
    return hipGetLastError();
}

}  // namespace mwd
