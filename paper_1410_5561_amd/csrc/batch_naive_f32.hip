// Batched naive sweep kernel, f32 grids.
#include "batch_naive.hpp"

namespace mwd {

// Two 1024-thread workgroups per CU (8 waves per SIMD: at most 64 registers),
// so that one workgroup's barriers overlap the other's work.
__global__ void __launch_bounds__(kNaiveBX * kNaiveBY, 8)
batch_naive_kernel_f32(NaiveLaunch<float> L)
{
    __shared__ __attribute__((aligned(16))) char lds[naive_lds_bytes<float>()];
    batch_naive_tile<float>(L, lds);
}

hipError_t batch_naive_launch_f32(const NaiveLaunch<float>& L, int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL(batch_naive_kernel_f32, dim3(nblocks), dim3(kNaiveBX * kNaiveBY), 0, s, L);
    return hipGetLastError();
}

}  // namespace mwd
