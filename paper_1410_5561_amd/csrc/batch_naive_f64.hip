// Batched naive sweep kernel, f64 grids.
#include "batch_naive.hpp"

namespace mwd {

__global__ void __launch_bounds__(kNaiveBX * kNaiveBY)
batch_naive_kernel_f64(NaiveLaunch<double> L)
{
    __shared__ __attribute__((aligned(16))) char lds[naive_lds_bytes<double>()];
    batch_naive_tile<double>(L, lds);
}

hipError_t batch_naive_launch_f64(const NaiveLaunch<double>& L, int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL(batch_naive_kernel_f64, dim3(nblocks), dim3(kNaiveBX * kNaiveBY), 0, s, L);
    return hipGetLastError();
}

}  // namespace mwd
