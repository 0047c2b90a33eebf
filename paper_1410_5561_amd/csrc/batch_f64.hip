// Batched persistent kernel, f64 grids.
#include "batch_variants.hpp"

namespace mwd {

using BShapes_f64 = BatchKernelShapes<double, MWD_BATCH_VARIANTS_F64>;

__global__ void __launch_bounds__(kBatchThreads)
batch_kernel_f64(BatchLaunch<double> L)
{
    __shared__ __attribute__((aligned(16))) char lds[BShapes_f64::lds_bytes()];
    batch_loop<double, MWD_BATCH_VARIANTS_F64>(L.tiles, L.ntiles, L.gargs, L.gvariant, L.done, L.counter,
                                        L.err, L.spin_limit, lds);
}

hipError_t batch_launch_f64(const BatchLaunch<double>& L, int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL(batch_kernel_f64, dim3(nblocks), dim3(kBatchThreads), 0, s, L);
    return hipGetLastError();
}

int batch_blocks_per_cu_f64()
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_kernel_f64, kBatchThreads, 0) != hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

}  // namespace mwd
