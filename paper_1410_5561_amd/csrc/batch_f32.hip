// Batched persistent kernel, f32 grids.
#include "batch_variants.hpp"

namespace mwd {

using BShapes_f32 = BatchKernelShapes<float, MWD_BATCH_VARIANTS_F32>;

__global__ void __launch_bounds__(kBatchThreads)
batch_kernel_f32(BatchLaunch<float> L)
{
    __shared__ __attribute__((aligned(16))) char lds[BShapes_f32::lds_bytes()];
    batch_loop<float, MWD_BATCH_VARIANTS_F32>(L.tiles, L.ntiles, L.gargs, L.gvariant, L.done, L.counter,
                                        L.err, L.spin_limit, lds);
}

hipError_t batch_launch_f32(const BatchLaunch<float>& L, int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL(batch_kernel_f32, dim3(nblocks), dim3(kBatchThreads), 0, s, L);
    return hipGetLastError();
}

int batch_blocks_per_cu_f32()
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_kernel_f32, kBatchThreads, 0) != hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

}  // namespace mwd
