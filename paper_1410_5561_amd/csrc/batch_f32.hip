// Batched row-group kernel, f32 grids.
#include "batch_variants.hpp"

namespace mwd {

using BShapes_f32 = BatchKernelShapes<float, MWD_BATCH_VARIANTS_F32>;

__global__ void __launch_bounds__(kBatchThreads)
batch_kernel_f32(BatchLaunch<float> L)
{
    __shared__ __attribute__((aligned(16))) char lds[BShapes_f32::lds_bytes()];
    batch_group<float, MWD_BATCH_VARIANTS_F32>(L.tiles, L.first, L.gargs, L.gvariant, lds);
}

hipError_t batch_launch_f32(const BatchLaunch<float>& L, int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL(batch_kernel_f32, dim3(nblocks), dim3(kBatchThreads), 0, s, L);
    return hipGetLastError();
}

hipError_t batch_halo_launch_f32(const HaloFill<float>* table, dim3 grid, hipStream_t s)
{
    hipLaunchKernelGGL((mwd_halo_fill_table_kernel<float>), grid, dim3(256), 0, s, table);
    return hipGetLastError();
}

}  // namespace mwd
