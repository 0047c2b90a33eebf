// Batched row-group kernel, f64 grids.
#include "batch_variants.hpp"

namespace mwd {

using BShapes_f64 = BatchKernelShapes<double, MWD_BATCH_VARIANTS_F64>;

__global__ void __launch_bounds__(kBatchThreads)
batch_kernel_f64(BatchLaunch<double> L)
{
    __shared__ __attribute__((aligned(16))) char lds[BShapes_f64::lds_bytes()];
    batch_group<double, MWD_BATCH_VARIANTS_F64>(L.tiles, L.first, L.gargs, L.gvariant, lds);
}

hipError_t batch_launch_f64(const BatchLaunch<double>& L, int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL(batch_kernel_f64, dim3(nblocks), dim3(kBatchThreads), 0, s, L);
    return hipGetLastError();
}

hipError_t batch_halo_launch_f64(const HaloFill<double>* table, dim3 grid, hipStream_t s)
{
    hipLaunchKernelGGL((mwd_halo_fill_table_kernel<double>), grid, dim3(256), 0, s, table);
    return hipGetLastError();
}

}  // namespace mwd
