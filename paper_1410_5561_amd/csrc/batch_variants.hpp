// The tile shapes compiled into the batched kernel (all fit 1024 threads).
// Variant index = position in this list; the host table in batch.hip mirrors it.
#pragma once

#include "batch_kernel.hpp"

namespace mwd {

// f64: 7-point constant (Dw 8 and 4) and 25-point constant at Dw 8, which holds
// one time level per row (a plain sweep through the same tiles); larger f64
// tiles of the 25-point stencil do not fit the registers of a 1024-thread
// workgroup.
#define MWD_BATCH_VARIANTS_F64                                                      \
    BatchVariant<K7C, 8, 2>, BatchVariant<K7C, 4, 4>, BatchVariant<K25C, 8, 2>
// f32: the same, plus the 25-point constant stencil at Dw 16 and the 7-point
// variable stencil at Dw 4.
#define MWD_BATCH_VARIANTS_F32 MWD_BATCH_VARIANTS_F64, BatchVariant<K25C, 16, 1>, BatchVariant<K7V, 4, 4>

struct BatchVariantInfo {
    int kind, dw, wpr;
};

static const BatchVariantInfo kBatchVariantInfo[] = {
    {K7C, 8, 2}, {K7C, 4, 4}, {K25C, 8, 2}, {K25C, 16, 1}, {K7V, 4, 4},
};
constexpr int kNumBatchVariants = sizeof(kBatchVariantInfo) / sizeof(kBatchVariantInfo[0]);
constexpr int kNumBatchVariantsF64 = 3;

template <typename T>
struct BatchLaunch {
    const BatchTile* tiles;
    int first;            // first table entry of this group
    const MwdArgs<T>* gargs;
    const int* gvariant;
};

hipError_t batch_launch_f64(const BatchLaunch<double>& L, int nblocks, hipStream_t s);
hipError_t batch_launch_f32(const BatchLaunch<float>& L, int nblocks, hipStream_t s);
// Boundary band of every grid into its scratch pairs: table entry z for grid z.
hipError_t batch_halo_launch_f64(const HaloFill<double>* table, dim3 grid, hipStream_t s);
hipError_t batch_halo_launch_f32(const HaloFill<float>* table, dim3 grid, hipStream_t s);

}  // namespace mwd
