// The FP64 reductions' allocation-free form (its kernels are those of
// norms_fp64, declared with the other internal interfaces).
#pragma once

#include "internal.hpp"

namespace mwd {

// The norms of norms_fp64 with the per-block partials in the library's
// static device array: allocates nothing; the two results go to out_dev
// (device memory), asynchronously on `stream`.
hipError_t norms_fp64_static(const DevGrid& ga, const void* a, const DevGrid& gb, const void* b,
                             int which, double* out_dev, hipStream_t stream);

}  // namespace mwd
