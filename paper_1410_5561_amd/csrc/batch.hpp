// Batched form: many grids advanced together by one captured hipGraph.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/mwd_stencil.h"

namespace mwd {

struct BatchState;

int batch_run(int plan_kind, int plan_dtype, BatchState** state, stencil_grid* grids,
              const stencil_coeffs* coeffs, int n, int T, hipStream_t stream);
void batch_free(BatchState* s);

}  // namespace mwd
