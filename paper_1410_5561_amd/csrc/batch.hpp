// Batched form: many grids advanced together by one captured hipGraph.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/mwd_stencil.h"

namespace mwd {

struct BatchState;

int batch_run(int plan_kind, int plan_dtype, BatchState** state, stencil_grid* grids,
              const stencil_coeffs* coeffs, int n, int T, hipStream_t stream);
void batch_free(BatchState* s);

// Milliseconds per replay of the batched graph over `count` copies of an
// nx x ny x nz grid of `kind` (zero fields and arrays, constant weights),
// every grid on batched tile variant `var` (an index of the batched kernel's
// variant table) or, for var = -1, on the batched naive sweep; T steps.
// Negative on failure.  Allocates and frees its grids; synchronous.  For the
// autotuner.
double batch_proxy_ms(int kind, int dtype, int nx, int ny, int nz, int T, int count, int var);

}  // namespace mwd
