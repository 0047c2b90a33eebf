// Schedule choice: default MWD shapes and the autotuner (tune.cpp).
#pragma once

#include "internal.hpp"

namespace mwd {

struct TuneChoice {
    int mode;        // STENCIL_MODE_NAIVE or STENCIL_MODE_MWD
    MwdShape shape;  // valid for MWD
};

// A shape that fits every supported size of this (kind, dtype).
MwdShape default_shape(int kind, int dtype);

// Choose naive or MWD and the MWD shape for grids of this kind, dtype and size.
// Returns a STENCIL_* code.
int tune_choose(int kind, int dtype, int nx, int ny, int nz, int T, TuneChoice* out);

// Tile shape of one grid inside the batched kernel (one of the shapes compiled
// into it, all sized for 1024-thread workgroups).
MwdShape tune_batch_shape(int kind, int dtype, int nx, int ny, int nz, int T);

}  // namespace mwd
