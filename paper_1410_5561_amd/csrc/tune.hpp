// Schedule choice: default MWD shapes and the autotuner (tune.cpp).
#pragma once

#include "internal.hpp"

namespace mwd {

struct TuneChoice {
    int mode;        // STENCIL_MODE_NAIVE or STENCIL_MODE_MWD
    MwdShape shape;  // valid for MWD
};

// Eq. (3) of Sec. III-B: the wavefront cache block in bytes for diamond
// width dw, nf frontlines and an x extent of `lanes` elements,
// N_xb [N_D Dw (Dw/2 - R + N_F) + 2R (Dw + W_w)], W_w = Dw - 2R + N_F.
double cache_block_model(int kind, int dtype, int dw, int lanes, int nf);

// A shape that fits every supported size of this (kind, dtype).
MwdShape default_shape(int kind, int dtype);

// Choose naive or MWD and the MWD shape for grids of this kind, dtype and size.
// Returns a STENCIL_* code.
int tune_choose(int kind, int dtype, int nx, int ny, int nz, int T, TuneChoice* out);

// Schedule of one grid inside a batch: the batched naive sweep, or one of the
// MWD tile shapes compiled into the batched kernel (all sized for 1024-thread
// workgroups).  MWD_TUNE=naive forces the naive sweep, MWD_TUNE=mwd (or
// mwd:<dw>:<lanes>) the best batched MWD shape.
TuneChoice tune_batch_choose(int kind, int dtype, int nx, int ny, int nz, int T);

}  // namespace mwd
