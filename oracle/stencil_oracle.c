/*
 * Plain, slow, obviously correct CPU oracle for the repeated Jacobi-like
 * stencil sweeps of Sec. I (Listings 1-3).
 *
 * TEST INFRASTRUCTURE ONLY: only tests, the package smoke check and the
 * benchmark's CPU baseline may load this library.  It shares no code, header,
 * table or helper with the GPU library, and it includes nothing from it.
 *
 * Build (done by __graft_entry__.build()):
 *   gcc -O2 -fopenmp -ffp-contract=off -fno-fast-math -fPIC -shared \
 *       oracle/stencil_oracle.c -o oracle/liboracle.so
 *
 * Multi-step temporal blocking (diamonds, wavefronts) is a reordering of the
 * very same lattice-site updates (Sec. II-A), so its result is, by
 * definition, the result of this plain sweep.
 */
#include <stddef.h>

#define ORACLE_7C 0
#define ORACLE_7V 1
#define ORACLE_25C 2
#define ORACLE_25V 3

#define REAL double
#define SWEEP_NAME oracle_sweep_f64
#define RUN_NAME oracle_run_f64
#include "oracle_body.h"
#undef REAL
#undef SWEEP_NAME
#undef RUN_NAME

#define REAL float
#define SWEEP_NAME oracle_sweep_f32
#define RUN_NAME oracle_run_f32
#include "oracle_body.h"
#undef REAL
#undef SWEEP_NAME
#undef RUN_NAME

int oracle_abi_version(void) { return 1; }
