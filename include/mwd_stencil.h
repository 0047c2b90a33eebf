/*
 * mwd_stencil.h - C ABI of the MI355X (gfx950) stencil library.
 *
 * The library applies T time steps of a Jacobi-like stencil sweep to a 3-D
 * grid held in two device arrays (the two-array scheme of Sec. I of Malas,
 * Hager, Ltaief, Keyes, "Towards energy efficiency and maximum computational
 * intensity for stencil algorithms using wavefront diamond temporal
 * blocking"), either as one full sweep per step (the spatial-blocking
 * baseline of Sec. IV) or reordered by multicore wavefront diamond (MWD)
 * temporal blocking (Sec. II-A): diamond tiles in y-t, a wavefront along z,
 * tiles along the leading dimension x (Sec. III-A).  MWD performs the very
 * same lattice-site updates in another order, so both modes return the same
 * bits.
 *
 * Conventions for every call:
 *   - return 0 on success or a negative STENCIL_E* code; nothing throws or
 *     aborts across the ABI; stencil_last_error() gives the detail;
 *   - all argument checks happen before any device work, so a rejected call
 *     leaves every buffer untouched;
 *   - pointers named "device" are HIP device allocations owned by the caller;
 *     "stream" is a hipStream_t passed as void* (NULL = the null stream);
 *   - a plan is not thread-safe; distinct plans may run on distinct streams.
 *
 * Grid layout: padded row-major [z][y][x], x contiguous (x is the leading
 * dimension, Sec. II-A).  Interior extents nx, ny, nz; a halo of `halo` cells
 * on every side holds the fixed boundary values (the listings never write
 * it).  Element (x, y, z), with -halo <= x < nx + halo etc., lives at
 *     buf[(z + halo) * sz + (y + halo) * sy + (x + halo)].
 */
#ifndef MWD_STENCIL_H
#define MWD_STENCIL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define STENCIL_OK            0
#define STENCIL_EINVAL       -1  /* bad pointer, size, stride, halo, T, kind or dtype   */
#define STENCIL_EUNSUPPORTED -2  /* valid request the compiled library cannot run     */
#define STENCIL_ENOMEM       -3  /* a device or host allocation failed                 */
#define STENCIL_EDEVICE      -4  /* a HIP runtime call failed (text in last_error)     */

/* Stencil operators (Sec. I-A).  Radius R = 1 for the 7-point kinds, 4 for the
 * 25-point kinds; N_D (domain-sized streams, Sec. III-B) = 2, 9, 2, 15. */
typedef enum {
    STENCIL_7PT_CONST = 0,  /* Listing 1: c0*V + c1*(x+ + x-) + c1*(y+ + y-) + c1*(z+ + z-)   */
    STENCIL_7PT_VAR = 1,    /* Listing 2: C0..C6 arrays weight centre, +x, -x, +y, -y, +z, -z */
    STENCIL_25PT_CONST = 2, /* Listing 3 with the 13 weights held constant                    */
    STENCIL_25PT_VAR = 3,   /* Listing 3 as printed: 13 coefficient arrays                    */
    STENCIL_KIND_MIXED = 15 /* plan for stencil_run_batched over grids of several kinds       */
} stencil_kind;

typedef enum { STENCIL_F64 = 0, STENCIL_F32 = 1 } stencil_dtype;

typedef enum {
    STENCIL_MODE_AUTO = 0,  /* let the plan choose (autotuned once per size and T)            */
    STENCIL_MODE_NAIVE = 1, /* one full sweep per time step                                   */
    STENCIL_MODE_MWD = 2    /* wavefront diamond temporal blocking                            */
} stencil_mode;

typedef struct stencil_plan stencil_plan; /* opaque, owned by the library */

/* A grid in device memory.  buf[cur] holds the current level u_t on entry.
 * On return from stencil_run, buf[cur] holds u_{t+T} and buf[cur ^ 1] holds
 * u_{t+T-1} (for T > 0), and cur has been updated.  Both buffers must carry
 * the same halo values; the library never writes the halo. */
typedef struct {
    int32_t nx, ny, nz;  /* interior extents, each >= 1                                        */
    int32_t halo;        /* halo width, >= R                                                   */
    int64_t sy, sz;      /* element strides: sy >= nx + 2*halo, sz >= sy * (ny + 2*halo)       */
    int32_t dtype;       /* stencil_dtype                                                      */
    int32_t cur;         /* 0 or 1: which buffer holds the current level                       */
    void *buf[2];        /* device pointers to the padded arrays (element 0 = corner of halo)  */
} stencil_grid;

/* Weights.  Constant kinds read c[]: 7-point c[0] = c0 (centre), c[1] = c1
 * (each neighbour); 25-point c[0] = C00, c[1..12] = C01..C12 in Listing 3's
 * order (radius 1..4 outer, axis x, y, z inner).  Values are converted to the
 * grid dtype.  Variable kinds read arr[]: 7 (7-point) or 13 (25-point) device
 * arrays with the grid's dtype, shape and strides; only interior entries are
 * read. */
typedef struct {
    int32_t kind;        /* stencil_kind of this grid                                          */
    int32_t reserved;
    double c[13];
    const void *arr[13];
} stencil_coeffs;

/* Schedule parameters; results never depend on them.  Pass NULL to
 * stencil_create for the autotuned choice. */
typedef struct {
    int32_t mode;        /* stencil_mode                                                       */
    int32_t dw;          /* MWD diamond width along y (multiple of 2R; 0 = plan's choice)      */
    int32_t lanes;       /* MWD x lanes per diamond row (64, 128 or 256; 0 = plan's choice)    */
    int32_t reserved;
} stencil_params;

/* What a plan chose, for reporting. */
typedef struct {
    int32_t kind, dtype, mode, dw;
    int32_t lanes;       /* x lanes per diamond row                                            */
    int32_t xtile;       /* x points each tile writes (lanes minus the overlap)                */
    int32_t levels;      /* time levels per diamond (Dw/R - 1)                                 */
    int32_t rows_per_T;  /* unused, 0                                                          */
    double model_bytes_per_lup;  /* Eq. (5) with s = element size (MWD) or s*N_D (naive)       */
} stencil_plan_desc;

/* Create a plan for grids of the given kind, dtype and interior size
 * (STENCIL_KIND_MIXED with nx = ny = nz = 0 for batched plans).  p == NULL
 * asks for the autotuned schedule (Sec. II-A: parameters are auto-tuned);
 * tuning runs at the first stencil_run (synchronously, on a proxy grid of
 * the same x-y extent that it allocates and frees: as many planes as 8 GiB
 * of arrays hold, but at least 64 and at most nz; if the proxy cannot be
 * allocated, the plan runs the naive sweep), predicting the whole run for
 * that call's T; the choice is kept for the plan's later runs.
 * MWD_TUNE=naive or MWD_TUNE=mwd:<dw>:<lanes> (environment) replaces the
 * tuning by that choice (a shape no kernel implements is ignored).
 * Errors: EINVAL (bad kind/dtype/size/params),
 * EUNSUPPORTED (parameters no kernel implements), ENOMEM. */
int stencil_create(stencil_plan **out, int32_t kind, int32_t dtype,
                   int32_t nx, int32_t ny, int32_t nz, const stencil_params *p);

/* Advance `grid` by T time steps (Sec. I, Listings 1-3) on `stream`
 * (asynchronous).  T == 0 is a no-op.  MWD plans allocate device scratch
 * (four more grid-sized arrays: two buffer pairs) on first use and keep it
 * until destroy; the
 * scratch holds intermediate levels so that concurrently running x-tiles
 * never read a value another tile overwrites.  The MWD tile kernel
 * addresses a padded plane with 32-bit byte offsets, so MWD runs grids whose
 * plane (sz elements) is below 4 GiB; for a larger plane an explicit MWD
 * plan fails with EUNSUPPORTED and an autotuned plan runs the naive sweep.
 * Runs of one plan on different streams must be ordered by the caller (they
 * share the plan's scratch).  Errors: EINVAL (null pointers, size or dtype
 * mismatch with the plan, halo < R, T < 0, bad strides, cur not 0/1,
 * coefficient kind mismatch) and EUNSUPPORTED, both before any device
 * work; ENOMEM, EDEVICE. */
int stencil_run(stencil_plan *plan, stencil_grid *grid, const stencil_coeffs *coeffs,
                int32_t T, void *stream);

/* Release a plan: waits for the plan's own last run (an event recorded on
 * that run's stream; work on other streams is not waited for), then frees
 * its scratch and graphs. */
int stencil_destroy(stencil_plan *plan);

/* Advance n independent grids (1 <= n <= 65535; uneven sizes, any kind; one
 * dtype per call) by T steps with ONE hipGraph launch (batched form of the
 * MWD method, Sec. II-A).  Per grid the plan picks, by kind and size bucket
 * (autotuned once per bucket: the batched graph itself is timed on a proxy
 * batch of copies of the bucket's grid, once per candidate schedule), either:
 *  - MWD tiles: the tiles of all such grids are grouped by diamond row, one
 *    kernel launch per group (a workgroup per tile, any grid), then a gather;
 *    kernel boundaries are the row-to-row dependencies.  Shapes: 7c and 25c
 *    in both dtypes, 7v in FP32 (those compiled into the batched kernel);
 *  - the naive sweep: grids grouped so that a group's arrays fit the GPU's
 *    last-level cache, each group taking its T one-step launches before the
 *    next group starts; groups alternate between two concurrent branches;
 *    within a group, runs of neighbouring blocks go to one XCD.
 * No workgroup waits on another.  The first call for a given set of grids
 * builds the tables, allocates scratch (two extra buffer pairs per MWD grid)
 * and captures the graph; later calls with the same grids (same pointers,
 * sizes, weights and cur) replay it; two such sets are cached.  Asynchronous
 * on `stream`; on return every grids[i].cur is updated as by stencil_run.
 * The plan must have been created with STENCIL_KIND_MIXED or the grids'
 * common kind.  MWD_TUNE=naive or MWD_TUNE=mwd (environment) forces every
 * grid onto one of the two schedules, MWD_TUNE=mwd:<dw>:<lanes> onto that
 * batched tile shape (a kind without a batched tile shape, or without that
 * one, or a grid whose plane is 4 GiB or more, stays naive);
 * MWD_BATCH_GROUP_BYTES (environment, bytes) replaces the 96 MiB budget of
 * one group of naive grids.  Errors: as stencil_run; EINVAL for n outside
 * 1..65535. */
int stencil_run_batched(stencil_plan *plan, stencil_grid *grids, const stencil_coeffs *coeffs,
                        int32_t n, int32_t T, void *stream);

/* FP64 norms over the interior, accumulated in FP64 whatever the grid dtype.
 * which = 0: of u = buf[cur]; which = 1: of the residual buf[cur] - buf[cur^1]
 * (u_T - u_{T-1} after a run).  out[0] = sqrt(sum of squares), out[1] = max
 * |.|, NaN if any interior value is NaN.  Synchronous: returns after the
 * result is on the host.  Calls from several threads are serialised inside
 * the library (the per-block partials live in one buffer per device). */
int stencil_norms(const stencil_grid *grid, int32_t which, double out[2], void *stream);

/* FP64 norms of a.buf[a.cur] - b.buf[b.cur] over the interior (same nx, ny,
 * nz; dtypes may differ, e.g. an FP32 run against an FP64 run).
 * Synchronous. */
int stencil_diff_norms(const stencil_grid *a, const stencil_grid *b, double out[2], void *stream);

/* The norms of stencil_norms without any allocation, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  The per-block partials
 * live in a fixed 32 KiB array inside the loaded library (one per device,
 * kept until the process ends; every grid size fits, since the reduction
 * uses at most 2048 blocks); the call allocates nothing and synchronises
 * nothing.  out_dev: caller-owned device memory for two doubles (8-byte
 * aligned), written asynchronously on `stream`: out_dev[0] = L2 norm,
 * out_dev[1] = max norm, of u (which = 0) or of the residual (which = 1),
 * bit-identical to stencil_norms on the same grid.  Calls that overlap on
 * one device share the array and race: order them (one stream, or events).
 * Errors: EINVAL (as stencil_norms, or out_dev NULL or misaligned), EDEVICE. */
int stencil_norms_noalloc(const stencil_grid *grid, int32_t which, double *out_dev, void *stream);

/* On-chip resources of the compiled MWD tile kernel of a shape (Dw, lanes),
 * for comparing its working set with the cache-block model (Eq. 3 of
 * Sec. III-B): out[0] = vector registers per lane, out[1] = LDS bytes per
 * workgroup, out[2] = register-spill (scratch) bytes per lane, out[3] =
 * threads per workgroup, out[4] = workgroups that fit one CU.  Needs a GPU.
 * Errors: EINVAL, EUNSUPPORTED (no kernel for the shape), EDEVICE. */
int stencil_kernel_resources(int32_t kind, int32_t dtype, int32_t dw, int32_t lanes, int32_t out[5]);

/* Describe a plan's chosen schedule (after the first run for autotuned plans). */
int stencil_plan_describe(const stencil_plan *plan, stencil_plan_desc *out);

/* Model code balance in bytes per lattice-site update: Eq. (5) of Sec. III-C,
 * 2 s R (N_D + 2) / Dw, for MWD with diamond width dw; s * N_D for dw == 0
 * (one sweep reading every stream once and writing one).  Negative on bad
 * arguments. */
double stencil_model_bytes_per_lup(int32_t kind, int32_t dtype, int32_t dw);

/* Wavefront cache block in bytes: Eq. (3) of Sec. III-B,
 * N_xb [N_D Dw (Dw/2 - R + N_F) + 2R (Dw + W_w)], W_w = Dw - 2R + N_F, for
 * diamond width dw, nf frontlines (N_F) and an x extent of `lanes` elements
 * (N_xb = lanes x element size).  The autotuner tries a tile shape only if
 * its block (nf = 1) fills at most half of a CU's LDS and registers.
 * Negative on bad arguments. */
double stencil_model_cache_block(int32_t kind, int32_t dtype, int32_t dw, int32_t lanes, int32_t nf);

/* Kernel timing for measurement tools.  While enabled, the plan records a HIP
 * event pair on the run's stream around every kernel it launches.
 * stencil_profile_read waits for those events and returns
 *   out[0] = summed milliseconds of the sweep / MWD tile kernels,
 *   out[1] = their launch count,
 *   out[2] = summed milliseconds of the plan's other kernels (the final
 *            gather of the MWD scratch pairs), out[3] = their count,
 * accumulated since the previous read, then forgets them. */
int stencil_profile_enable(stencil_plan *plan, int32_t enable);
int stencil_profile_read(stencil_plan *plan, double out[4]);

/* Streaming device-to-device copy of `bytes` bytes (a multiple of 16; both
 * pointers 16-byte aligned device memory, not overlapping), asynchronous on
 * `stream`.  It is the practical-bandwidth reference, the analogue of the
 * STREAM COPY figure the paper measures its memory bound with (Sec. IV-A),
 * and the kernel of known traffic used to calibrate HBM byte counters.
 * Errors: EINVAL (NULL, misaligned, size not a multiple of 16), EDEVICE. */
int stencil_stream_copy(void *dst, const void *src, int64_t bytes, void *stream);

const char *stencil_strerror(int code);
const char *stencil_last_error(void);  /* thread-local detail of the last failure */
int stencil_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MWD_STENCIL_H */
