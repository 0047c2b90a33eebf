// C ABI of the library: argument checks, plans, dispatch to the naive and
// MWD kernels, error reporting.  Declarations and semantics: mwd_stencil.h.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "../../include/mwd_stencil.h"
#include "batch.hpp"
#include "internal.hpp"
#include "reduce.hpp"
#include "tune.hpp"

namespace mwd {

static thread_local std::string t_last_error;

void set_last_error(const std::string& s) { t_last_error = s; }

static int fail(int code, const std::string& msg)
{
    set_last_error(msg);
    return code;
}

static int hip_fail(hipError_t e, const char* where)
{
    return fail(STENCIL_EDEVICE, std::string(where) + ": " + hipGetErrorName(e) + " (" +
                                     hipGetErrorString(e) + ")");
}

static size_t elem_size(int dtype) { return dtype == STENCIL_F64 ? 8 : 4; }

static bool kind_ok(int k) { return k >= STENCIL_7PT_CONST && k <= STENCIL_25PT_VAR; }

// Checks shared by every entry point that takes a grid.
int check_grid(const stencil_grid* g, const char* name)
{
    if (!g) return fail(STENCIL_EINVAL, std::string(name) + " is NULL");
    if (g->nx < 1 || g->ny < 1 || g->nz < 1)
        return fail(STENCIL_EINVAL, std::string(name) + ": interior extents must be >= 1");
    if (g->halo < 0) return fail(STENCIL_EINVAL, std::string(name) + ": negative halo");
    if (g->dtype != STENCIL_F64 && g->dtype != STENCIL_F32)
        return fail(STENCIL_EINVAL, std::string(name) + ": unknown dtype");
    if (g->cur != 0 && g->cur != 1) return fail(STENCIL_EINVAL, std::string(name) + ": cur must be 0 or 1");
    const int64_t h2 = 2LL * g->halo;
    if (g->sy < g->nx + h2 || g->sz < g->sy * (g->ny + h2))
        return fail(STENCIL_EINVAL, std::string(name) + ": strides too small for extents and halo");
    if (!g->buf[0] || !g->buf[1]) return fail(STENCIL_EINVAL, std::string(name) + ": NULL buffer");
    if (g->buf[0] == g->buf[1]) return fail(STENCIL_EINVAL, std::string(name) + ": buffers alias");
    const size_t es = elem_size(g->dtype);
    if ((reinterpret_cast<uintptr_t>(g->buf[0]) % es) || (reinterpret_cast<uintptr_t>(g->buf[1]) % es))
        return fail(STENCIL_EINVAL, std::string(name) + ": misaligned buffer");
    return STENCIL_OK;
}

DevGrid to_dev(const stencil_grid* g)
{
    DevGrid d;
    d.nx = g->nx;
    d.ny = g->ny;
    d.nz = g->nz;
    d.halo = g->halo;
    d.sy = g->sy;
    d.sz = g->sz;
    d.dtype = g->dtype;
    d.cur = g->cur;
    const size_t es = elem_size(g->dtype);
    const long long off = (long long)g->halo * g->sz + (long long)g->halo * g->sy + g->halo;
    for (int i = 0; i < 2; ++i) d.org[i] = static_cast<char*>(g->buf[i]) + off * es;
    return d;
}

int check_coeffs(const stencil_coeffs* c, int kind, const stencil_grid* g, HostWeights* out)
{
    if (!c) return fail(STENCIL_EINVAL, "coeffs is NULL");
    if (c->kind != kind) return fail(STENCIL_EINVAL, "coeffs.kind does not match the stencil kind");
    out->kind = kind;
    const size_t es = elem_size(g->dtype);
    const long long off = (long long)g->halo * g->sz + (long long)g->halo * g->sy + g->halo;
    for (int m = 0; m < 13; ++m) {
        out->c[m] = c->c[m];
        out->org[m] = nullptr;
    }
    const int na = narr_of(kind);
    for (int m = 0; m < na; ++m) {
        if (!c->arr[m]) return fail(STENCIL_EINVAL, "coefficient array " + std::to_string(m) + " is NULL");
        if (reinterpret_cast<uintptr_t>(c->arr[m]) % es)
            return fail(STENCIL_EINVAL, "misaligned coefficient array");
        out->org[m] = static_cast<const char*>(c->arr[m]) + off * es;
    }
    return STENCIL_OK;
}

}  // namespace mwd

using namespace mwd;

struct stencil_plan {
    int kind, dtype, nx, ny, nz;
    bool autotune;
    int mode;            // resolved mode (naive or mwd) once chosen
    MwdShape shape;
    bool chosen;
    // MWD scratch: two extra buffer pairs laid out like the last grid run
    void* scratch_base[4];
    void* scratch_org[4];
    size_t scratch_bytes;
    long long scratch_sy, scratch_sz;
    int scratch_halo, scratch_dev;
    BatchState* batch;
    Prof* prof;
    // completion of the plan's last run (event on its stream), for destroy
    hipEvent_t done;
    int done_dev;
};

// Record the completion of a run on its stream (not while the stream is
// being captured into a graph: a captured run completes when the graph does).
static void mark_done(stencil_plan* p, hipStream_t s)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
        (void)hipGetLastError();
        return;
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    if (p->done && p->done_dev != dev) {
        // a run on another device: wait for the earlier one before the event is replaced
        (void)hipEventSynchronize(p->done);
        (void)hipEventDestroy(p->done);
        p->done = nullptr;
    }
    if (!p->done) {
        if (hipEventCreateWithFlags(&p->done, hipEventDisableTiming) != hipSuccess) {
            p->done = nullptr;
            (void)hipGetLastError();
            return;
        }
        p->done_dev = dev;
    }
    if (hipEventRecord(p->done, s) != hipSuccess) (void)hipGetLastError();
}

static void free_scratch(stencil_plan* p)
{
    for (int i = 0; i < 4; ++i) {
        if (p->scratch_base[i]) (void)hipFree(p->scratch_base[i]);
        p->scratch_base[i] = p->scratch_org[i] = nullptr;
    }
    p->scratch_bytes = 0;
}

static int ensure_scratch(stencil_plan* p, const stencil_grid* g)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    const size_t es = elem_size(g->dtype);
    const size_t bytes = (size_t)g->sz * (size_t)(g->nz + 2 * g->halo) * es;
    if (p->scratch_base[0] && p->scratch_bytes == bytes && p->scratch_sy == g->sy &&
        p->scratch_sz == g->sz && p->scratch_halo == g->halo && p->scratch_dev == dev)
        return STENCIL_OK;
    free_scratch(p);
    for (int i = 0; i < 4; ++i) {
        e = hipMalloc(&p->scratch_base[i], bytes);
        if (e != hipSuccess) {
            p->scratch_base[i] = nullptr;
            free_scratch(p);
            (void)hipGetLastError();
            return fail(STENCIL_ENOMEM, "MWD scratch allocation of 4 x " + std::to_string(bytes) + " bytes failed");
        }
        const long long off = (long long)g->halo * g->sz + (long long)g->halo * g->sy + g->halo;
        p->scratch_org[i] = static_cast<char*>(p->scratch_base[i]) + off * es;
    }
    p->scratch_bytes = bytes;
    p->scratch_sy = g->sy;
    p->scratch_sz = g->sz;
    p->scratch_halo = g->halo;
    p->scratch_dev = dev;
    return STENCIL_OK;
}

extern "C" {

int stencil_abi_version(void) { return 1; }

const char* stencil_strerror(int code)
{
    switch (code) {
        case STENCIL_OK: return "success";
        case STENCIL_EINVAL: return "invalid argument";
        case STENCIL_EUNSUPPORTED: return "unsupported request";
        case STENCIL_ENOMEM: return "out of memory";
        case STENCIL_EDEVICE: return "HIP device error";
        default: return "unknown error code";
    }
}

const char* stencil_last_error(void) { return t_last_error.c_str(); }

double stencil_model_bytes_per_lup(int32_t kind, int32_t dtype, int32_t dw)
{
    if (!kind_ok(kind) || (dtype != STENCIL_F64 && dtype != STENCIL_F32) || dw < 0) return -1.0;
    const double s = (double)elem_size(dtype);
    const double R = radius_of(kind), ND = ndomain_of(kind);
    if (dw == 0) return s * ND;
    // Eq. (5): (2Dw - 2R) writes and (N_D Dw + 2R) reads per extruded
    // diamond of Dw^2 / (2R) updates, each of s bytes.
    return s * 2.0 * R * ((2.0 * dw - 2.0 * R) + (ND * dw + 2.0 * R)) / ((double)dw * dw);
}

double stencil_model_cache_block(int32_t kind, int32_t dtype, int32_t dw, int32_t lanes, int32_t nf)
{
    if (!kind_ok(kind) || (dtype != STENCIL_F64 && dtype != STENCIL_F32) || dw < 1 || lanes < 1 || nf < 1)
        return -1.0;
    return cache_block_model(kind, dtype, dw, lanes, nf);
}

int stencil_create(stencil_plan** out, int32_t kind, int32_t dtype, int32_t nx, int32_t ny, int32_t nz,
                   const stencil_params* p)
{
    if (!out) return fail(STENCIL_EINVAL, "out is NULL");
    *out = nullptr;
    if (!(kind_ok(kind) || kind == STENCIL_KIND_MIXED)) return fail(STENCIL_EINVAL, "unknown stencil kind");
    if (dtype != STENCIL_F64 && dtype != STENCIL_F32) return fail(STENCIL_EINVAL, "unknown dtype");
    if (kind != STENCIL_KIND_MIXED && (nx < 1 || ny < 1 || nz < 1))
        return fail(STENCIL_EINVAL, "interior extents must be >= 1");
    if (kind == STENCIL_KIND_MIXED && (nx < 0 || ny < 0 || nz < 0))
        return fail(STENCIL_EINVAL, "negative extents");
    stencil_plan* pl = new (std::nothrow) stencil_plan();
    if (!pl) return fail(STENCIL_ENOMEM, "plan allocation failed");
    std::memset(pl, 0, sizeof(*pl));
    pl->kind = kind;
    pl->dtype = dtype;
    pl->nx = nx;
    pl->ny = ny;
    pl->nz = nz;
    pl->autotune = (p == nullptr) || p->mode == STENCIL_MODE_AUTO;
    if (p && p->mode != STENCIL_MODE_AUTO) {
        if (p->mode == STENCIL_MODE_NAIVE) {
            pl->mode = STENCIL_MODE_NAIVE;
            pl->chosen = true;
        } else if (p->mode == STENCIL_MODE_MWD) {
            if (kind == STENCIL_KIND_MIXED) {
                delete pl;
                return fail(STENCIL_EINVAL, "explicit MWD parameters need a single kind");
            }
            MwdShape s = default_shape(kind, dtype);
            if (p->dw) s.dw = p->dw;
            if (p->lanes) {
                if (p->lanes % 64) {
                    delete pl;
                    return fail(STENCIL_EINVAL, "lanes must be a multiple of 64");
                }
                s.wpr = p->lanes / 64;
            }
            if (!mwd_supported(kind, dtype, s)) {
                delete pl;
                return fail(STENCIL_EUNSUPPORTED, "no MWD kernel for dw=" + std::to_string(s.dw) +
                                                      " lanes=" + std::to_string(64 * s.wpr));
            }
            pl->mode = STENCIL_MODE_MWD;
            pl->shape = s;
            pl->chosen = true;
        } else {
            delete pl;
            return fail(STENCIL_EINVAL, "unknown mode");
        }
    }
    *out = pl;
    return STENCIL_OK;
}

int stencil_destroy(stencil_plan* p)
{
    if (!p) return fail(STENCIL_EINVAL, "plan is NULL");
    // wait for this plan's own last run only (other streams keep running)
    if (p->done) {
        (void)hipEventSynchronize(p->done);
        (void)hipEventDestroy(p->done);
        p->done = nullptr;
    }
    free_scratch(p);
    batch_free(p->batch);
    if (p->prof) {
        double tmp[4];
        (void)p->prof->collect(tmp);
        delete p->prof;
    }
    delete p;
    return STENCIL_OK;
}

int stencil_run(stencil_plan* p, stencil_grid* g, const stencil_coeffs* c, int32_t T, void* stream)
{
    if (!p) return fail(STENCIL_EINVAL, "plan is NULL");
    if (p->kind == STENCIL_KIND_MIXED) return fail(STENCIL_EINVAL, "mixed plans run only batched");
    int rc = check_grid(g, "grid");
    if (rc) return rc;
    if (g->nx != p->nx || g->ny != p->ny || g->nz != p->nz)
        return fail(STENCIL_EINVAL, "grid extents differ from the plan's");
    if (g->dtype != p->dtype) return fail(STENCIL_EINVAL, "grid dtype differs from the plan's");
    if (g->halo < radius_of(p->kind)) return fail(STENCIL_EINVAL, "halo narrower than the stencil radius");
    if (T < 0) return fail(STENCIL_EINVAL, "T < 0");
    HostWeights w;
    rc = check_coeffs(c, p->kind, g, &w);
    if (rc) return rc;
    if (T == 0) return STENCIL_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!p->chosen) {
        TuneChoice tc;
        rc = tune_choose(p->kind, p->dtype, p->nx, p->ny, p->nz, T, &tc);
        if (rc) return rc;
        p->mode = tc.mode;
        p->shape = tc.shape;
        p->chosen = true;
    }
    // the MWD tile kernel addresses a padded plane with 32-bit byte offsets
    const bool plane_ok = mwd_plane_ok(g->sz, g->dtype);
    if (p->mode == STENCIL_MODE_MWD && !plane_ok) {
        if (!p->autotune)
            return fail(STENCIL_EUNSUPPORTED, "MWD needs a padded plane (sz elements) below 4 GiB");
    }
    const int mode = (p->mode == STENCIL_MODE_MWD && !plane_ok) ? STENCIL_MODE_NAIVE : p->mode;
    DevGrid d = to_dev(g);
    if (mode == STENCIL_MODE_NAIVE) {
        for (int t = 0; t < T; ++t) {
            if (p->prof) p->prof->begin(s);
            hipError_t e = naive_sweep(d, w, d.org[(d.cur + t) & 1], d.org[(d.cur + t + 1) & 1], s);
            if (p->prof) p->prof->end(s, 0);
            if (e != hipSuccess) return hip_fail(e, "naive sweep launch");
        }
    } else {
        rc = ensure_scratch(p, g);
        if (rc) return rc;
        hipError_t e = mwd_run(d, w, T, p->shape, p->scratch_org, s, p->prof);
        if (e != hipSuccess) return hip_fail(e, "MWD launch");
    }
    mark_done(p, s);
    g->cur ^= (T & 1);
    return STENCIL_OK;
}

int stencil_plan_describe(const stencil_plan* p, stencil_plan_desc* out)
{
    if (!p || !out) return fail(STENCIL_EINVAL, "NULL argument");
    std::memset(out, 0, sizeof(*out));
    out->kind = p->kind;
    out->dtype = p->dtype;
    out->mode = p->chosen ? p->mode : STENCIL_MODE_AUTO;
    if (p->chosen && p->mode == STENCIL_MODE_MWD && p->kind != STENCIL_KIND_MIXED) {
        out->dw = p->shape.dw;
        out->lanes = p->shape.lanes();
        out->xtile = mwd_xtile(p->kind, p->shape);
        out->levels = mwd_levels(p->kind, p->shape);
        out->model_bytes_per_lup = stencil_model_bytes_per_lup(p->kind, p->dtype, p->shape.dw);
    } else if (p->kind != STENCIL_KIND_MIXED) {
        out->model_bytes_per_lup = stencil_model_bytes_per_lup(p->kind, p->dtype, 0);
    }
    return STENCIL_OK;
}

int stencil_profile_enable(stencil_plan* p, int32_t enable)
{
    if (!p) return fail(STENCIL_EINVAL, "plan is NULL");
    if (enable) {
        if (!p->prof) {
            p->prof = new (std::nothrow) Prof();
            if (!p->prof) return fail(STENCIL_ENOMEM, "profiler allocation failed");
        }
        p->prof->on = true;
    } else if (p->prof) {
        p->prof->on = false;
    }
    return STENCIL_OK;
}

int stencil_profile_read(stencil_plan* p, double out[4])
{
    if (!p || !out) return fail(STENCIL_EINVAL, "NULL argument");
    if (!p->prof) {
        out[0] = out[1] = out[2] = out[3] = 0.0;
        return STENCIL_OK;
    }
    hipError_t e = p->prof->collect(out);
    if (e != hipSuccess) return hip_fail(e, "profile events");
    return STENCIL_OK;
}

int stencil_norms(const stencil_grid* g, int32_t which, double out[2], void* stream)
{
    int rc = check_grid(g, "grid");
    if (rc) return rc;
    if (!out) return fail(STENCIL_EINVAL, "out is NULL");
    if (which != 0 && which != 1) return fail(STENCIL_EINVAL, "which must be 0 or 1");
    DevGrid d = to_dev(g);
    hipError_t e = norms_fp64(d, d.org[d.cur], d, d.org[d.cur ^ 1], which, out,
                              static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "norms");
    return STENCIL_OK;
}

int stencil_diff_norms(const stencil_grid* a, const stencil_grid* b, double out[2], void* stream)
{
    int rc = check_grid(a, "a");
    if (rc) return rc;
    rc = check_grid(b, "b");
    if (rc) return rc;
    if (!out) return fail(STENCIL_EINVAL, "out is NULL");
    if (a->nx != b->nx || a->ny != b->ny || a->nz != b->nz)
        return fail(STENCIL_EINVAL, "grids have different interior extents");
    DevGrid da = to_dev(a), db = to_dev(b);
    hipError_t e = norms_fp64(da, da.org[da.cur], db, db.org[db.cur], 1, out, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "diff norms");
    return STENCIL_OK;
}

int stencil_stream_copy(void* dst, const void* src, int64_t bytes, void* stream)
{
    if (!dst || !src) return fail(STENCIL_EINVAL, "NULL pointer");
    if (bytes < 0 || bytes % 16) return fail(STENCIL_EINVAL, "size must be a non-negative multiple of 16");
    if ((reinterpret_cast<uintptr_t>(dst) % 16) || (reinterpret_cast<uintptr_t>(src) % 16))
        return fail(STENCIL_EINVAL, "pointers must be 16-byte aligned");
    hipError_t e = stream_copy(dst, src, bytes, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "stream copy");
    return STENCIL_OK;
}

int stencil_run_batched(stencil_plan* p, stencil_grid* grids, const stencil_coeffs* coeffs, int32_t n,
                        int32_t T, void* stream)
{
    if (!p) return fail(STENCIL_EINVAL, "plan is NULL");
    const int rc = batch_run(p->kind, p->dtype, &p->batch, grids, coeffs, n, T, static_cast<hipStream_t>(stream));
    if (rc == STENCIL_OK) mark_done(p, static_cast<hipStream_t>(stream));
    return rc;
}

int stencil_kernel_resources(int32_t kind, int32_t dtype, int32_t dw, int32_t lanes, int32_t out[5])
{
    if (!kind_ok(kind) || (dtype != STENCIL_F64 && dtype != STENCIL_F32) || !out)
        return fail(STENCIL_EINVAL, "bad kind, dtype or out");
    if (lanes <= 0 || lanes % 64) return fail(STENCIL_EINVAL, "lanes must be a positive multiple of 64");
    const MwdShape s{dw, lanes / 64};
    if (!mwd_supported(kind, dtype, s)) return fail(STENCIL_EUNSUPPORTED, "no MWD kernel for this shape");
    int r[5];
    hipError_t e = mwd_kernel_resources(kind, dtype, s, r);
    if (e != hipSuccess) return hip_fail(e, "kernel attributes");
    for (int i = 0; i < 5; ++i) out[i] = r[i];
    return STENCIL_OK;
}

int stencil_norms_noalloc(const stencil_grid* g, int32_t which, double* out_dev, void* stream)
{
    int rc = check_grid(g, "grid");
    if (rc) return rc;
    if (!out_dev) return fail(STENCIL_EINVAL, "out_dev is NULL");
    if (reinterpret_cast<uintptr_t>(out_dev) % sizeof(double))
        return fail(STENCIL_EINVAL, "out_dev is not 8-byte aligned");
    if (which != 0 && which != 1) return fail(STENCIL_EINVAL, "which must be 0 or 1");
    DevGrid d = to_dev(g);
    hipError_t e = norms_fp64_static(d, d.org[d.cur], d, d.org[d.cur ^ 1], which, out_dev,
                                     static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "norms (static scratch)");
    return STENCIL_OK;
}

}  // extern "C"
