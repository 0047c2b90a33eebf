// Autotuner: choose between the naive sweep and the compiled MWD shapes
// (diamond width, x lanes) by timing them on a proxy grid of the same x-y
// extent, in the spirit of the paper's auto-tuning of diamond width,
// frontlines and x-tile (Sec. II-A, Sec. IV-B).  The search space is pruned
// as the paper prunes it, by the cache block: a shape whose wavefront cache
// block (Eq. 3 of Sec. III-B, with N_F = 1 and N_xb = lanes x element size)
// exceeds half of a CU's on-chip storage (LDS plus registers; the model holds
// while the block fills at most about half of the cache, Sec. IV-B) is not
// tried, and neither is a shape whose compiled kernel spills more than a few
// registers to scratch memory.  Each candidate's time for the whole run is
// predicted from a few timed sweeps or diamond rows.  Choices are cached per
// device, stencil, grid size and T for the life of the process and, if
// MWD_TUNE_CACHE names a file, across processes.  MWD_TUNE_VERBOSE=1 prints
// every pruning decision and every prediction to stderr.
#include "tune.hpp"

#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/mwd_stencil.h"
#include "batch.hpp"
#include "batch_variants.hpp"

namespace mwd {

double cache_block_model(int kind, int dtype, int dw, int lanes, int nf)
{
    const double R = radius_of(kind), ND = ndomain_of(kind), Dw = dw, NF = nf;
    const double Nxb = (double)lanes * (dtype == 0 ? 8.0 : 4.0);
    const double Ww = Dw - 2.0 * R + NF;
    return Nxb * (ND * Dw * (Dw / 2.0 - R + NF) + 2.0 * R * (Dw + Ww));
}

MwdShape default_shape(int kind, int dtype)
{
    if (kind == K25C || kind == K25V) return MwdShape{16, 1};
    if (kind == K7V && dtype == 0) return MwdShape{8, 1};
    return MwdShape{8, 2};
}

namespace {

using Key = std::tuple<int, int, int, int, int, int, int, int>;  // dev kind dtype nx ny nz T batch

std::mutex g_mu;
std::map<Key, TuneChoice> g_cache;
bool g_file_loaded = false;

// The proxy grid holds at most this many bytes (its arrays: two levels, four
// scratch arrays, the coefficient arrays) and at least this many planes.
constexpr size_t kProxyBytes = size_t(8) << 30;
constexpr int kMinProxyNz = 64;
// A tile kernel that spills more than this to scratch memory (bytes per lane)
// is not tried; a few spilled registers outside the step loop cost little.
constexpr size_t kMaxSpillBytes = 128;
// On-chip storage of one CU of gfx950: 160 KiB of LDS and a 512 KiB vector
// register file.
constexpr double kCuOnChipBytes = (160.0 + 512.0) * 1024.0;

double cache_block_bytes(int kind, int dtype, const MwdShape& s)
{
    return mwd::cache_block_model(kind, dtype, s.dw, s.lanes(), 1);
}


bool tune_verbose()
{
    const char* ve = std::getenv("MWD_TUNE_VERBOSE");
    return ve && *ve && *ve != '0';
}

const char* cache_path()
{
    const char* p = std::getenv("MWD_TUNE_CACHE");
    return (p && *p) ? p : nullptr;
}

void load_file()
{
    if (g_file_loaded) return;
    g_file_loaded = true;
    const char* path = cache_path();
    if (!path) return;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    int v[11];
    while (std::fscanf(f, "%d %d %d %d %d %d %d %d %d %d %d", &v[0], &v[1], &v[2], &v[3], &v[4], &v[5], &v[6],
                       &v[7], &v[8], &v[9], &v[10]) == 11) {
        g_cache[Key{v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7]}] = TuneChoice{v[8], MwdShape{v[9], v[10]}};
    }
    std::fclose(f);
}

void save_entry(const Key& k, const TuneChoice& c)
{
    const char* path = cache_path();
    if (!path) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%d %d %d %d %d %d %d %d %d %d %d\n", std::get<0>(k), std::get<1>(k), std::get<2>(k),
                 std::get<3>(k), std::get<4>(k), std::get<5>(k), std::get<6>(k), std::get<7>(k), c.mode,
                 c.shape.dw, c.shape.wpr);
    std::fclose(f);
}

// MWD_TUNE=naive or MWD_TUNE=mwd:<dw>:<lanes> forces a choice (measurement sweeps).
bool forced(int kind, int dtype, TuneChoice* out)
{
    const char* e = std::getenv("MWD_TUNE");
    if (!e || !*e) return false;
    if (std::strcmp(e, "naive") == 0) {
        *out = TuneChoice{STENCIL_MODE_NAIVE, MwdShape{0, 0}};
        return true;
    }
    int dw = 0, lanes = 0;
    if (std::sscanf(e, "mwd:%d:%d", &dw, &lanes) == 2 && lanes % 64 == 0) {
        MwdShape s{dw, lanes / 64};
        if (mwd_supported(kind, dtype, s)) {
            *out = TuneChoice{STENCIL_MODE_MWD, s};
            return true;
        }
    }
    return false;
}

struct Proxy {
    std::vector<void*> allocs;
    DevGrid g{};
    HostWeights w{};
    void* scratch[4] = {nullptr, nullptr, nullptr, nullptr};
    ~Proxy() {
        for (void* p : allocs) (void)hipFree(p);
    }
    bool alloc(size_t bytes, void** base) {
        if (hipMalloc(base, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        allocs.push_back(*base);
        return hipMemset(*base, 0, bytes) == hipSuccess;
    }
};

bool make_proxy(Proxy& P, int kind, int dtype, int nx, int ny, int nz)
{
    const int h = radius_of(kind);
    const size_t es = dtype == 0 ? 8 : 4;
    P.g.nx = nx;
    P.g.ny = ny;
    P.g.nz = nz;
    P.g.halo = h;
    P.g.sy = nx + 2 * h;
    P.g.sz = P.g.sy * (ny + 2 * h);
    P.g.dtype = dtype;
    P.g.cur = 0;
    const size_t bytes = (size_t)P.g.sz * (nz + 2 * h) * es;
    const long long off = (long long)h * P.g.sz + (long long)h * P.g.sy + h;
    void* base = nullptr;
    for (int i = 0; i < 2; ++i) {
        if (!P.alloc(bytes, &base)) return false;
        P.g.org[i] = static_cast<char*>(base) + off * es;
    }
    for (int i = 0; i < 4; ++i) {
        if (!P.alloc(bytes, &base)) return false;
        P.scratch[i] = static_cast<char*>(base) + off * es;
    }
    P.w.kind = kind;
    for (int m = 0; m < 13; ++m) {
        P.w.c[m] = 0.05;
        P.w.org[m] = nullptr;
    }
    for (int m = 0; m < narr_of(kind); ++m) {
        if (!P.alloc(bytes, &base)) return false;
        P.w.org[m] = static_cast<char*>(base) + off * es;
    }
    return true;
}

// Milliseconds of one call of f, averaged over three calls after a warm-up
// call, or a negative value.
template <class F>
double time_ms(F&& f, hipStream_t s)
{
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -1.0;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return -1.0;
    }
    double ms = -1.0;
    hipError_t e = f();  // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int r = 0; r < 3 && e == hipSuccess; ++r) e = f();
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.f;
    if (e == hipSuccess && hipEventElapsedTime(&t, e0, e1) == hipSuccess) ms = t / 3.0;
    (void)hipGetLastError();
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ms;
}

// Predicted milliseconds of a whole run of T steps over nz planes with the
// given choice, from timing a part of it on the proxy (nzp planes): a few
// sweeps of the naive schedule, or a few interior diamond rows of MWD (each
// row costs about the same; the first and last rows are partial and count
// as one row together).
double predict_ms(Proxy& P, int T, int nz, const TuneChoice& c, hipStream_t s)
{
    const double zscale = (double)nz / (double)P.g.nz;
    if (c.mode == STENCIL_MODE_NAIVE) {
        const int ns = T < 4 ? (T > 0 ? T : 1) : 4;
        const double ms = time_ms([&]() -> hipError_t {
            for (int t = 0; t < ns; ++t) {
                hipError_t e = naive_sweep(P.g, P.w, P.g.org[t & 1], P.g.org[(t + 1) & 1], s);
                if (e != hipSuccess) return e;
            }
            return hipSuccess;
        }, s);
        return ms < 0 ? ms : ms / ns * T * zscale;
    }
    const int h = c.shape.dw / (2 * radius_of(P.w.kind));
    const int rho_max = (T + h - 1) / h;
    if (rho_max <= 4) {
        const double ms = time_ms([&]() { return mwd_run(P.g, P.w, T, c.shape, P.scratch, s, nullptr); }, s);
        return ms < 0 ? ms : ms * zscale;
    }
    constexpr int kRows = 3;
    const double ms = time_ms([&]() { return mwd_run_rows(P.g, P.w, T, c.shape, P.scratch, s, 1, kRows); }, s);
    return ms < 0 ? ms : ms / kRows * rho_max * zscale;
}

int tune_generic(int kind, int dtype, int nx, int ny, int nz, int T, int batch, TuneChoice* out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return STENCIL_EDEVICE;
    const Key key{dev, kind, dtype, nx, ny, nz, T, batch};
    std::lock_guard<std::mutex> lk(g_mu);
    load_file();
    auto it = g_cache.find(key);
    if (it != g_cache.end()) {
        *out = it->second;
        return STENCIL_OK;
    }
    // candidates (for a batch also the index of the batched tile variant)
    std::vector<TuneChoice> cands;
    std::vector<int> cand_var;
    if (batch) {
        // batch 1: the batched naive sweep or a batched MWD shape; 2: MWD only
        if (batch == 1) {
            cands.push_back(TuneChoice{STENCIL_MODE_NAIVE, MwdShape{0, 0}});
            cand_var.push_back(-1);
        }
        const int nv = dtype == 0 ? kNumBatchVariantsF64 : kNumBatchVariants;
        for (int i = 0; i < nv; ++i)
            if (kBatchVariantInfo[i].kind == kind) {
                cands.push_back(TuneChoice{STENCIL_MODE_MWD, MwdShape{kBatchVariantInfo[i].dw, kBatchVariantInfo[i].wpr}});
                cand_var.push_back(i);
            }
    } else {
        cands.push_back(TuneChoice{STENCIL_MODE_NAIVE, MwdShape{0, 0}});
        // the proxy's plane (and the run's, at least as large) must be one the
        // MWD kernel can address; otherwise MWD is not timed at all
        const int h = radius_of(kind);
        const long long proxy_sz = (long long)(nx + 2 * h) * (long long)(ny + 2 * h);
        MwdShape shapes[16];
        const bool plane_ok = mwd_plane_ok(proxy_sz, dtype);
        const int ns = plane_ok ? mwd_shapes(kind, dtype, shapes, 16) : 0;
        if (!plane_ok && tune_verbose())
            std::fprintf(stderr, "[mwd tune] kind %d dtype %d %dx%d: plane of 4 GiB or more, naive only\n", kind,
                         dtype, nx, ny);
        for (int i = 0; i < ns; ++i) {
            size_t scratch = 0;
            const bool spill_ok =
                mwd_kernel_scratch(kind, dtype, shapes[i], &scratch) == hipSuccess && scratch <= kMaxSpillBytes;
            const double cs = cache_block_bytes(kind, dtype, shapes[i]);
            const bool cs_ok = cs <= 0.5 * kCuOnChipBytes;
            if (tune_verbose())
                std::fprintf(stderr, "[mwd tune] kind %d dtype %d dw %d lanes %d: cache block (Eq. 3) %.1f KiB of "
                             "%.0f KiB on chip, spill %zu B/lane: %s\n", kind, dtype, shapes[i].dw,
                             shapes[i].lanes(), cs / 1024.0, kCuOnChipBytes / 1024.0, scratch,
                             !cs_ok ? "pruned (cache block above half the on-chip storage)"
                                    : !spill_ok ? "pruned (register spill)" : "candidate");
            if (spill_ok && cs_ok) cands.push_back(TuneChoice{STENCIL_MODE_MWD, shapes[i]});
        }
    }
    if (cands.empty()) return STENCIL_EUNSUPPORTED;
    TuneChoice best = cands[0];
    const bool verbose = tune_verbose();
    if (cands.size() > 1 && batch) {
        // the batched graph itself, timed on a proxy batch of copies of this
        // bucket's grid (as many as make about 2^26 points, 2 to 64 grids)
        const long long pts = std::max(1LL, (long long)nx * ny * nz);
        const int count = (int)std::max(2LL, std::min(64LL, (1LL << 26) / pts));
        double best_per = -1.0;
        for (size_t ci = 0; ci < cands.size(); ++ci) {
            const TuneChoice& c = cands[ci];
            const double ms = batch_proxy_ms(kind, dtype, nx, ny, nz, T, count, cand_var[ci]);
            if (verbose)
                std::fprintf(stderr, "[mwd tune] kind %d dtype %d %dx%dx%d T=%d (batched proxy: %d grids): %s dw %d "
                             "lanes %d: %.3f ms, %.2f GLUP/s\n", kind, dtype, nx, ny, nz, T, count,
                             c.mode == STENCIL_MODE_NAIVE ? "naive" : "mwd", c.shape.dw, c.shape.wpr * 64, ms,
                             ms > 0 ? (double)count * pts * T / (ms * 1e6) : 0.0);
            if (ms > 0 && (best_per < 0 || ms < best_per)) {
                best_per = ms;
                best = c;
            }
        }
    } else if (cands.size() > 1) {
        // proxy: the same x-y extent, and as many planes as fit the budget
        const int h = radius_of(kind);
        const size_t es = dtype == 0 ? 8 : 4;
        const size_t plane = (size_t)(nx + 2 * h) * (size_t)(ny + 2 * h) * es;
        const size_t arrays = 6 + (size_t)narr_of(kind);
        const long long fit = (long long)(kProxyBytes / (arrays * plane)) - 2 * h;
        const int nzp = (int)std::max<long long>(std::min<long long>(nz, kMinProxyNz), std::min<long long>(nz, fit));
        Proxy P;
        hipStream_t s = nullptr;
        double best_ms = -1.0;
        if (make_proxy(P, kind, dtype, nx, ny, nzp) && hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess) {
            for (const TuneChoice& c : cands) {
                const double ms = predict_ms(P, T, nz, c, s);
                if (verbose)
                    std::fprintf(stderr, "[mwd tune] kind %d dtype %d %dx%dx%d (proxy %d planes) T=%d: %s dw %d "
                                 "lanes %d: predicted %.3f ms, %.2f GLUP/s\n", kind, dtype, nx, ny, nz, nzp, T,
                                 c.mode == STENCIL_MODE_NAIVE ? "naive" : "mwd", c.shape.dw, c.shape.wpr * 64, ms,
                                 ms > 0 ? (double)nx * ny * nz * T / (ms * 1e6) : 0.0);
                if (ms > 0 && (best_ms < 0 || ms < best_ms)) {
                    best_ms = ms;
                    best = c;
                }
            }
            (void)hipStreamDestroy(s);
        }
        (void)hipGetLastError();
    }
    if (verbose)
        std::fprintf(stderr, "[mwd tune] kind %d dtype %d %dx%dx%d T=%d%s: chose %s dw %d lanes %d\n", kind, dtype,
                     nx, ny, nz, T, batch ? " (batched)" : "", best.mode == STENCIL_MODE_NAIVE ? "naive" : "mwd",
                     best.shape.dw, best.shape.wpr * 64);
    g_cache[key] = best;
    save_entry(key, best);
    *out = best;
    return STENCIL_OK;
}

}  // namespace

int tune_choose(int kind, int dtype, int nx, int ny, int nz, int T, TuneChoice* out)
{
    if (forced(kind, dtype, out)) return STENCIL_OK;
    return tune_generic(kind, dtype, nx, ny, nz, T, 0, out);
}

TuneChoice tune_batch_choose(int kind, int dtype, int nx, int ny, int nz, int T)
{
    const char* e = std::getenv("MWD_TUNE");
    if (e && std::strcmp(e, "naive") == 0) return TuneChoice{STENCIL_MODE_NAIVE, MwdShape{0, 0}};
    const int nv = dtype == 0 ? kNumBatchVariantsF64 : kNumBatchVariants;
    // MWD_TUNE=mwd:<dw>:<lanes>: that batched tile shape for the kinds that
    // have it, the naive sweep for the others
    int fdw = 0, flanes = 0;
    if (e && std::sscanf(e, "mwd:%d:%d", &fdw, &flanes) == 2) {
        for (int i = 0; i < nv; ++i)
            if (kBatchVariantInfo[i].kind == kind && kBatchVariantInfo[i].dw == fdw &&
                64 * kBatchVariantInfo[i].wpr == flanes)
                return TuneChoice{STENCIL_MODE_MWD, MwdShape{fdw, kBatchVariantInfo[i].wpr}};
        return TuneChoice{STENCIL_MODE_NAIVE, MwdShape{0, 0}};
    }
    const bool mwd_only = e && std::strncmp(e, "mwd", 3) == 0;
    // bucket the extents so that a batch of many uneven grids tunes a few
    // representative sizes
    auto bucket = [](int n) { return n <= 64 ? 64 : n <= 128 ? 128 : 256; };
    TuneChoice c;
    if (tune_generic(kind, dtype, bucket(nx), bucket(ny), bucket(nz), T, mwd_only ? 2 : 1, &c) == STENCIL_OK)
        return c;
    // the first compiled variant of this kind
    for (int i = 0; i < nv; ++i)
        if (kBatchVariantInfo[i].kind == kind)
            return TuneChoice{STENCIL_MODE_MWD, MwdShape{kBatchVariantInfo[i].dw, kBatchVariantInfo[i].wpr}};
    return TuneChoice{STENCIL_MODE_NAIVE, MwdShape{0, 0}};
}

}  // namespace mwd
