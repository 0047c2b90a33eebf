// Host side of the batched form: tile table, per-grid shapes, scratch, the
// captured hipGraph and its replay.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "batch.hpp"
#include "batch_naive.hpp"
#include "batch_variants.hpp"
#include "internal.hpp"
#include "tune.hpp"

namespace mwd {

int check_grid(const stencil_grid* g, const char* name);
DevGrid to_dev(const stencil_grid* g);
int check_coeffs(const stencil_coeffs* c, int kind, const stencil_grid* g, HostWeights* out);

struct BatchKey {
    std::vector<uintptr_t> ptrs;
    std::vector<long long> dims;
    int T, dtype;
    bool operator==(const BatchKey& o) const {
        return T == o.T && dtype == o.dtype && ptrs == o.ptrs && dims == o.dims;
    }
};

struct BatchGraph {
    BatchKey key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void* dev = nullptr;        // tiles | gargs | gvariant | halo table
    void* scratch = nullptr;    // two extra buffer pairs per grid
    int ntiles = 0;
    std::vector<int> variants;  // chosen variant per grid (for reporting)
    void release() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (dev) (void)hipFree(dev);
        if (scratch) (void)hipFree(scratch);
        exec = nullptr;
        graph = nullptr;
        dev = scratch = nullptr;
    }
};

struct BatchState {
    std::vector<BatchGraph> cache;  // at most two: runs with odd T alternate cur
};

static size_t es_of(int dtype) { return dtype == 0 ? 8 : 4; }

// run of adjacent tiles given to one XCD in a batched row group
constexpr int kBatchXcdRun = 4;
// arrays of one group of naive grids; kNaiveBranches groups run at a time,
// together within the 256 MiB last-level cache
constexpr size_t kCacheGroupBytes = size_t(96) << 20;
constexpr int kNaiveBranches = 2;

// The group budget; MWD_BATCH_GROUP_BYTES (environment, bytes) overrides it,
// for tests that need many groups from a few small grids.
static size_t cache_group_bytes()
{
    const char* e = std::getenv("MWD_BATCH_GROUP_BYTES");
    if (e && *e) {
        const long long v = std::atoll(e);
        if (v > 0) return (size_t)v;
    }
    return kCacheGroupBytes;
}
// workgroups per launch below which a group's z chunks are halved
constexpr long long kNaiveMinBlocks = 2048;
// runs of this many consecutive naive blocks (neighbours in x and y, whose
// halos overlap) go to one XCD: the blocks one XCD holds at once
constexpr int kNaiveXcdRun = 64;

static int variant_index(int kind, int dtype, const MwdShape& s)
{
    const int nv = dtype == 0 ? kNumBatchVariantsF64 : kNumBatchVariants;
    for (int i = 0; i < nv; ++i)
        if (kBatchVariantInfo[i].kind == kind && kBatchVariantInfo[i].dw == s.dw && kBatchVariantInfo[i].wpr == s.wpr)
            return i;
    return -1;
}

template <typename T>
static void fill_args(MwdArgs<T>& a, const DevGrid& d, const HostWeights& w, T* const pr[4], int T_steps)
{
    std::memset(&a, 0, sizeof(a));
    a.pair[0][0] = static_cast<T*>(d.org[0]);
    a.pair[0][1] = static_cast<T*>(d.org[1]);
    a.pair[1][0] = pr[0];
    a.pair[1][1] = pr[1];
    a.pair[2][0] = pr[2];
    a.pair[2][1] = pr[3];
    a.halo = static_cast<const T*>(d.org[d.cur]);
    for (int m = 0; m < 13; ++m) {
        a.w.c[m] = static_cast<T>(w.c[m]);
        a.w.arr[m] = static_cast<const T*>(w.org[m]);
    }
    a.nx = d.nx;
    a.ny = d.ny;
    a.nz = d.nz;
    a.sy = d.sy;
    a.sz = d.sz;
    a.cur = d.cur;
    a.nsteps = T_steps;
}

template <typename T>
static int build_graph(BatchGraph& bg, stencil_grid* grids, const HostWeights* hw, int n, int T_steps,
                       int dtype, std::string* errmsg, const int* forced = nullptr)
{
    // 1. schedule per grid (autotuned per kind and size bucket, or forced):
    //    the batched naive sweep (var -1) or a batched MWD shape
    std::vector<int> var(n);
    for (int i = 0; i < n; ++i) {
        if (forced) {
            var[i] = (forced[i] >= 0 && mwd_plane_ok(grids[i].sz, dtype)) ? forced[i] : -1;
            continue;
        }
        const TuneChoice c = tune_batch_choose(hw[i].kind, dtype, grids[i].nx, grids[i].ny, grids[i].nz, T_steps);
        // the tile kernel addresses a plane with 32-bit byte offsets
        if (c.mode == STENCIL_MODE_NAIVE || !mwd_plane_ok(grids[i].sz, dtype)) {
            var[i] = -1;
            continue;
        }
        int v = variant_index(hw[i].kind, dtype, c.shape);
        if (v < 0) {
            *errmsg = "no batched tile shape for kind " + std::to_string(hw[i].kind);
            return STENCIL_EUNSUPPORTED;
        }
        var[i] = v;
    }
    // 2. scratch: two extra pairs per grid, each laid out like the grid
    std::vector<size_t> soff(n + 1, 0);
    for (int i = 0; i < n; ++i) {
        const size_t bytes = (size_t)grids[i].sz * (size_t)(grids[i].nz + 2 * grids[i].halo) * es_of(dtype);
        const size_t aligned = (bytes + 255) & ~size_t(255);
        soff[i + 1] = soff[i] + (var[i] >= 0 ? 4 * aligned : 0);
    }
    if (hipMalloc(&bg.scratch, soff[n] ? soff[n] : 256) != hipSuccess) {
        (void)hipGetLastError();
        bg.scratch = nullptr;
        *errmsg = "batched scratch allocation of " + std::to_string(soff[n]) + " bytes failed";
        return STENCIL_ENOMEM;
    }
    // 3. tile table, rows of all grids interleaved row by row (topological)
    std::vector<MwdArgs<T>> gargs(n);
    std::vector<HaloFill<T>> halo(n);
    int hgx = 1, hgy = 1;
    std::vector<BatchTile> tiles;
    std::vector<int> rows(n), nxt(n);
    int max_rows = 0;
    std::vector<NaiveArgs<T>> nargs(n);
    std::vector<NaiveTile> ntiles;
    for (int i = 0; i < n; ++i) {
        DevGrid d = to_dev(&grids[i]);
        if (var[i] < 0) {
            // naive: (x block, y block, z chunk) entries of this grid
            NaiveArgs<T>& na = nargs[i];
            std::memset(&na, 0, sizeof(na));
            na.buf[0] = static_cast<T*>(d.org[0]);
            na.buf[1] = static_cast<T*>(d.org[1]);
            for (int m = 0; m < 13; ++m) {
                na.w.c[m] = static_cast<T>(hw[i].c[m]);
                na.w.arr[m] = static_cast<const T*>(hw[i].org[m]);
            }
            na.kind = hw[i].kind;
            na.nx = d.nx;
            na.ny = d.ny;
            na.nz = d.nz;
            na.zchunk = 64;  // set per group below
            na.cur = d.cur;
            na.sy = d.sy;
            na.sz = d.sz;
            std::memset(&gargs[i], 0, sizeof(gargs[i]));
            std::memset(&halo[i], 0, sizeof(halo[i]));  // nx = 0: the fill skips it
            rows[i] = 0;
            nxt[i] = 0;
            continue;
        }
        const BatchVariantInfo& vi = kBatchVariantInfo[var[i]];
        const MwdShape s{vi.dw, vi.wpr};
        const int R = radius_of(vi.kind), H = vi.dw / (2 * R);
        const int XT = mwd_xtile(vi.kind, s);
        const size_t es = es_of(dtype);
        const size_t bytes = (soff[i + 1] - soff[i]) / 4;
        const long long off = (long long)d.halo * d.sz + (long long)d.halo * d.sy + d.halo;
        T* pr[4];
        for (int k = 0; k < 4; ++k)
            pr[k] = reinterpret_cast<T*>(static_cast<char*>(bg.scratch) + soff[i] + k * bytes + off * es);
        fill_args<T>(gargs[i], d, hw[i], pr, T_steps);
        HaloFill<T>& hf = halo[i];
        hf.src = gargs[i].halo;
        for (int k = 0; k < 4; ++k) hf.dst[k] = pr[k];
        hf.nx = d.nx;
        hf.ny = d.ny;
        hf.nz = d.nz;
        hf.r = R;
        hf.sy = d.sy;
        hf.sz = d.sz;
        hgx = std::max(hgx, (d.nx + 2 * R + 63) / 64);
        hgy = std::max(hgy, (d.ny + 2 * R + 3) / 4);
        nxt[i] = (d.nx + XT - 1) / XT;
        gargs[i].nxt = nxt[i];
        rows[i] = (T_steps + H - 1) / H + 1;  // rows 0 .. rho_max
        max_rows = std::max(max_rows, rows[i]);
    }
    // naive grids in groups whose arrays fit the last-level cache; a group
    // runs all T steps before the next one starts
    std::vector<std::pair<int, int>> ngroups;  // (first table entry, count)
    {
        std::vector<int> nidx;
        for (int i = 0; i < n; ++i)
            if (var[i] < 0) nidx.push_back(i);
        const size_t group_bytes = cache_group_bytes();
        size_t k = 0;
        while (k < nidx.size()) {
            size_t bytes = 0, k1 = k;
            while (k1 < nidx.size()) {
                const stencil_grid& gg = grids[nidx[k1]];
                const size_t gb = (size_t)(2 + narr_of(hw[nidx[k1]].kind)) * (size_t)gg.sz *
                                  (size_t)(gg.nz + 2 * gg.halo) * es_of(dtype);
                if (k1 > k && bytes + gb > group_bytes) break;
                bytes += gb;
                ++k1;
            }
            // z chunks short enough that a group's launch has work for
            // every CU several times over
            long long cols = 0;
            for (size_t q = k; q < k1; ++q) {
                const stencil_grid& gg = grids[nidx[q]];
                cols += (long long)((gg.nx + kNaiveBX - 1) / kNaiveBX) * ((gg.ny + kNaiveBY - 1) / kNaiveBY) * gg.nz;
            }
            int zc = 64;
            while (zc > 16 && cols / zc < kNaiveMinBlocks) zc /= 2;
            const int first = (int)ntiles.size();
            for (size_t q = k; q < k1; ++q) {
                const int i = nidx[q];
                NaiveArgs<T>& na = nargs[i];
                na.zchunk = zc;
                for (int bz = 0; bz * zc < na.nz; ++bz)
                    for (int by = 0; by * kNaiveBY < na.ny; ++by)
                        for (int bx = 0; bx * kNaiveBX < na.nx; ++bx) ntiles.push_back(NaiveTile{i, bx, by, bz});
            }
            const int cnt = (int)ntiles.size() - first;
            std::vector<NaiveTile> g(ntiles.begin() + first, ntiles.end());
            for (int q = 0; q < cnt; ++q) ntiles[first + q] = g[xcd_tile(q, cnt, kNaiveXcdRun)];
            ngroups.emplace_back(first, cnt);
            k = k1;
        }
    }
    std::vector<int> group_first;  // table index where each row group starts
    for (int rho = 0; rho < max_rows; ++rho) {
        const size_t gstart = tiles.size();
        group_first.push_back((int)gstart);
        // larger grids first within a group
        std::vector<int> order;
        for (int i = 0; i < n; ++i)
            if (rho < rows[i]) order.push_back(i);
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
            return (long long)grids[a].nx * grids[a].ny * grids[a].nz > (long long)grids[b].nx * grids[b].ny * grids[b].nz;
        });
        for (int i : order) {
            const BatchVariantInfo& vi = kBatchVariantInfo[var[i]];
            const int R = radius_of(vi.kind), H = vi.dw / (2 * R);
            const int yoff = (rho % 2) * (vi.dw / 2);
            const int ybase = yoff > 0 ? yoff - vi.dw : 0;
            const int nB = (grids[i].ny - 1 - ybase) / vi.dw + 1;
            for (int b = 0; b < nB; ++b)
                for (int j = 0; j < nxt[i]; ++j)
                    tiles.push_back(BatchTile{i, 0, rho, (rho - 1) * H, ybase, b, j, 0});
        }
        // workgroup k of the group runs entry k; place runs of adjacent x
        // tiles on one XCD (as the row kernel does)
        const int cnt = (int)(tiles.size() - gstart);
        std::vector<BatchTile> g(tiles.begin() + gstart, tiles.end());
        for (int k = 0; k < cnt; ++k) tiles[gstart + k] = g[xcd_tile(k, cnt, kBatchXcdRun)];
    }
    // the gather of every grid's last two levels
    group_first.push_back((int)tiles.size());
    for (int i = 0; i < n; ++i) {
        if (var[i] < 0) continue;
        const int zc = std::max(1, (int)(65536 / std::max(1LL, (long long)grids[i].nx * grids[i].ny)));
        for (int z0 = 0; z0 < grids[i].nz; z0 += zc)
            tiles.push_back(BatchTile{i, 1, -1, 0, 0, z0, std::min(zc, grids[i].nz - z0), 0});
    }
    group_first.push_back((int)tiles.size());
    // 4. device tables
    const size_t tb = tiles.size() * sizeof(BatchTile);
    const size_t ab = (size_t)n * sizeof(MwdArgs<T>);
    const size_t vb = (size_t)n * sizeof(int);
    const size_t hb = (size_t)n * sizeof(HaloFill<T>);
    const size_t ntb = ntiles.size() * sizeof(NaiveTile);
    const size_t nab = (size_t)n * sizeof(NaiveArgs<T>);
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    if (hipMalloc(&bg.dev, al(tb) + al(ab) + al(vb) + al(hb) + al(ntb) + al(nab)) != hipSuccess) {
        (void)hipGetLastError();
        bg.dev = nullptr;
        *errmsg = "batched table allocation failed";
        return STENCIL_ENOMEM;
    }
    char* base = static_cast<char*>(bg.dev);
    BatchTile* d_tiles = reinterpret_cast<BatchTile*>(base);
    MwdArgs<T>* d_args = reinterpret_cast<MwdArgs<T>*>(base + al(tb));
    int* d_var = reinterpret_cast<int*>(base + al(tb) + al(ab));
    HaloFill<T>* d_halo = reinterpret_cast<HaloFill<T>*>(base + al(tb) + al(ab) + al(vb));
    NaiveTile* d_ntiles = reinterpret_cast<NaiveTile*>(base + al(tb) + al(ab) + al(vb) + al(hb));
    NaiveArgs<T>* d_nargs = reinterpret_cast<NaiveArgs<T>*>(base + al(tb) + al(ab) + al(vb) + al(hb) + al(ntb));
    hipError_t e = hipMemcpy(d_tiles, tiles.data(), tb, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_args, gargs.data(), ab, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_var, var.data(), vb, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_halo, halo.data(), hb, hipMemcpyHostToDevice);
    if (e == hipSuccess && ntb) e = hipMemcpy(d_ntiles, ntiles.data(), ntb, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_nargs, nargs.data(), nab, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        *errmsg = std::string("batched table upload: ") + hipGetErrorString(e);
        return STENCIL_EDEVICE;
    }
    bg.ntiles = (int)tiles.size();
    bg.variants = var;
    // 5. capture one launch per group, in order, into a graph
    hipStream_t cs = nullptr;
    e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) {
        *errmsg = std::string("stream: ") + hipGetErrorString(e);
        return STENCIL_EDEVICE;
    }
    // branch streams and fork/join events for the naive groups
    hipStream_t bstreams[kNaiveBranches - 1] = {};
    hipEvent_t fork_ev = nullptr, join_ev[kNaiveBranches - 1] = {};
    if (e == hipSuccess) e = hipEventCreateWithFlags(&fork_ev, hipEventDisableTiming);
    for (int b = 0; b < kNaiveBranches - 1 && e == hipSuccess; ++b) {
        e = hipStreamCreateWithFlags(&bstreams[b], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&join_ev[b], hipEventDisableTiming);
    }
    auto release_branches = [&]() {
        for (int b = 0; b < kNaiveBranches - 1; ++b) {
            if (bstreams[b]) (void)hipStreamDestroy(bstreams[b]);
            if (join_ev[b]) (void)hipEventDestroy(join_ev[b]);
        }
        if (fork_ev) (void)hipEventDestroy(fork_ev);
    };
    if (e != hipSuccess) {
        release_branches();
        (void)hipStreamDestroy(cs);
        *errmsg = std::string("stream: ") + hipGetErrorString(e);
        return STENCIL_EDEVICE;
    }
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        // boundary band into the scratch pairs first (each entry checks its own extent)
        const dim3 hgrid(hgx, std::min(hgy, kMaxGridYZ), n);
        hipError_t el = sizeof(T) == 8 ? batch_halo_launch_f64(reinterpret_cast<const HaloFill<double>*>(d_halo), hgrid, cs)
                                       : batch_halo_launch_f32(reinterpret_cast<const HaloFill<float>*>(d_halo), hgrid, cs);
        // the naive grids: group by group, one launch per time step; the
        // groups alternate between kNaiveBranches concurrent graph branches
        // (forked from and joined back into the capturing stream), so that
        // one group's launch gaps and tails overlap another group's work
        if (el == hipSuccess && !ngroups.empty()) el = hipEventRecord(fork_ev, cs);
        for (int b = 0; b < kNaiveBranches - 1 && el == hipSuccess && !ngroups.empty(); ++b)
            el = hipStreamWaitEvent(bstreams[b], fork_ev, 0);
        for (size_t gi = 0; gi < ngroups.size() && el == hipSuccess; ++gi) {
            const auto& ng = ngroups[gi];
            const int br = (int)(gi % kNaiveBranches);
            hipStream_t st = br == 0 ? cs : bstreams[br - 1];
            for (int t = 0; t < T_steps && ng.second > 0 && el == hipSuccess; ++t) {
                NaiveLaunch<T> NL{d_ntiles, d_nargs, ng.first, t};
                if constexpr (sizeof(T) == 8) el = batch_naive_launch_f64(NL, ng.second, st);
                else el = batch_naive_launch_f32(NL, ng.second, st);
            }
        }
        for (int b = 0; b < kNaiveBranches - 1 && el == hipSuccess && !ngroups.empty(); ++b) {
            el = hipEventRecord(join_ev[b], bstreams[b]);
            if (el == hipSuccess) el = hipStreamWaitEvent(cs, join_ev[b], 0);
        }
        for (size_t g = 0; g + 1 < group_first.size() && el == hipSuccess; ++g) {
            const int cnt = group_first[g + 1] - group_first[g];
            if (cnt <= 0) continue;
            BatchLaunch<T> L{d_tiles, group_first[g], d_args, d_var};
            if constexpr (sizeof(T) == 8) el = batch_launch_f64(L, cnt, cs);
            else el = batch_launch_f32(L, cnt, cs);
        }
        e = hipStreamEndCapture(cs, &bg.graph);
        if (e == hipSuccess && el != hipSuccess) e = el;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&bg.exec, bg.graph, nullptr, nullptr, 0);
    release_branches();
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        *errmsg = std::string("graph capture: ") + hipGetErrorString(e);
        return STENCIL_EDEVICE;
    }
    return STENCIL_OK;
}

int batch_run(int plan_kind, int plan_dtype, BatchState** state, stencil_grid* grids, const stencil_coeffs* coeffs,
              int n, int T, hipStream_t stream)
{
    if (!grids || !coeffs || n < 1 || n > 65535) {
        set_last_error("batched run needs 1 <= n <= 65535 grids and coefficients");
        return STENCIL_EINVAL;
    }
    if (T < 0) {
        set_last_error("T < 0");
        return STENCIL_EINVAL;
    }
    std::vector<HostWeights> hw(n);
    for (int i = 0; i < n; ++i) {
        int rc = check_grid(&grids[i], "grids[i]");
        if (rc) return rc;
        if (grids[i].dtype != plan_dtype) {
            set_last_error("grid dtype differs from the plan's");
            return STENCIL_EINVAL;
        }
        const int kind = coeffs[i].kind;
        if (kind < 0 || kind > 3 || (plan_kind != STENCIL_KIND_MIXED && kind != plan_kind)) {
            set_last_error("grid kind not allowed by the plan");
            return STENCIL_EINVAL;
        }
        if (grids[i].halo < radius_of(kind)) {
            set_last_error("halo narrower than the stencil radius");
            return STENCIL_EINVAL;
        }
        rc = check_coeffs(&coeffs[i], kind, &grids[i], &hw[i]);
        if (rc) return rc;
    }
    if (T == 0) return STENCIL_OK;
    BatchKey key;
    key.T = T;
    key.dtype = plan_dtype;
    for (int i = 0; i < n; ++i) {
        key.ptrs.push_back((uintptr_t)grids[i].buf[0]);
        key.ptrs.push_back((uintptr_t)grids[i].buf[1]);
        for (int m = 0; m < 13; ++m) key.ptrs.push_back((uintptr_t)coeffs[i].arr[m]);
        long long dims[] = {grids[i].nx, grids[i].ny, grids[i].nz, grids[i].halo, grids[i].sy, grids[i].sz,
                            grids[i].cur, coeffs[i].kind};
        key.dims.insert(key.dims.end(), dims, dims + 8);
        for (int m = 0; m < 13; ++m) {
            long long bits;
            std::memcpy(&bits, &coeffs[i].c[m], sizeof(bits));
            key.dims.push_back(bits);
        }
    }
    if (!*state) *state = new BatchState();
    BatchState* st = *state;
    BatchGraph* bg = nullptr;
    for (auto& c : st->cache)
        if (c.key == key) bg = &c;
    if (!bg) {
        if (st->cache.size() >= 2) {
            st->cache.front().release();
            st->cache.erase(st->cache.begin());
        }
        st->cache.emplace_back();
        bg = &st->cache.back();
        bg->key = key;
        std::string msg;
        int rc = plan_dtype == 0 ? build_graph<double>(*bg, grids, hw.data(), n, T, plan_dtype, &msg)
                                 : build_graph<float>(*bg, grids, hw.data(), n, T, plan_dtype, &msg);
        if (rc) {
            bg->release();
            st->cache.pop_back();
            set_last_error(msg);
            return rc;
        }
    }
    hipError_t e = hipGraphLaunch(bg->exec, stream);
    if (e != hipSuccess) {
        set_last_error(std::string("hipGraphLaunch: ") + hipGetErrorString(e));
        return STENCIL_EDEVICE;
    }
    for (int i = 0; i < n; ++i) grids[i].cur ^= (T & 1);
    return STENCIL_OK;
}

double batch_proxy_ms(int kind, int dtype, int nx, int ny, int nz, int T, int count, int var)
{
    const int h = radius_of(kind);
    const size_t es = es_of(dtype);
    const long long sy = nx + 2 * h, sz = sy * (ny + 2 * h);
    const size_t bytes = ((size_t)sz * (size_t)(nz + 2 * h) * es + 255) & ~size_t(255);
    const int narr = narr_of(kind);
    const size_t total = (size_t)count * (size_t)(2 + narr) * bytes;
    void* base = nullptr;
    if (hipMalloc(&base, total) != hipSuccess) {
        (void)hipGetLastError();
        return -1.0;
    }
    double ms = -1.0;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    BatchGraph bg;
    hipError_t e = hipMemset(base, 0, total);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) {
        const long long off = (long long)h * sz + (long long)h * sy + h;
        std::vector<stencil_grid> grids(count);
        std::vector<HostWeights> hw(count);
        for (int i = 0; i < count; ++i) {
            char* gb = static_cast<char*>(base) + (size_t)i * (size_t)(2 + narr) * bytes;
            stencil_grid& g = grids[i];
            std::memset(&g, 0, sizeof(g));
            g.nx = nx;
            g.ny = ny;
            g.nz = nz;
            g.halo = h;
            g.sy = sy;
            g.sz = sz;
            g.dtype = dtype;
            g.cur = 0;
            g.buf[0] = gb;
            g.buf[1] = gb + bytes;
            hw[i].kind = kind;
            for (int m = 0; m < 13; ++m) {
                hw[i].c[m] = 0.05;
                hw[i].org[m] = m < narr ? gb + (2 + m) * bytes + off * es : nullptr;
            }
        }
        std::vector<int> forced(count, var);
        std::string msg;
        const int rc = dtype == 0 ? build_graph<double>(bg, grids.data(), hw.data(), count, T, dtype, &msg, forced.data())
                                  : build_graph<float>(bg, grids.data(), hw.data(), count, T, dtype, &msg, forced.data());
        if (rc == STENCIL_OK) {
            e = hipGraphLaunch(bg.exec, st);  // warm-up
            if (e == hipSuccess) e = hipEventRecord(e0, st);
            for (int r = 0; r < 2 && e == hipSuccess; ++r) e = hipGraphLaunch(bg.exec, st);
            if (e == hipSuccess) e = hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float t = 0.f;
            if (e == hipSuccess && hipEventElapsedTime(&t, e0, e1) == hipSuccess) ms = t / 2.0;
        }
    }
    if (st) (void)hipStreamSynchronize(st);
    bg.release();
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
    (void)hipFree(base);
    (void)hipGetLastError();
    return ms;
}

void batch_free(BatchState* s)
{
    if (!s) return;
    for (auto& c : s->cache) c.release();
    delete s;
}

}  // namespace mwd
