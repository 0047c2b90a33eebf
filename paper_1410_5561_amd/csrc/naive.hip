// The naive sweep: one launch per time step over the whole grid.
#include <algorithm>

#include "internal.hpp"
#include "naive_block.hpp"

namespace mwd {

// One-dimensional grid over the blocks (bx fastest, then by, then bz).  Runs
// of `patch` consecutive blocks (whole block rows) go to one XCD, so that a
// block's x- and y-neighbours, whose halo rows and partial cache lines it
// reads, mostly run at the same time on the same L2.  A 1024-thread block is
// held to 64 registers per lane (two blocks per CU), except for the 25-point
// variable stencil, whose 13 coefficient rings need more.
template <int K, int BX, int BY>
constexpr int naive_min_waves() { return (BX * BY >= 1024 && K != K25V) ? 8 : 1; }

// Rows of (x, y) columns per thread: two for the FP32 radius-4 constant
// star (half the barriers and halo cells per update; its rings still fit 64
// registers with two planes of prefetch), one elsewhere (the FP64 rings
// would spill; the radius-1 sweeps gain nothing from it).
template <int K, typename T>
constexpr int naive_rows() { return (K == K25C && sizeof(T) == 4) ? 2 : 1; }

template <int K, typename T, int BX, int BY>
__global__ void __launch_bounds__(BX * BY, (naive_min_waves<K, BX, BY>()))
naive_sweep_kernel(const T* __restrict__ src, T* __restrict__ dst, Weights<T> w,
                   int nx, int ny, int nz, long long sy, long long sz, int zchunk, int nbx, int nby, int patch)
{
    constexpr int PF = naive_prefetch<K, T>(false);
    constexpr int RY = naive_rows<K, T>();
    using G = NaiveGeom<K, BX, BY, PF, false, RY>;
    __shared__ T tile[G::NB][G::TY][G::TX];
    const int t = xcd_tile(blockIdx.x, gridDim.x, patch);
    const int r = t / nbx;
    naive_block<K, T, BX, BY, PF, false, RY>(src, dst, w, nx, ny, nz, sy, sz, zchunk, t - r * nbx, r % nby, r / nby,
                                             tile);
}

// two 1024-thread (or four 512-thread) workgroups on each of 256 CUs
constexpr long long kNaiveMinBlocks = 512;

template <int K, typename T>
static hipError_t launch_naive(const DevGrid& g, const HostWeights& hw, const void* src, void* dst,
                               hipStream_t stream)
{
    constexpr int R = KindTraits<K>::R;
    constexpr int BX = 64;
    // radius 4: 16 rows (a block's threads also load its 2R(BX + BY) halo cells)
    constexpr int BY = (R == 1) ? 8 : 16;
    Weights<T> w;
    for (int m = 0; m < 13; ++m) {
        w.c[m] = static_cast<T>(hw.c[m]);
        w.arr[m] = static_cast<const T*>(hw.org[m]);
    }
    constexpr int HY = BY * naive_rows<K, T>();  // rows of a block
    const long long nbx = (g.nx + BX - 1) / BX, nby = (g.ny + HY - 1) / HY;
    // planes per block: 64 (128 at radius 4), halved down to 2 while the
    // launch has fewer than two workgroups per CU (small grids: more, shorter
    // z chunks; a block re-reads 2R planes per chunk, from cache at this size)
    int zchunk = (R == 1) ? 64 : 128;
    while (zchunk > 2 && nbx * nby * ((g.nz + zchunk - 1) / zchunk) < kNaiveMinBlocks) zchunk /= 2;
    const long long nbz = (g.nz + zchunk - 1) / zchunk;
    const long long nblocks = nbx * nby * nbz;
    if (nblocks > 0x7fffffffLL) return hipErrorInvalidValue;
    // about as many blocks per patch as one XCD (32 CUs) holds at once: two
    // 1024-thread blocks or four 512-thread blocks per CU
    const int resident = 32 * ((BX * BY) <= 512 ? 4 : 2);
    const int patch = (int)(nbx * std::max<long long>(1, std::min<long long>(nby, resident / nbx)));
    hipLaunchKernelGGL((naive_sweep_kernel<K, T, BX, BY>), dim3((unsigned)nblocks), dim3(BX * BY), 0, stream,
                       static_cast<const T*>(src), static_cast<T*>(dst), w,
                       g.nx, g.ny, g.nz, g.sy, g.sz, zchunk, (int)nbx, (int)nby, patch);
    return hipGetLastError();
}

hipError_t naive_sweep(const DevGrid& g, const HostWeights& w, const void* src, void* dst,
                       hipStream_t stream)
{
    const bool f64 = g.dtype == 0;
    switch (w.kind) {
        case K7C:  return f64 ? launch_naive<K7C, double>(g, w, src, dst, stream)
                              : launch_naive<K7C, float>(g, w, src, dst, stream);
        case K7V:  return f64 ? launch_naive<K7V, double>(g, w, src, dst, stream)
                              : launch_naive<K7V, float>(g, w, src, dst, stream);
        case K25C: return f64 ? launch_naive<K25C, double>(g, w, src, dst, stream)
                              : launch_naive<K25C, float>(g, w, src, dst, stream);
        case K25V: return f64 ? launch_naive<K25V, double>(g, w, src, dst, stream)
                              : launch_naive<K25V, float>(g, w, src, dst, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace mwd
