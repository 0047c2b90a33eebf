// Kernels of the batched form: many independent grids advanced together.
//
// The tiles of all grids are laid out in one table, grouped by diamond row:
// group rho holds the row-rho tiles (diamond x x-tile) of every grid that has
// such a row; a final group holds the gather of each grid's last two levels
// out of the rotating buffer pairs.  Group rho runs as one kernel launch in
// which every workgroup computes one tile; the launches of all groups are
// captured once into a hipGraph and replayed with a single hipGraphLaunch.
// Kernel boundaries carry the dependencies (row rho reads what rows rho-1 and
// rho-2 wrote, and reuses the pair rows rho-3 wrote, already consumed), so no
// workgroup ever waits on another one.
#pragma once

#include "mwd_tile.hpp"

namespace mwd {

struct BatchTile {
    int grid;     // index into the per-grid argument table
    int gather;   // 0: an MWD tile; 1: a gather tile
    int rho, t0, ybase;
    int b, j;     // diamond and x tile; for gather tiles: first plane and plane count
    int pad;
};

constexpr int kBatchThreads = 1024;

// Copy u_T and u_{T-1} of planes [z0, z0 + nzc) out of the rotating pairs into
// the caller's buffers.
template <typename T, int R, int DW>
__device__ void batch_gather(const MwdArgs<T>& a, int z0, int nzc)
{
    const long long plane = (long long)a.nx * a.ny;
    const long long total = plane * nzc;
    for (long long i = threadIdx.x; i < total; i += kBatchThreads) {
        const int z = z0 + (int)(i / plane);
        const long long r = i % plane;
        const int y = (int)(r / a.nx), x = (int)(r % a.nx);
        const long long off = (long long)z * a.sz + (long long)y * a.sy + x;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int t = a.nsteps - k;
            if (t < 1) continue;
            const int p = pair_of_row(row_of<R, DW>(y, t));
            if (p != 0) {
                const int bi = (a.cur + t) & 1;
                a.pair[0][bi][off] = a.pair[p][bi][off];
            }
        }
    }
}

// One compiled tile shape of the batched kernel.
template <int K, int DW, int WPR>
struct BatchVariant {
    static constexpr int kind = K, dw = DW, wpr = WPR;
};

template <typename T, class... V>
struct BatchKernelShapes {
    template <class Vv>
    static constexpr size_t lds_of() {
        using G = MwdGeom<Vv::kind, Vv::dw, Vv::wpr>;
        return sizeof(T) * 2 * G::L * G::NSX * G::LX;
    }
    static constexpr size_t lds_bytes() {
        size_t m = 16;
        ((m = lds_of<V>() > m ? lds_of<V>() : m), ...);
        return m;
    }
};

template <typename T, int I, class V, class... Rest>
__device__ __forceinline__ void batch_dispatch(int variant, const MwdArgs<T>& a, const MwdRow& row,
                                               const BatchTile& t, char* lds)
{
    if (variant == I) {
        using G = MwdGeom<V::kind, V::dw, V::wpr>;
        static_assert(G::NT <= kBatchThreads, "tile shape larger than the batch workgroup");
        if (t.gather) {
            batch_gather<T, G::R, V::dw>(a, t.b, t.j);
        } else {
            mwd_tile<V::kind, T, V::dw, V::wpr>(
                a, row, t.b, t.j, reinterpret_cast<T (*)[G::L][G::NSX][G::LX]>(lds));
        }
        return;
    }
    if constexpr (sizeof...(Rest) > 0) batch_dispatch<T, I + 1, Rest...>(variant, a, row, t, lds);
}

// Workgroup blockIdx.x computes tile first + blockIdx.x of the table.
template <typename T, class... V>
__device__ __forceinline__ void batch_group(const BatchTile* __restrict__ tiles, int first,
                                            const MwdArgs<T>* __restrict__ gargs,
                                            const int* __restrict__ gvariant, char* lds)
{
    const BatchTile t = tiles[first + blockIdx.x];
    const MwdRow row{t.rho, t.t0, t.ybase};
    batch_dispatch<T, 0, V...>(gvariant[t.grid], gargs[t.grid], row, t, lds);
}

}  // namespace mwd
