// Persistent kernel of the batched form: many independent grids advanced in
// one launch.  The tiles of every grid (MWD diamond x x-tile tiles, one row
// after another, then the gather of the grid's last two levels) form one
// table in a topological order; each workgroup repeatedly takes the next
// ticket from a device counter, waits until the tiles its tile depends on are
// complete, runs it, and publishes its completion.
//
// Dependencies are per grid and per row: a tile of row rho starts once every
// tile of rows < rho of the same grid has completed (the `need` count of the
// grid's completion counter).  That covers the reads (rows rho-1, rho-2) and
// the reuse of buffer pair (rho+1) mod 3, last read by rows rho-1 and rho-2.
// Because every tile only waits on tiles with smaller tickets, and a ticket is
// only taken by a running workgroup, the smallest unfinished ticket can
// always proceed: the schedule cannot deadlock.  Completion is published with
// an agent-scope release after the tile's stores and observed with an
// agent-scope acquire before the dependent tile's loads (the workgroups may
// sit on different XCDs, whose L2 caches are not coherent with each other).
// A wait that exceeds a wall-clock limit sets an error flag and gives up, so
// the kernel always drains.
#pragma once

#include "mwd_tile.hpp"

namespace mwd {

struct BatchTile {
    int grid;     // index into the per-grid argument table
    int variant;  // tile shape (index into the batch variant list), or kGatherVariant
    int rho, t0, ybase;
    int b, j;     // diamond and x tile; for gather tiles: first plane and plane count
    int need;     // completed tiles of this grid required before starting
};

constexpr int kGatherVariant = 255;
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
        return sizeof(T) * 2 * G::L * G::NS * G::LX;
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
        if (t.variant == kGatherVariant) {
            batch_gather<T, G::R, V::dw>(a, t.b, t.j);
        } else {
            mwd_tile<V::kind, T, V::dw, V::wpr>(
                a, row, t.b, t.j, reinterpret_cast<T (*)[G::L][G::NS][G::LX]>(lds));
        }
        return;
    }
    if constexpr (sizeof...(Rest) > 0) batch_dispatch<T, I + 1, Rest...>(variant, a, row, t, lds);
}

template <typename T, class... V>
__device__ __forceinline__ void batch_loop(const BatchTile* __restrict__ tiles, int ntiles,
                                           const MwdArgs<T>* __restrict__ gargs,
                                           const int* __restrict__ gvariant,
                                           int* done, int* counter, int* err, long long spin_limit,
                                           char* lds)
{
    __shared__ int s_ticket;
    for (;;) {
        if (threadIdx.x == 0) s_ticket = atomicAdd(counter, 1);
        __syncthreads();
        const int tk = s_ticket;
        __syncthreads();
        if (tk >= ntiles) break;
        const BatchTile t = tiles[tk];
        if (threadIdx.x == 0) {
            if (t.need > 0) {
                const long long start = wall_clock64();
                while (__hip_atomic_load(&done[t.grid], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < t.need) {
                    __builtin_amdgcn_s_sleep(4);
                    if (wall_clock64() - start > spin_limit) {
                        __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        break;
                    }
                }
            }
            // acquire: later loads of this workgroup see the producers' stores
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        __syncthreads();
        const MwdRow row{t.rho, t.t0, t.ybase};
        batch_dispatch<T, 0, V...>(gvariant[t.grid], gargs[t.grid], row, t, lds);
        __syncthreads();
        if (threadIdx.x == 0) {
            // release: this tile's stores are visible before the count moves
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __hip_atomic_fetch_add(&done[t.grid], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

}  // namespace mwd
