// MWD row kernel, final gather and the per-instantiation row scheduler.
// Included by the mwd_inst_*.hip files, one per (kind, dtype), so that the
// kernel instantiations compile in parallel.
#pragma once

#include <algorithm>

#include "internal.hpp"
#include "mwd_tile.hpp"

namespace mwd {

template <int K, typename T, int DW, int WPR>
__global__ void __launch_bounds__(64 * DW * WPR)
mwd_row_kernel(MwdArgs<T> a, MwdRow row)
{
    using G = MwdGeom<K, DW, WPR>;
    __shared__ T ex[2][G::L][G::NSX][G::LX];
    const int t = xcd_tile(blockIdx.x, gridDim.x, a.nxt);
    mwd_tile<K, T, DW, WPR>(a, row, t / a.nxt, t % a.nxt, ex);
}

// After the last row, copy u_T and u_{T-1} of every point out of the pair
// that holds them into the caller's buffers (pair 0).  A block takes 4 rows
// of 64 points over kGatherPlanes consecutive planes: the pair of each level
// depends on the row only, and each thread has several planes' copies in
// flight (short blocks of one plane each were dispatch-bound).
constexpr int kGatherPlanes = 16;

template <typename T, int R, int DW>
__global__ void __launch_bounds__(256)
mwd_gather_kernel(MwdArgs<T> a)
{
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    if (x >= a.nx) return;
    // y and z stride over the launch's blocks (gridDim.y, gridDim.z <= 65535)
    for (int y = blockIdx.y * 4 + (threadIdx.x >> 6); y < a.ny; y += gridDim.y * 4) {
        int src[2];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int t = a.nsteps - k;
            src[k] = t < 1 ? 0 : pair_of_row(row_of<R, DW>(y, t));
        }
        if (src[0] == 0 && src[1] == 0) continue;
        for (int z0 = blockIdx.z * kGatherPlanes; z0 < a.nz; z0 += gridDim.z * kGatherPlanes) {
            const int z1 = min(a.nz, z0 + kGatherPlanes);
#pragma unroll 4
            for (int z = z0; z < z1; ++z) {
                const long long off = (long long)z * a.sz + (long long)y * a.sy + x;
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    if (src[k] != 0) {
                        const int bi = (a.cur + a.nsteps - k) & 1;
                        a.pair[0][bi][off] = a.pair[src[k]][bi][off];
                    }
                }
            }
        }
    }
}

template <int K, typename T, int DW, int WPR>
static hipError_t run_rows(const DevGrid& g, const HostWeights& hw, int nsteps, void* const scratch[4],
                           hipStream_t stream, Prof* prof, int rho_lo, int rho_hi)
{
    using G = MwdGeom<K, DW, WPR>;
    MwdArgs<T> a{};
    T* o0 = static_cast<T*>(g.org[0]);
    T* o1 = static_cast<T*>(g.org[1]);
    a.pair[0][0] = o0;
    a.pair[0][1] = o1;
    a.pair[1][0] = static_cast<T*>(scratch[0]);
    a.pair[1][1] = static_cast<T*>(scratch[1]);
    a.pair[2][0] = static_cast<T*>(scratch[2]);
    a.pair[2][1] = static_cast<T*>(scratch[3]);
    a.halo = static_cast<const T*>(g.org[g.cur]);
    for (int m = 0; m < 13; ++m) {
        a.w.c[m] = static_cast<T>(hw.c[m]);
        a.w.arr[m] = static_cast<const T*>(hw.org[m]);
    }
    a.nx = g.nx;
    a.ny = g.ny;
    a.nz = g.nz;
    a.sy = g.sy;
    a.sz = g.sz;
    a.cur = g.cur;
    a.nsteps = nsteps;
    a.nxt = (g.nx + G::XT - 1) / G::XT;
    const int rho_max = (nsteps + G::H - 1) / G::H;
    // rows [rho_lo, rho_hi] of the schedule; a partial range (the tuner's
    // timing) skips the boundary fill and the gather
    const bool whole = rho_lo <= 0 && rho_hi >= rho_max;
    rho_lo = rho_lo < 0 ? 0 : rho_lo;
    rho_hi = rho_hi > rho_max ? rho_max : rho_hi;
    // boundary values into the scratch pairs
    if (whole) {
        HaloFill<T> hf;
        hf.src = a.halo;
        for (int k = 0; k < 4; ++k) hf.dst[k] = static_cast<T*>(scratch[k]);
        hf.nx = g.nx;
        hf.ny = g.ny;
        hf.nz = g.nz;
        hf.r = G::R;
        hf.sy = g.sy;
        hf.sz = g.sz;
        dim3 hg((g.nx + 2 * G::R + 63) / 64, std::min((g.ny + 2 * G::R + 3) / 4, kMaxGridYZ),
                std::min((g.nz + 2 * G::R + kFillPlanes - 1) / kFillPlanes, kMaxGridYZ));
        if (prof) prof->begin(stream);
        hipLaunchKernelGGL((mwd_halo_fill_kernel<T>), hg, dim3(256), 0, stream, hf);
        if (prof) prof->end(stream, 1);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    for (int rho = rho_lo; rho <= rho_hi; ++rho) {
        MwdRow row;
        row.rho = rho;
        row.t0 = (rho - 1) * G::H;
        const int yoff = (rho % 2) * (DW / 2);
        row.ybase = yoff > 0 ? yoff - DW : 0;
        const int nB = (g.ny - 1 - row.ybase) / DW + 1;
        if (prof) prof->begin(stream);
        hipLaunchKernelGGL((mwd_row_kernel<K, T, DW, WPR>), dim3(nB * a.nxt), dim3(G::NT), 0, stream, a, row);
        if (prof) prof->end(stream, 0);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (!whole) return hipSuccess;
    dim3 gg((g.nx + 63) / 64, std::min((g.ny + 3) / 4, kMaxGridYZ),
            std::min((g.nz + kGatherPlanes - 1) / kGatherPlanes, kMaxGridYZ));
    if (prof) prof->begin(stream);
    hipLaunchKernelGGL((mwd_gather_kernel<T, G::R, DW>), gg, dim3(256), 0, stream, a);
    if (prof) prof->end(stream, 1);
    return hipGetLastError();
}

using RunFn = hipError_t (*)(const DevGrid&, const HostWeights&, int, void* const*, hipStream_t, Prof*, int, int);

struct MwdEntry {
    int kind, dtype, dw, wpr;
    RunFn fn;
    int levels, xtile;
    const void* kernel;  // the row kernel, for resource queries
};

#define MWD_ENTRY(K, TT, DTI, DW, WPR)                                               \
    MwdEntry{K, DTI, DW, WPR, &run_rows<K, TT, DW, WPR>, MwdGeom<K, DW, WPR>::L,     \
             MwdGeom<K, DW, WPR>::XT,                                                \
             reinterpret_cast<const void*>(&mwd_row_kernel<K, TT, DW, WPR>)}


}  // namespace mwd
