// MWD row kernel, final gather and the per-instantiation row scheduler.
// Included by the mwd_inst_*.hip files, one per (kind, dtype), so that the
// kernel instantiations compile in parallel.
#pragma once

#include <algorithm>

#include "internal.hpp"
#include "mwd_tile.hpp"

namespace mwd {

// One launch: diamonds [d0[0], d0[0] + n[0]) of row r[0], then diamonds
// [d0[1], d0[1] + n[1]) of row r[1] (n[1] may be 0), every x tile of each.
struct MwdBand {
    MwdRow r[2];
    int d0[2], n[2];
};

template <int K, typename T, int DW, int WPR>
__global__ void __launch_bounds__(64 * DW * WPR)
mwd_row_kernel(MwdArgs<T> a, MwdBand band)
{
    using G = MwdGeom<K, DW, WPR>;
    __shared__ T ex[2][G::L][G::NSX][G::LX];
    int t = xcd_tile(blockIdx.x, gridDim.x, a.nxt);
    const int n0 = band.n[0] * a.nxt;
    const int s = t < n0 ? 0 : 1;
    t -= s * n0;
    mwd_tile<K, T, DW, WPR>(a, band.r[s], band.d0[s] + t / a.nxt, t % a.nxt, ex);
}

// After the last row, copy u_T and u_{T-1} of every point out of the pair
// that holds them into the caller's buffers (pair 0).
template <typename T, int R, int DW>
__global__ void __launch_bounds__(256)
mwd_gather_kernel(MwdArgs<T> a)
{
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int z = blockIdx.z;
    if (x >= a.nx || y >= a.ny) return;
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
        dim3 hg((g.nx + 2 * G::R + 63) / 64, (g.ny + 2 * G::R + 3) / 4, 1);
        if (prof) prof->begin(stream);
        hipLaunchKernelGGL((mwd_halo_fill_kernel<T>), hg, dim3(256), 0, stream, hf);
        if (prof) prof->end(stream, 1);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    auto row_of_rho = [&](int rho) {
        MwdRow row;
        row.rho = rho;
        row.t0 = (rho - 1) * G::H;
        const int yoff = (rho % 2) * (DW / 2);
        row.ybase = yoff > 0 ? yoff - DW : 0;
        return row;
    };
    auto diamonds = [&](const MwdRow& row) { return (g.ny - 1 - row.ybase) / DW + 1; };
    // Workgroups the GPU holds at once.  A row whose tiles need more than
    // that runs in launches of whole rounds (m rounds: at most m * slots
    // tiles each), and the launch that ends a row also starts the next row
    // with the diamonds that need nothing from this launch: next-row diamond
    // e reads rows [yL' - R, yL' + Dw + R) and writes [yL', yL' + Dw), this
    // launch's part of the row, from diamond D on, reads from yL(D) - R and
    // writes from yL(D), and the next row writes the pair this row reads, so
    // yL'(e) + Dw + R <= yL(D) keeps the two parts apart.  That removes most
    // of the partly filled last round of every row.
    int slots = 0;
    {
        int dev = 0, ncu = 0, per = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &per, reinterpret_cast<const void*>(&mwd_row_kernel<K, T, DW, WPR>), G::NT, 0) == hipSuccess)
            slots = ncu * per;
        (void)hipGetLastError();
    }
    int rho = rho_lo, d = 0;
    while (rho <= rho_hi) {
        const MwdRow row = row_of_rho(rho);
        const int nb = diamonds(row);
        int cap = nb;
        if (slots > 0 && (long long)nb * a.nxt > slots) {
            const long long m = (long long)nb * a.nxt / slots;
            cap = (int)std::max(1LL, m * slots / a.nxt);
        }
        MwdBand band;
        band.r[0] = row;
        band.d0[0] = d;
        band.n[0] = std::min(cap, nb - d);
        band.r[1] = row;
        band.d0[1] = 0;
        band.n[1] = 0;
        const int D = d;
        d += band.n[0];
        if (d >= nb) {
            if (rho + 1 <= rho_hi && D > 0) {
                const MwdRow next = row_of_rho(rho + 1);
                // next-row diamonds e = 0 .. E-1 with yL'(e) + Dw + R <= yL(D)
                const int E = floordiv(row.ybase + D * DW - DW - G::R - next.ybase, DW) + 1;
                band.r[1] = next;
                band.n[1] = std::max(0, std::min({cap - band.n[0], E, diamonds(next)}));
            }
            ++rho;
            d = band.n[1];
        }
        const int ntiles = (band.n[0] + band.n[1]) * a.nxt;
        if (prof) prof->begin(stream);
        hipLaunchKernelGGL((mwd_row_kernel<K, T, DW, WPR>), dim3(ntiles), dim3(G::NT), 0, stream, a, band);
        if (prof) prof->end(stream, 0);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (!whole) return hipSuccess;
    dim3 gg((g.nx + 63) / 64, (g.ny + 3) / 4, g.nz);
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
