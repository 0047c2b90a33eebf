// Multicore wavefront diamond (MWD) temporal blocking on gfx950: the tile
// kernel body and the tiling geometry (Sec. II-A, Sec. III-A).
//
// Tiling.  With h = Dw / (2R), every space-time point (y, t) belongs to the
// diamond tile (A, B) = (floor((y + R t) / Dw), floor((y - R t) / Dw)); all
// dependencies of a lattice-site update point to tiles with A' <= A and
// B' >= B, so the tiles of one row rho = A - B are independent and rows run
// in order (Fig. 1).  Row rho's tiles sit at yL = B Dw + rho Dw / 2 and cover
// the time levels t0 + tau, t0 = (rho - 1) h, tau = 1 .. L = 2h - 1; at level
// tau the tile holds the 2 R min(tau, 2h - tau) rows centred in [yL, yL + Dw).
// The diamond is extruded over x and z (Fig. 2): a workgroup owns one diamond
// and one x tile, and sweeps a wavefront along z in which level tau lags level
// tau - 1 by R planes.
//
// GPU mapping.  One wave (or WPR waves) per diamond row y; lanes are x, so every
// HBM access of a wave is a contiguous row segment.  A lane keeps, for each
// time level, the 2R+1 most recent z-planes of its own (x, y) column in
// registers (the z-neighbours), and publishes one plane per level per step to
// an LDS exchange array that gives the x- and y-neighbours.  One workgroup
// barrier per wavefront step; the exchange array is double-buffered.
//
// x tiles (Sec. III-A) run concurrently: each tile recomputes an R-wide ring
// per remaining level around its x range (level tau spans x0 - (L - tau) R ..
// x0 + XT + (L - tau) R) and writes only [x0, x0 + XT).  Because a tile then
// reads, in its overlap, points that a neighbouring tile is rewriting, every
// row writes its levels into its own buffer pair, rotating over three pairs
// (row rho uses pair (rho + 1) mod 3; the input is pair 0); a row reads only
// what rows rho - 1 and rho - 2 wrote, so no row reads a pair it writes.
// Only the last two time levels of each point leave the chip (the two-array
// scheme's ping-pong, Sec. III-C): these are exactly what later rows read.
#pragma once

#include "common.hpp"

namespace mwd {

template <int K, int DW, int WPR>
struct MwdGeom {
    static constexpr int R = KindTraits<K>::R;
    static constexpr int NARR = KindTraits<K>::NARR;
    static_assert(DW % (2 * R) == 0, "diamond width must be a multiple of 2R");
    static constexpr int H = DW / (2 * R);          // half height in time levels
    static constexpr int L = 2 * H - 1;             // computed levels per tile
    static constexpr int LX = 64 * WPR;             // x lanes per diamond row
    static constexpr int XT = LX - 2 * L * R;       // x points written per tile
    static_assert(XT > 0, "x tile smaller than the recomputed ring");
    static constexpr int NWAVES = DW * WPR;
    static constexpr int NT = 64 * NWAVES;
    static_assert(NT <= 1024, "workgroup too large");
    static constexpr int Q = 2 * R + 1;             // z-queue length per level
    // coefficient ring: planes [s - LR, s - R] are in use at step s, and the
    // load for plane s + 1 - R is issued during step s
    static constexpr int WIN = NARR ? Q * (((L - 1) * R + 2 + Q - 1) / Q) : 1;
    static constexpr int U = clcm(Q, WIN);          // unroll: ring slots become constants
    static constexpr int NS = DW + 2 * R;           // LDS row slots (diamond rows + side rows)
    static constexpr int NSX = NS + 1;              // plus a spare row for writes nobody reads
    static constexpr int S0 = U * ((R + 1 + U - 1) / U);  // step offset, multiple of U, > R
};

// Which buffer pair holds the levels written by row rho.
__host__ __device__ __forceinline__ int pair_of_row(int rho) { return (rho + 1) % 3; }

// Row of the tile containing space-time point (y, t), t >= 1.
template <int R, int DW>
__host__ __device__ __forceinline__ int row_of(int y, int t) {
    return floordiv(y + R * t, DW) - floordiv(y - R * t, DW);
}

template <typename T>
struct MwdArgs {
    T* pair[3][2];        // interior-origin pointers; pair 0 = the caller's two buffers
    const T* halo;        // one of the caller's buffers: source of boundary values
    Weights<T> w;
    int nx, ny, nz;
    long long sy, sz;
    int cur;              // level t lives in buffer (cur + t) & 1 of its pair
    int nsteps;           // total number of time steps of the run
    int nxt;              // x tiles per diamond
};

// One diamond row of the schedule.
struct MwdRow {
    int rho, t0;          // row index and the level just below the row's tiles
    int ybase;            // yL of the row's first diamond
};

// Copy the boundary band (width R around the interior) of one array into the
// four scratch arrays, so that every array a tile loads from holds the fixed
// boundary values.  Entry blockIdx.z of the table.
template <typename T>
struct HaloFill {
    const T* src;
    T* dst[4];
    int nx, ny, nz, r;
    long long sy, sz;
};

template <typename T>
__device__ __forceinline__ void halo_fill_one(const HaloFill<T>& e)
{
    const int x = blockIdx.x * 64 + (threadIdx.x & 63) - e.r;
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6) - e.r;
    if (x >= e.nx + e.r || y >= e.ny + e.r) return;
    const bool col_inside = x >= 0 && x < e.nx && y >= 0 && y < e.ny;
    for (int z = -e.r; z < e.nz + e.r; ++z) {
        if (col_inside && z == 0) z = e.nz;  // skip the interior of an interior column
        const long long off = (long long)z * e.sz + (long long)y * e.sy + x;
        const T v = e.src[off];
#pragma unroll
        for (int k = 0; k < 4; ++k) e.dst[k][off] = v;
    }
}

template <typename T>
__global__ void __launch_bounds__(256) mwd_halo_fill_kernel(HaloFill<T> e)
{
    halo_fill_one(e);
}

// Batched: entry blockIdx.z of a device table.
template <typename T>
__global__ void __launch_bounds__(256) mwd_halo_fill_table_kernel(const HaloFill<T>* __restrict__ table)
{
    halo_fill_one(table[blockIdx.z]);
}

// The tile (diamond b of the row, x tile j) computed by one workgroup.
template <int K, typename T, int DW, int WPR>
__device__ __forceinline__ void mwd_tile(const MwdArgs<T>& a, const MwdRow& row, int b, int j,
                                         T (*ex)[MwdGeom<K, DW, WPR>::L][MwdGeom<K, DW, WPR>::NSX]
                                              [MwdGeom<K, DW, WPR>::LX])
{
    using G = MwdGeom<K, DW, WPR>;
    constexpr int R = G::R, H = G::H, L = G::L, Q = G::Q, LX = G::LX, XT = G::XT;
    constexpr int NARR = G::NARR, WIN = G::WIN, U = G::U;

    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    // Waves beyond this tile shape's count (when the workgroup is sized for a
    // larger shape, as in the batched kernel) only take part in the barriers.
    const bool wave_active = wave < G::NWAVES;
    const int yr = wave / WPR;
    const int xl = (wave % WPR) * 64 + lane;
    const int yL = row.ybase + b * DW;
    const int x0 = j * XT;
    const int x = x0 - L * R + xl;
    const int y = yL + yr;
    const bool yin = y >= 0 && y < a.ny;
    const bool xin = x >= 0 && x < a.nx;
    const bool xact = x >= -R && x < a.nx + R;
    const bool xout = xl >= L * R && xl < L * R + XT && x < a.nx;

    // Is level tau of diamond row yrr computed by this tile (clipped to the
    // domain and to 1 <= t <= T)?  Wave-uniform.
    auto computed = [&](int yrr, int tau) -> bool {
        if (tau < 1 || tau > L || yrr < 0 || yrr >= DW) return false;
        const int t = row.t0 + tau;
        if (t < 1 || t > a.nsteps) return false;
        const int yy = yL + yrr;
        if (yy < 0 || yy >= a.ny) return false;
        const int d = yrr < DW / 2 ? DW / 2 - 1 - yrr : yrr - DW / 2;
        return d < R * min(tau, 2 * H - tau);
    };
    auto needed = [&](int yrr, int tau) -> bool {
        if (tau >= L) return false;
        bool n = false;
        for (int dy = -R; dy <= R; ++dy) n = n || computed(yrr + dy, tau + 1);
        return n;
    };
    // Source of a level-t value at row yy that this tile does not compute.
    auto level_src = [&](int yy, int t) -> const T* {
        if (t < 0 || yy < 0 || yy >= a.ny) return a.halo;
        const int p = (t == 0) ? 0 : pair_of_row(row_of<R, DW>(yy, t));
        return a.pair[p][(a.cur + t) & 1];
    };

    uint32_t cmask = 0, pmask = 0, smask = 0;
    int thi = -1;
    for (int tau = 0; tau <= L; ++tau) {
        const bool c = computed(yr, tau);
        if (c) { cmask |= 1u << tau; thi = tau; }
        if (c || needed(yr, tau)) pmask |= 1u << tau;
    }
    for (int tau = 0; tau <= L; ++tau)
        if (((cmask >> tau) & 1u) && tau >= thi - 1) smask |= 1u << tau;
    if (!wave_active) cmask = pmask = smask = 0u;
    cmask = __builtin_amdgcn_readfirstlane(cmask);
    pmask = __builtin_amdgcn_readfirstlane(pmask);
    smask = __builtin_amdgcn_readfirstlane(smask);

    const T* src[L + 1];
    T* dst[L + 1];
    T* const* outp = a.pair[pair_of_row(row.rho)];
#pragma unroll
    for (int tau = 0; tau <= L; ++tau) {
        src[tau] = level_src(y, row.t0 + tau);
        dst[tau] = outp[(a.cur + row.t0 + tau) & 1];
    }

    // Side rows: R rows beyond each edge of the diamond, needed only at level
    // h - 1 by the widest level h; loaded by the edge waves straight into LDS.
    const bool left_edge = wave_active && yr == 0, right_edge = wave_active && yr == DW - 1;
    const bool side_wave = left_edge || right_edge;
    bool sv_present[R];
    const T* sv_src[R];
    int sv_y[R];
    int side_slot[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int yrs = left_edge ? (-R + k) : (DW + k);
        sv_y[k] = yL + yrs;
        sv_present[k] = side_wave && needed(yrs, H - 1);
        sv_src[k] = level_src(sv_y[k], row.t0 + H - 1);
        side_slot[k] = sv_present[k] ? (left_edge ? k : DW + R + k) : G::NS;  // NS: the spare row
    }

    T q[L + 1][Q];
    T lv[L + 1];
    T sv[R];
    T cr[NARR > 0 ? NARR : 1][WIN];
#pragma unroll
    for (int tau = 0; tau <= L; ++tau) {
        lv[tau] = T(0);
#pragma unroll
        for (int k = 0; k < Q; ++k) q[tau][k] = T(0);
    }
#pragma unroll
    for (int k = 0; k < R; ++k) sv[k] = T(0);
#pragma unroll
    for (int m = 0; m < (NARR > 0 ? NARR : 1); ++m)
#pragma unroll
        for (int k = 0; k < WIN; ++k) cr[m][k] = T(0);

    const long long col = (long long)y * a.sy + x;
    const int s_first = -G::S0;
    // one step past the last plane of the last level, for its delayed stores
    const int s_last = a.nz + R + L * R;
    // Every step issues the same global loads in the same order: a lane with
    // nothing to load reads the interior origin of the same array instead.
    // The scratch pairs carry a copy of the boundary values (filled before the
    // first row), so a level's source array also serves its boundary lanes.

    for (int sb = s_first; sb <= s_last; sb += U) {
        static_for<0, U>([&](auto uc) {
            constexpr int u = decltype(uc)::value;
            const int s = sb + u;
            const int eb = s & 1;
            // (1) publish, for every level tau < L, the plane level tau + 1
            //     reads in-plane neighbours from at this step, and the side rows
            static_for<0, L>([&](auto tc) {
                constexpr int tau = decltype(tc)::value;
                const int p = s - (tau + 1) * R;
                if (((pmask >> tau) & 1u) && p >= 0 && p < a.nz)
                    ex[eb][tau][yr + R][xl] = q[tau][cmod(u - (tau + 1) * R, Q)];
            });
            // side rows: unconditional, so the wait for their loads is the
            // same on every path; other waves write a spare row nobody reads
#pragma unroll
            for (int k = 0; k < R; ++k)
                ex[eb][H - 1][side_slot[k]][xl] = sv[k];
            __syncthreads();
            // (2) take the values loaded during the previous step into the
            //     queues (lanes that compute below overwrite theirs)
            static_for<0, L + 1>([&](auto tc) {
                constexpr int tau = decltype(tc)::value;
                q[tau][cmod(u - tau * R, Q)] = lv[tau];
            });
            // (3) stores of the previous step (its values are still in the
            //     queues): the last two levels of each point.  Issued before
            //     this step's loads, so waits on those loads stay exact.
            static_for<1, L + 1>([&](auto tc) {
                constexpr int tau = decltype(tc)::value;
                const int p = s - 1 - tau * R;
                if (((smask >> tau) & 1u) && p >= 0 && p < a.nz && xout)
                    dst[tau][(long long)p * a.sz + col] = q[tau][cmod(u - 1 - tau * R, Q)];
            });
            // (4) issue every global load of the next step now, unconditionally
            //     (a lane with nothing to load reads its array's origin): level values a
            //     tile does not compute, coefficients, side rows
            static_for<0, L + 1>([&](auto tc) {
                constexpr int tau = decltype(tc)::value;
                const int pn = s - tau * R + 1;
                const bool prange = ((pmask >> tau) & 1u) && pn >= -R && pn < a.nz + R;
                const bool pin = pn >= 0 && pn < a.nz;
                const bool ctype = tau >= 1 && ((cmask >> tau) & 1u);
                const bool lact = xact & (xl >= tau * R) & (xl < LX - tau * R);
                const bool need = prange & lact & !(ctype & xin & pin);
                lv[tau] = src[tau][need ? (long long)pn * a.sz + col : 0LL];
            });
            if constexpr (NARR > 0) {
                const int pc = s + 1 - R;
                const bool need = (cmask != 0u) & (pc >= 0) & (pc < a.nz) & xin & (xl >= R) & (xl < LX - R);
                const long long off = need ? (long long)pc * a.sz + col : 0LL;
#pragma unroll
                for (int m = 0; m < NARR; ++m) cr[m][cmod(u + 1 - R, WIN)] = a.w.arr[m][off];
            }
            {
                const int ps = s + 1 - H * R;
                const bool lane_ok = side_wave & (ps >= 0) & (ps < a.nz) & xact & (xl >= (H - 1) * R) &
                                     (xl < LX - (H - 1) * R);
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    const bool need = lane_ok & sv_present[k];
                    sv[k] = sv_src[k][need ? (long long)ps * a.sz + (long long)sv_y[k] * a.sy + x : 0LL];
                }
            }
            // (5) advance every computed level by one plane, lowest level
            //     first: level tau reads level tau - 1's plane p + R just made
            static_for<1, L + 1>([&](auto tc) {
                constexpr int tau = decltype(tc)::value;
                const int p = s - tau * R;
                if (((cmask >> tau) & 1u) && p >= 0 && p < a.nz) {
                    if (xin && xl >= tau * R && xl < LX - tau * R) {
                        auto nb = [&](int dx, int dy, int dz) -> T {
                            if (dz != 0) return q[tau - 1][cmod(u - tau * R + dz, Q)];
                            if (dy != 0) return ex[eb][tau - 1][yr + R + dy][xl];
                            if (dx != 0) return ex[eb][tau - 1][yr + R][xl + dx];
                            return q[tau - 1][cmod(u - tau * R, Q)];
                        };
                        if constexpr (NARR > 0) {
                            q[tau][cmod(u - tau * R, Q)] = apply_stencil<K, T>(nb, [&](int m) -> T {
                                return cr[m][cmod(u - tau * R, WIN)];
                            });
                        } else {
                            q[tau][cmod(u - tau * R, Q)] =
                                apply_stencil<K, T>(nb, [&](int m) -> T { return a.w.c[m]; });
                        }
                    }
                }
            });
        });
    }
}

}  // namespace mwd
