// One block of the naive sweep (one full stencil sweep per time step: the
// non-temporally-blocked baseline, the paper's "spatial blocking" column of
// Tables I-III).
//
// A workgroup owns a BX x BY block of (x, y) columns and marches along z over
// a chunk of planes.  A thread keeps its own column's 2R+1 planes in a
// register queue (z-neighbours) and publishes the current plane, plus one
// cell of the block's in-plane halo ring, to LDS (x- and y-neighbours).  x is
// the lane dimension, so every global access of a wave is one contiguous row
// segment.  Ideal traffic: every domain-sized stream read once and the result
// written once, s * N_D bytes per LUP.
//
// Memory-level parallelism: every load is issued P planes before the step
// that consumes it, into register rings whose slots are compile-time
// constants (the plane loop is unrolled by the rings' common period), so a
// thread keeps P planes of its column, its halo cell and its coefficients in
// flight.  The LDS plane is double-buffered in the single-grid sweep: one
// barrier per plane (a thread rewrites a buffer only after the next plane's
// barrier, which every thread reaches after it has finished reading that
// buffer).  The batched kernel keeps one buffer and a second barrier after
// the computation: on its many small grids (short z chunks, blocks of two
// stencil kinds sharing a CU) that ran faster (measured).
#pragma once

#include "common.hpp"

namespace mwd {

// Loads issued ahead of the plane that consumes them, beyond the next one:
// three planes in the single-grid sweep, fewer where a thread's rings would
// not fit the registers (the 13 coefficient arrays of the 25-point variable
// stencil); one in the register-capped batched kernel (measured fastest there).
// (In the standalone sweep every kind fits two 1024-thread blocks per CU,
// except the 25-point variable stencil: the radius-4 constant stencil
// therefore takes two planes, in FP64 for its wider registers and in FP32
// because its threads hold two rows.)
template <int K, typename T>
constexpr int naive_prefetch(bool capped)
{
    if constexpr (K == K25V) return (capped || sizeof(T) == 8) ? 0 : 1;
    if constexpr (K == K25C) return capped ? 1 : 2;
    return capped ? 1 : 3;
}

// ROT = false: the plane loop is unrolled by the rings' period, so that ring
// slots are compile-time constants (no register moves), and the LDS plane is
// double-buffered.  ROT = true (the batched kernel): the rings shift by one
// slot per plane (register moves), the loop is unrolled by two only (compact
// code: workgroups of several stencil kinds share a CU's instruction cache),
// and one LDS plane buffer with two barriers per plane.
//
// RY: rows per thread.  A thread owns the columns (x, y0 + ty + j BY),
// j < RY, so the block covers BX x (BY RY) columns: fewer barriers and fewer
// halo cells per update, at RY times the registers of the column rings.
template <int K, int BX, int BY, int PF, bool ROT = false, int RY = 1>
struct NaiveGeom {
    static constexpr int NB = ROT ? 1 : 2;               // LDS plane buffers
    static constexpr int R = KindTraits<K>::R;
    static constexpr int P = PF;
    static constexpr int Q = 2 * R + 1;
    static constexpr int NQ = Q + P;                     // own column: z-R .. z+R+P
    static constexpr int NH = P + 1;                     // halo cell, coefficients: z .. z+P
    static constexpr int U = ROT ? 2 : clcm(clcm(NQ, NH), 2);  // unroll (even: LDS buffer parity)
    static constexpr int HY = BY * RY;                   // rows of the block
    static constexpr int TY = HY + 2 * R, TX = BX + 2 * R;
    // cells of the in-plane halo ring (no corners: the operators are stars),
    // and how many of them each thread loads
    static constexpr int NCELL = 2 * R * (BX + HY);
    static constexpr int HC = (NCELL + BX * BY - 1) / (BX * BY);
};

template <int K, typename T, int BX, int BY, int PF, bool ROT = false, int RY = 1>
__device__ __forceinline__ void naive_block(const T* __restrict__ src, T* __restrict__ dst, const Weights<T>& w,
                                            int nx, int ny, int nz, long long sy, long long sz, int zchunk,
                                            int bx, int by, int bz,
                                            T (*tile)[NaiveGeom<K, BX, BY, PF, false, RY>::TY]
                                                     [NaiveGeom<K, BX, BY, PF, false, RY>::TX])
{
    using G = NaiveGeom<K, BX, BY, PF, ROT, RY>;
    constexpr int R = G::R, P = G::P, NQ = G::NQ, NH = G::NH, U = G::U, HY = G::HY;
    constexpr int NARR = KindTraits<K>::NARR;

    const int tid = threadIdx.x;
    const int tx = tid % BX, ty = tid / BX;
    const int x0 = bx * BX, y0 = by * HY;
    const int x = x0 + tx;
    const int z0 = bz * zchunk;
    const int z1 = min(nz, z0 + zchunk);

    // This thread's own columns: loaded if inside the padded array's useful part.
    bool own_ld[RY], own_up[RY];
    long long own_off[RY];
#pragma unroll
    for (int j = 0; j < RY; ++j) {
        const int y = y0 + ty + j * BY;
        own_ld[j] = (x < nx + R) && (y < ny + R);
        own_up[j] = (x < nx) && (y < ny);
        own_off[j] = (long long)y * sy + x;
    }

    // Cells tid, tid + BX BY, ... of the in-plane halo ring: first the x
    // sides (R columns left and right of each row), then the y sides (R rows
    // below and above the block).
    constexpr int HC = G::HC;
    int hr[HC], hc[HC];
    bool halo_ld[HC];
    long long halo_off[HC];
#pragma unroll
    for (int k = 0; k < HC; ++k) {
        const int cell = tid + k * BX * BY;
        int hx = 0, hy = 0;
        hr[k] = -1;
        hc[k] = -1;
        if (cell < 2 * R * HY) {
            const int side = cell / (R * HY), rem = cell % (R * HY);
            const int row = rem / R, c = rem % R;
            hr[k] = row + R;
            hc[k] = side == 0 ? c : BX + R + c;
            hx = side == 0 ? x0 - R + c : x0 + BX + c;
            hy = y0 + row;
        } else if (cell < G::NCELL) {
            const int t2 = cell - 2 * R * HY;
            const int side = t2 / (R * BX), rem = t2 % (R * BX);
            const int r = rem / BX, col = rem % BX;
            hr[k] = side == 0 ? r : HY + R + r;
            hc[k] = col + R;
            hx = x0 + col;
            hy = side == 0 ? y0 - R + r : y0 + HY + r;
        }
        halo_ld[k] = hr[k] >= 0 && hx < nx + R && hy < ny + R;
        halo_off[k] = (long long)hy * sy + hx;
    }

    // Planes a load may touch: the column's up to z1 - 1 + R (and inside the
    // array, z < nz + R); a halo cell's and a coefficient's up to z1 - 1.
    const int zlim_own = min(nz + R, z1 + R);
    const int zlim_cell = z1;

    // Rings: own plane p in slot (p - z0 + R) mod NQ; halo / coefficient
    // plane p in slot (p - z0) mod NH (ROT: at step z, own plane z + d in
    // slot R + d and halo / coefficient plane z + d in slot d).
    T q[RY][NQ], hq[HC][NH];
    T cw[NARR > 0 ? NARR : 1][RY][NH];
#pragma unroll
    for (int j = 0; j < RY; ++j)
#pragma unroll
        for (int i = 0; i < NQ; ++i) {
            const int p = z0 - R + i;
            q[j][i] = (own_ld[j] && p < zlim_own) ? src[(long long)p * sz + own_off[j]] : T(0);
        }
#pragma unroll
    for (int k = 0; k < HC; ++k)
#pragma unroll
        for (int i = 0; i < NH; ++i) {
            const int p = z0 + i;
            hq[k][i] = (halo_ld[k] && p < zlim_cell) ? src[(long long)p * sz + halo_off[k]] : T(0);
        }
#pragma unroll
    for (int m = 0; m < (NARR > 0 ? NARR : 1); ++m)
#pragma unroll
        for (int j = 0; j < RY; ++j)
#pragma unroll
            for (int i = 0; i < NH; ++i) {
                const int p = z0 + i;
                cw[m][j][i] = (NARR > 0 && own_up[j] && p < zlim_cell) ? w.arr[m][(long long)p * sz + own_off[j]]
                                                                       : T(0);
            }

    for (int zb = z0; zb < z1; zb += U) {
        static_for<0, U>([&](auto uc) MWD_INLINE {
            constexpr int u = decltype(uc)::value;
            constexpr int eb = ROT ? 0 : (u & 1);
            const int z = zb + u;
            // slots of own plane z + d and of halo / coefficient plane z + d
            constexpr int ua = ROT ? 0 : u;
            auto qs = [](int d) constexpr { return cmod(ua + R + d, NQ); };
            auto hs = [](int d) constexpr { return cmod(ua + d, NH); };
            if (z < z1) {  // uniform over the workgroup
#pragma unroll
                for (int j = 0; j < RY; ++j) tile[eb][ty + j * BY + R][tx + R] = q[j][qs(0)];
#pragma unroll
                for (int k = 0; k < HC; ++k)
                    if (hr[k] >= 0) tile[eb][hr[k]][hc[k]] = hq[k][hs(0)];
                __syncthreads();
#pragma unroll
                for (int j = 0; j < RY; ++j) {
                    if (own_up[j]) {
                        const int ly = ty + j * BY + R;
                        auto nb = [&](int dx, int dy, int dz) MWD_INLINE -> T {
                            if (dz != 0) return q[j][qs(dz)];
                            return tile[eb][ly + dy][tx + R + dx];
                        };
                        T v;
                        if constexpr (NARR > 0) {
                            v = apply_stencil<K, T>(nb, [&](int m) MWD_INLINE -> T { return cw[m][j][hs(0)]; });
                        } else {
                            v = apply_stencil<K, T>(nb, [&](int m) MWD_INLINE -> T { return w.c[m]; });
                        }
                        dst[(long long)z * sz + own_off[j]] = v;
                    }
                }
                // one buffer: every thread has read the plane before any rewrites it
                if constexpr (G::NB == 1) __syncthreads();
                if constexpr (ROT) {
                    // shift every ring by one plane; the freed last slots take the loads
#pragma unroll
                    for (int j = 0; j < RY; ++j)
#pragma unroll
                        for (int i = 0; i + 1 < NQ; ++i) q[j][i] = q[j][i + 1];
#pragma unroll
                    for (int k = 0; k < HC; ++k)
#pragma unroll
                        for (int i = 0; i + 1 < NH; ++i) hq[k][i] = hq[k][i + 1];
                    if constexpr (NARR > 0) {
#pragma unroll
                        for (int m = 0; m < NARR; ++m)
#pragma unroll
                            for (int j = 0; j < RY; ++j)
#pragma unroll
                                for (int i = 0; i + 1 < NH; ++i) cw[m][j][i] = cw[m][j][i + 1];
                    }
                }
                // refill, P planes ahead: own plane z + R + P + 1 (the slot of
                // plane z - R, just consumed; ROT: the last slot) and halo /
                // coefficient plane z + P + 1 (the slot of plane z; ROT: the last)
                constexpr int sq = ROT ? NQ - 1 : cmod(u, NQ);
                constexpr int sh = ROT ? NH - 1 : cmod(u, NH);
                const int pq = z + R + P + 1;
#pragma unroll
                for (int j = 0; j < RY; ++j)
                    if (own_ld[j] && pq < zlim_own) q[j][sq] = src[(long long)pq * sz + own_off[j]];
                const int ph = z + P + 1;
#pragma unroll
                for (int k = 0; k < HC; ++k)
                    if (halo_ld[k] && ph < zlim_cell) hq[k][sh] = src[(long long)ph * sz + halo_off[k]];
                if constexpr (NARR > 0) {
#pragma unroll
                    for (int j = 0; j < RY; ++j) {
                        if (own_up[j] && ph < zlim_cell) {
#pragma unroll
                            for (int m = 0; m < NARR; ++m)
                                cw[m][j][sh] = w.arr[m][(long long)ph * sz + own_off[j]];
                        }
                    }
                }
            }
        });
    }
}

}  // namespace mwd
