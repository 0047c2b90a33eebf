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
#pragma once

#include "common.hpp"

namespace mwd {

template <int K, typename T, int BX, int BY>
__device__ __forceinline__ void naive_block(const T* __restrict__ src, T* __restrict__ dst, const Weights<T>& w,
                                            int nx, int ny, int nz, long long sy, long long sz, int zchunk,
                                            int bx, int by, int bz, T (*tile)[BX + 2 * KindTraits<K>::R])
{
    constexpr int R = KindTraits<K>::R;
    constexpr int Q = 2 * R + 1;
    constexpr int NARR = KindTraits<K>::NARR;

    const int tid = threadIdx.x;
    const int tx = tid % BX, ty = tid / BX;
    const int x0 = bx * BX, y0 = by * BY;
    const int x = x0 + tx, y = y0 + ty;
    const int z0 = bz * zchunk;
    const int z1 = min(nz, z0 + zchunk);

    // This thread's own column: loaded if inside the padded array's useful part.
    const bool own_ld = (x < nx + R) && (y < ny + R);
    const bool own_up = (x < nx) && (y < ny);
    const long long own_off = (long long)y * sy + x;

    // One cell of the in-plane halo ring (no corners: the operators are stars).
    int hx = 0, hy = 0, hr = -1, hc = -1;
    if (tid < 2 * R * BY) {
        const int side = tid / (R * BY), rem = tid % (R * BY);
        const int row = rem / R, c = rem % R;
        hr = row + R;
        hc = side == 0 ? c : BX + R + c;
        hx = side == 0 ? x0 - R + c : x0 + BX + c;
        hy = y0 + row;
    } else if (tid < 2 * R * (BY + BX)) {
        const int t2 = tid - 2 * R * BY;
        const int side = t2 / (R * BX), rem = t2 % (R * BX);
        const int r = rem / BX, col = rem % BX;
        hr = side == 0 ? r : BY + R + r;
        hc = col + R;
        hx = x0 + col;
        hy = side == 0 ? y0 - R + r : y0 + BY + r;
    }
    const bool halo_ld = hr >= 0 && hx < nx + R && hy < ny + R;
    const long long halo_off = (long long)hy * sy + hx;

    T q[Q], hq[Q];
    T qn = T(0), hn = T(0);
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        const int z = z0 - R + k;
        q[k] = own_ld ? src[(long long)z * sz + own_off] : T(0);
        hq[k] = halo_ld ? src[(long long)z * sz + halo_off] : T(0);
    }
    if (z0 + R + 1 < nz + R) {
        qn = own_ld ? src[(long long)(z0 + R + 1) * sz + own_off] : T(0);
        hn = halo_ld ? src[(long long)(z0 + R + 1) * sz + halo_off] : T(0);
    }
    T cw[NARR > 0 ? NARR : 1], cn[NARR > 0 ? NARR : 1];
    if constexpr (NARR > 0) {
#pragma unroll
        for (int m = 0; m < NARR; ++m) {
            cw[m] = own_up && z0 < z1 ? w.arr[m][(long long)z0 * sz + own_off] : T(0);
            cn[m] = T(0);
        }
    }

    for (int z = z0; z < z1; ++z) {
        tile[ty + R][tx + R] = q[R];
        if (hr >= 0) tile[hr][hc] = hq[R];
        if constexpr (NARR > 0) {
            if (own_up && z + 1 < z1) {
#pragma unroll
                for (int m = 0; m < NARR; ++m) cn[m] = w.arr[m][(long long)(z + 1) * sz + own_off];
            }
        }
        __syncthreads();
        if (own_up) {
            auto nb = [&](int dx, int dy, int dz) MWD_INLINE -> T {
                if (dz != 0) return q[R + dz];
                return tile[ty + R + dy][tx + R + dx];
            };
            T u;
            if constexpr (NARR > 0) {
                u = apply_stencil<K, T>(nb, [&](int m) MWD_INLINE -> T { return cw[m]; });
            } else {
                u = apply_stencil<K, T>(nb, [&](int m) MWD_INLINE -> T { return w.c[m]; });
            }
            dst[(long long)z * sz + own_off] = u;
        }
        __syncthreads();
        // advance the queues by one plane; prefetch two planes ahead
#pragma unroll
        for (int k = 0; k < Q - 1; ++k) { q[k] = q[k + 1]; hq[k] = hq[k + 1]; }
        q[Q - 1] = qn;
        hq[Q - 1] = hn;
        const int zp = z + R + 2;
        if (zp < nz + R && z + 1 < z1) {
            qn = own_ld ? src[(long long)zp * sz + own_off] : T(0);
            hn = halo_ld ? src[(long long)zp * sz + halo_off] : T(0);
        }
        if constexpr (NARR > 0) {
#pragma unroll
            for (int m = 0; m < NARR; ++m) cw[m] = cn[m];
        }
    }
}

}  // namespace mwd
