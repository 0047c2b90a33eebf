// Batched naive sweep: one launch advances a group of naive-planned grids of
// a batch by one step; a workgroup takes one (grid, x block, y block, z
// chunk) entry of a table.  Used, inside the batch's hipGraph, for the grids
// the tuner finds faster without MWD tiles (small grids, where the tiles are
// mostly overlap and edge).  The grids are grouped so that a group's arrays
// fit the GPU's last-level (Infinity) cache, and each group takes all T steps
// before the next starts: temporal blocking in that cache, the same aim as
// the diamonds' blocking in registers and LDS (Sec. II).
#pragma once

#include "naive_block.hpp"

namespace mwd {

constexpr int kNaiveBX = 64, kNaiveBY = 16;  // 1024 threads for every kind

struct NaiveTile {
    int grid, bx, by, bz;
};

template <typename T>
struct NaiveArgs {
    T* buf[2];  // interior-origin pointers of the grid's two buffers
    Weights<T> w;
    int kind, nx, ny, nz, zchunk, cur;
    long long sy, sz;
};

template <typename T>
struct NaiveLaunch {
    const NaiveTile* tiles;
    const NaiveArgs<T>* args;
    int first;  // first table entry of this launch
    int t;      // step of this launch: reads level t, writes level t + 1
};

template <typename T>
__device__ __forceinline__ void batch_naive_tile(const NaiveLaunch<T>& L, char* lds)
{
    const NaiveTile e = L.tiles[L.first + blockIdx.x];
    const NaiveArgs<T>& a = L.args[e.grid];
    const T* src = a.buf[(a.cur + L.t) & 1];
    T* dst = a.buf[(a.cur + L.t + 1) & 1];
    switch (a.kind) {
        case K7C:
            naive_block<K7C, T, kNaiveBX, kNaiveBY, naive_prefetch<K7C, T>(true), true>(src, dst, a.w, a.nx, a.ny, a.nz, a.sy, a.sz, a.zchunk, e.bx,
                                                    e.by, e.bz, reinterpret_cast<T (*)[kNaiveBY + 2][kNaiveBX + 2]>(lds));
            break;
        case K7V:
            naive_block<K7V, T, kNaiveBX, kNaiveBY, naive_prefetch<K7V, T>(true), true>(src, dst, a.w, a.nx, a.ny, a.nz, a.sy, a.sz, a.zchunk, e.bx,
                                                    e.by, e.bz, reinterpret_cast<T (*)[kNaiveBY + 2][kNaiveBX + 2]>(lds));
            break;
        case K25C:
            naive_block<K25C, T, kNaiveBX, kNaiveBY, naive_prefetch<K25C, T>(true), true>(src, dst, a.w, a.nx, a.ny, a.nz, a.sy, a.sz, a.zchunk, e.bx,
                                                     e.by, e.bz, reinterpret_cast<T (*)[kNaiveBY + 8][kNaiveBX + 8]>(lds));
            break;
        default:
            naive_block<K25V, T, kNaiveBX, kNaiveBY, naive_prefetch<K25V, T>(true), true>(src, dst, a.w, a.nx, a.ny, a.nz, a.sy, a.sz, a.zchunk, e.bx,
                                                     e.by, e.bz, reinterpret_cast<T (*)[kNaiveBY + 8][kNaiveBX + 8]>(lds));
            break;
    }
}

// LDS of the largest block (radius 4): one plane buffer
template <typename T>
constexpr size_t naive_lds_bytes() { return sizeof(T) * (kNaiveBY + 8) * (kNaiveBX + 8); }

hipError_t batch_naive_launch_f64(const NaiveLaunch<double>& L, int nblocks, hipStream_t s);
hipError_t batch_naive_launch_f32(const NaiveLaunch<float>& L, int nblocks, hipStream_t s);

}  // namespace mwd
