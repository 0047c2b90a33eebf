// Shared device-side definitions of the gfx950 stencil library: the stencil
// operators of Listings 1-3 (Sec. I-A) and small compile-time helpers.
//
// Every operator is evaluated in the listing's left-to-right C order with
// separately rounded multiplies and adds (this library is built with
// -ffp-contract=off and the pragma below), so any schedule of the same
// lattice-site updates returns the same bits as one plain sweep.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>
#include <utility>

#include "internal.hpp"

#pragma clang fp contract(off)

namespace mwd {

template <int K> struct KindTraits;
template <> struct KindTraits<K7C>  { static constexpr int R = 1, NARR = 0,  NW = 2,  ND = 2;  };
template <> struct KindTraits<K7V>  { static constexpr int R = 1, NARR = 7,  NW = 7,  ND = 9;  };
template <> struct KindTraits<K25C> { static constexpr int R = 4, NARR = 0,  NW = 13, ND = 2;  };
template <> struct KindTraits<K25V> { static constexpr int R = 4, NARR = 13, NW = 13, ND = 15; };

// Lambdas of the hot loops are always inlined: a step body that is not would
// keep its register queues in scratch memory.
#define MWD_INLINE __attribute__((always_inline))

// Compile-time loop: f(std::integral_constant<int, i>) for i in [B, E).
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

constexpr int cgcd(int a, int b) { return b == 0 ? a : cgcd(b, a % b); }
constexpr int clcm(int a, int b) { return a / cgcd(a, b) * b; }
constexpr int cmod(int a, int m) { return ((a % m) + m) % m; }

// Floor division for a possibly negative numerator and a positive divisor.
__host__ __device__ __forceinline__ int floordiv(int a, int b) {
    return a >= 0 ? a / b : -((-a + b - 1) / b);
}

// One lattice-site update (one LUP) of stencil K.
//   nb(dx, dy, dz) -> V at the neighbour (x+dx, y+dy, z+dz) of the previous level
//   w(m)           -> weight m (a constant, or coefficient array m at the point)
// Listing 1: c0*V + c1*(x+ + x-) + c1*(y+ + y-) + c1*(z+ + z-)
// Listing 2: C0*V + C1*x+ + C2*x- + C3*y+ + C4*y- + C5*z+ + C6*z-
// Listing 3: C00*V + sum over r = 1..4, axis x, y, z of C_{r,axis}*(V(+r) + V(-r))
template <int K, typename T, class NB, class WF>
__device__ __forceinline__ T apply_stencil(const NB& nb, const WF& w) {
    if constexpr (K == K7C) {
        T u = w(0) * nb(0, 0, 0);
        u = u + w(1) * (nb(1, 0, 0) + nb(-1, 0, 0));
        u = u + w(1) * (nb(0, 1, 0) + nb(0, -1, 0));
        u = u + w(1) * (nb(0, 0, 1) + nb(0, 0, -1));
        return u;
    } else if constexpr (K == K7V) {
        T u = w(0) * nb(0, 0, 0);
        u = u + w(1) * nb(1, 0, 0);
        u = u + w(2) * nb(-1, 0, 0);
        u = u + w(3) * nb(0, 1, 0);
        u = u + w(4) * nb(0, -1, 0);
        u = u + w(5) * nb(0, 0, 1);
        u = u + w(6) * nb(0, 0, -1);
        return u;
    } else {
        T u = w(0) * nb(0, 0, 0);
        static_for<1, 5>([&](auto rc) MWD_INLINE {
            constexpr int r = decltype(rc)::value;
            u = u + w(3 * (r - 1) + 1) * (nb(r, 0, 0) + nb(-r, 0, 0));
            u = u + w(3 * (r - 1) + 2) * (nb(0, r, 0) + nb(0, -r, 0));
            u = u + w(3 * (r - 1) + 3) * (nb(0, 0, r) + nb(0, 0, -r));
        });
        return u;
    }
}

// Kernel-argument view of the weights.  Pointers address the interior origin
// (element (0,0,0)) of coefficient arrays laid out like the grid.
template <typename T>
struct Weights {
    T c[13];
    const T* arr[13];
};

// Logical block of workgroup blk in a launch of ntiles blocks.  Workgroups
// go to the eight XCDs round-robin (block i to XCD i mod 8), each XCD with
// its own L2.  Neighbouring blocks that share cache lines (the overlapping x
// tiles of one diamond; the x- and y-neighbours of a sweep's blocks) should
// run on one XCD, where the second read of a shared line can hit in L2: so
// runs of c consecutive logical blocks go to one XCD.  The last, partial
// group of 8c blocks keeps the identity; the map is a bijection.
__host__ __device__ __forceinline__ int xcd_tile(int blk, int ntiles, int c)
{
    constexpr int NXCD = 8;
    const int gsz = NXCD * c;
    const int g = blk / gsz;
    if ((g + 1) * gsz > ntiles) return blk;
    const int r = blk - g * gsz;
    return g * gsz + (r % NXCD) * c + r / NXCD;
}

}  // namespace mwd
