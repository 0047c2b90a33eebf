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
// an LDS exchange array that gives the y-neighbours and, except for radius-1
// rows of one wave (whose x-neighbours move between lanes by DPP shifts), the
// x-neighbours.  One workgroup barrier per wavefront step; the exchange array
// is double-buffered.
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
    // Loads are issued PL steps before the step that consumes them, so that
    // PL steps of compute cover the memory latency (two for the radius-4
    // stencil, whose 9-plane queues leave fewer registers).
    static constexpr int PL = R == 1 ? 3 : 2;
    // coefficient ring: planes [s - LR, s - R] are in use at step s, and the
    // load for plane s + PD - R is in flight; the ring is rounded up to a
    // multiple of Q and PD takes what the rounding leaves (at least 2)
    static constexpr int WIN = NARR ? Q * (((L - 1) * R + 3 + Q - 1) / Q) : 1;
    static constexpr int PD = NARR ? ((WIN - (L - 1) * R - 1) < PL ? (WIN - (L - 1) * R - 1) : PL) : 1;
    static_assert(NARR == 0 || (PD >= 1 && PD + (L - 1) * R < WIN), "coefficient ring too short");
    static constexpr int U = clcm(clcm(Q, WIN), PL);  // unroll: ring slots become constants
    static constexpr int NS = DW + 2 * R;           // LDS row slots (diamond rows + side rows)
    static constexpr int NSX = NS + 1;              // plus a spare row for writes nobody reads
    static constexpr int S0 = U * ((R + PL + U - 1) / U);  // step offset, multiple of U, >= R + PL
};

// A value the compiler must recompute where it is used (it passes through a
// vector register): keeps per-step offsets (a compile-time step times a
// run-time stride) from being hoisted out of the chunk loop, where they would
// hold one register each for the whole loop.
__device__ __forceinline__ uint32_t opaque_u32(uint32_t v)
{
    asm volatile("" : "+v"(v));
    return v;
}

// The same for a wave-uniform value that stays in a scalar register: stops
// loop strength reduction from turning every per-step address of the cold
// (boundary) steps into an induction variable of its own.
__device__ __forceinline__ int opaque_uniform(int v)
{
    asm volatile("" : "+v"(v));
    return __builtin_amdgcn_readfirstlane(v);
}

// An empty side effect: a branch around it stays a branch instead of
// becoming per-lane selects.
__device__ __forceinline__ void keep_branch() { asm volatile(""); }

// Cross-lane moves of a wave (DPP wavefront shifts by one lane): lane i takes
// lane i + 1's value (kDppFromAbove) or lane i - 1's (kDppFromBelow); the
// lane with no source takes 0.  Every lane of the wave must be active.
constexpr int kDppFromAbove = 0x130;  // wave_shl:1
constexpr int kDppFromBelow = 0x138;  // wave_shr:1

template <int CTRL, typename T>
__device__ __forceinline__ T dpp_move(T v)
{
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, false));
    } else {
        const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
        const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xf, 0xf, false);
        const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, false);
        return __builtin_bit_cast(T, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
    }
}

// Level sets of the diamond rows of a tile that no clipping touches (every
// row inside the domain, every level inside 1 .. T).  Row yr of such a tile
// computes level tau iff its distance d from the diamond's centre satisfies
// d < R min(tau, 2h - tau); it holds (publishes) level tau if it computes it
// or a row within R of it computes tau + 1; it stores its top two computed
// levels.  Rows with equal sets share one row type; the steady-state body is
// compiled once per type with these sets as constants, so that a wave of such
// a tile runs no per-level tests.
template <int R, int DW, int H, int L>
struct CanonRows {
    static constexpr bool computed(int yrr, int tau)
    {
        if (tau < 1 || tau > L || yrr < 0 || yrr >= DW) return false;
        const int d = yrr < DW / 2 ? DW / 2 - 1 - yrr : yrr - DW / 2;
        return d < R * (tau < 2 * H - tau ? tau : 2 * H - tau);
    }
    static constexpr uint32_t cmask(int yr)
    {
        uint32_t m = 0;
        for (int tau = 0; tau <= L; ++tau)
            if (computed(yr, tau)) m |= 1u << tau;
        return m;
    }
    static constexpr uint32_t pmask(int yr)
    {
        uint32_t m = cmask(yr);
        for (int tau = 0; tau < L; ++tau)
            for (int dy = -R; dy <= R; ++dy)
                if (computed(yr + dy, tau + 1)) m |= 1u << tau;
        return m;
    }
    static constexpr uint32_t smask(int yr)
    {
        const uint32_t c = cmask(yr);
        int thi = -1;
        for (int tau = 0; tau <= L; ++tau)
            if ((c >> tau) & 1u) thi = tau;
        uint32_t m = 0;
        for (int tau = 0; tau <= L; ++tau)
            if (((c >> tau) & 1u) && tau >= thi - 1) m |= 1u << tau;
        return m;
    }
    static constexpr bool same(int a, int b)
    {
        return cmask(a) == cmask(b) && pmask(a) == pmask(b) && smask(a) == smask(b);
    }
    static constexpr bool first_of_type(int yr)
    {
        for (int o = 0; o < yr; ++o)
            if (same(o, yr)) return false;
        return true;
    }
    static constexpr int ntypes()
    {
        int n = 0;
        for (int yr = 0; yr < DW; ++yr)
            if (first_of_type(yr)) ++n;
        return n;
    }
    // a row of type i
    static constexpr int rep(int i)
    {
        for (int yr = 0, n = 0; yr < DW; ++yr)
            if (first_of_type(yr) && n++ == i) return yr;
        return -1;
    }
    static constexpr int lowbit(uint32_t m)
    {
        for (int b = 0; b < 32; ++b)
            if ((m >> b) & 1u) return b;
        return -1;
    }
    // edge levels (held, not computed) of type i, -1: none
    static constexpr int ta(int i) { return lowbit(pmask(rep(i)) & ~cmask(rep(i))); }
    static constexpr int tb(int i)
    {
        const uint32_t e = pmask(rep(i)) & ~cmask(rep(i));
        return lowbit(e & (e - 1u));
    }
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

// Lanes take x; rows y stride over the grid's y blocks (the launch may have
// fewer y blocks than the rows need: gridDim.y is at most 65535); planes
// [z0, z1) of the padded range [-r, nz + r).
template <typename T>
__device__ __forceinline__ void halo_fill_one(const HaloFill<T>& e, int z0, int z1)
{
    const int x = blockIdx.x * 64 + (threadIdx.x & 63) - e.r;
    if (x >= e.nx + e.r) return;
    for (int y = blockIdx.y * 4 + (threadIdx.x >> 6) - e.r; y < e.ny + e.r; y += gridDim.y * 4) {
        const bool col_inside = x >= 0 && x < e.nx && y >= 0 && y < e.ny;
        for (int z = z0; z < z1; ++z) {
            if (col_inside && z >= 0 && z < e.nz) {  // skip the interior of an interior column
                z = e.nz - 1;
                continue;
            }
            const long long off = (long long)z * e.sz + (long long)y * e.sy + x;
            const T v = e.src[off];
#pragma unroll
            for (int k = 0; k < 4; ++k) e.dst[k][off] = v;
        }
    }
}

// Largest y or z extent of a launch grid.
constexpr int kMaxGridYZ = 65535;
// Planes per block of the single-grid fill: the columns on the domain's x
// and y faces hold boundary values in every plane, and one thread walking
// all of them in sequence was latency-bound.
constexpr int kFillPlanes = 32;

template <typename T>
__global__ void __launch_bounds__(256) mwd_halo_fill_kernel(HaloFill<T> e)
{
    // z chunks stride over the launch's blocks (gridDim.z <= 65535)
    for (int z0 = -e.r + (int)blockIdx.z * kFillPlanes; z0 < e.nz + e.r; z0 += gridDim.z * kFillPlanes)
        halo_fill_one(e, z0, min(e.nz + e.r, z0 + kFillPlanes));
}

// Batched: entry blockIdx.z of a device table, all planes.
template <typename T>
__global__ void __launch_bounds__(256) mwd_halo_fill_table_kernel(const HaloFill<T>* __restrict__ table)
{
    const HaloFill<T>& e = table[blockIdx.z];
    halo_fill_one(e, -e.r, e.nz + e.r);
}

// The tile (diamond b of the row, x tile j) computed by one workgroup.
template <int K, typename T, int DW, int WPR>
__device__ __forceinline__ void mwd_tile(const MwdArgs<T>& a, const MwdRow& row, int b, int j,
                                         T (*ex)[MwdGeom<K, DW, WPR>::L][MwdGeom<K, DW, WPR>::NSX]
                                              [MwdGeom<K, DW, WPR>::LX])
{
    using G = MwdGeom<K, DW, WPR>;
    constexpr int R = G::R, H = G::H, L = G::L, Q = G::Q, LX = G::LX, XT = G::XT;
    constexpr int NARR = G::NARR, WIN = G::WIN, U = G::U, PL = G::PL;

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
    auto computed = [&](int yrr, int tau) MWD_INLINE -> bool {
        if (tau < 1 || tau > L || yrr < 0 || yrr >= DW) return false;
        const int t = row.t0 + tau;
        if (t < 1 || t > a.nsteps) return false;
        const int yy = yL + yrr;
        if (yy < 0 || yy >= a.ny) return false;
        const int d = yrr < DW / 2 ? DW / 2 - 1 - yrr : yrr - DW / 2;
        return d < R * min(tau, 2 * H - tau);
    };
    auto needed = [&](int yrr, int tau) MWD_INLINE -> bool {
        if (tau >= L) return false;
        bool n = false;
        for (int dy = -R; dy <= R; ++dy) n = n || computed(yrr + dy, tau + 1);
        return n;
    };
    // Source of a level-t value at row yy that this tile does not compute.
    auto level_src = [&](int yy, int t) MWD_INLINE -> const T* {
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

    T* dst[L + 1];
    T* const* outp = a.pair[pair_of_row(row.rho)];
#pragma unroll
    for (int tau = 0; tau <= L; ++tau) dst[tau] = outp[(a.cur + row.t0 + tau) & 1];

    // Edge levels: the levels of this row that the tile needs but does not
    // compute.  On the rising side of a diamond level tau + 1 reaches R rows
    // further out on each side than level tau, so a row is needed, before its
    // first computed level, at the two levels just below it (fewer where the
    // diamond is clipped); they are read from the rows below.  ta < tb.
    const uint32_t emask = pmask & ~cmask;
    const uint32_t erest = emask & (emask - 1u);
    const bool has_a = emask != 0u, has_b = erest != 0u;
    const int ta = has_a ? __builtin_ctz(emask) : 0;
    const int tb = has_b ? __builtin_ctz(erest) : 0;
    const T* srca = level_src(y, row.t0 + ta);
    const T* srcb = level_src(y, row.t0 + tb);
    // Boundary values are the same at every level: a lane outside the domain
    // (and every lane at a boundary plane) loads level 0 from the boundary
    // array and each higher level copies the same plane from the level below.
    const bool lane_in = xin && yin;

    // Side rows: R rows beyond each edge of the diamond, needed only at level
    // h - 1 by the widest level h.  Diamond row yr < 2R loads one of them
    // (yr < R: left side row yr - R; else right side row DW + yr - R) straight
    // into its LDS slot; the other waves write a spare LDS row nobody reads.
    const bool side_wave = wave_active && yr < 2 * R;
    const int yrs = yr < R ? yr - R : DW + yr - R;
    const int sv_y = yL + yrs;
    const bool sv_present = side_wave && needed(yrs, H - 1);
    const T* sv_src = level_src(sv_y, row.t0 + H - 1);
    const int side_slot = sv_present ? yrs + R : G::NS;  // NS: the spare row

    // z-queues of levels 0 .. L-1; the top level L is read by no other level,
    // only by the delayed stores, so it keeps just its current and previous plane
    T q[L][Q];
    T qtop = T(0), qtop_prev = T(0);
    T lea[PL], leb[PL], bzr[PL], sv[PL];
    T cr[NARR > 0 ? NARR : 1][WIN];
#pragma unroll
    for (int tau = 0; tau < L; ++tau)
#pragma unroll
        for (int k = 0; k < Q; ++k) q[tau][k] = T(0);
#pragma unroll
    for (int k = 0; k < PL; ++k) {
        lea[k] = leb[k] = bzr[k] = sv[k] = T(0);
    }
#pragma unroll
    for (int m = 0; m < (NARR > 0 ? NARR : 1); ++m)
#pragma unroll
        for (int k = 0; k < WIN; ++k) cr[m][k] = T(0);

    const long long col = (long long)y * a.sy + x;
    const int s_first = -G::S0;
    // one step past the last plane of the last level, for its delayed stores
    const int s_last = a.nz + R + L * R;

    // Steady state: the steps s in [LR + 1, nz - PL) touch only planes inside
    // the domain (every level's plane, every load and every store), so they
    // run without plane checks.  They are taken in whole chunks of U steps,
    // and only while U + LR + 1 planes span less than 4 GiB, so that a chunk
    // can address each array through one 64-bit base and 32-bit lane offsets.
    const long long szb = a.sz * (long long)sizeof(T);
    const bool fast_ok = (long long)(U + L * R + 1) * szb < (1LL << 32);
    const int s_fast_begin = fast_ok ? U * ((L * R + 1 + U - 1) / U) : s_first;
    const int s_fast_end = fast_ok ? max(s_fast_begin, U * floordiv(a.nz - PL, U)) : s_first;
    // does any lane of this wave stand for a point outside the domain?
    const bool wave_bnd = __any(wave_active && xact && !lane_in && pmask != 0u);
    // lane byte offsets from the plane corner (x, y) = (-R, -R); 0 for a
    // lane with nothing to load (it then reads the corner)
    const long long corner = (long long)R * a.sy + R;
    const bool col_ok = xact && y >= -R && y < a.ny + R;
    const uint32_t colb = col_ok ? (uint32_t)((col + corner) * (long long)sizeof(T)) : 0u;
    const uint32_t off_s = sv_present && xact
                               ? (uint32_t)(((long long)(sv_y + R) * a.sy + x + R) * (long long)sizeof(T))
                               : 0u;
    // byte address of the corner of plane p of an array
    auto plane = [&](const T* arr, int p) MWD_INLINE -> const char* {
        return reinterpret_cast<const char*>(arr) + ((long long)p * a.sz - corner) * (long long)sizeof(T);
    };
    auto ld = [](const char* base, uint32_t off) MWD_INLINE -> T { return *reinterpret_cast<const T*>(base + off); };
    const int par0 = (a.cur + row.t0) & 1;  // buffer of the even levels
    const int ea = has_a ? ta : -1, eb_ = has_b ? tb : -1;  // edge levels, -1: none

    // One wavefront step.  FAST: a steady-state step (see above).  ti: the
    // wave's row type (its level sets as constants), or -1 (any row).
    using CR = CanonRows<R, DW, H, L>;
    auto step = [&](auto uc, auto fc, auto ti, int s, const char* const* cb) MWD_INLINE {
        constexpr int u = decltype(uc)::value;
        constexpr bool FAST = decltype(fc)::value;
        constexpr int TI = decltype(ti)::value;
        constexpr bool CAN = TI >= 0;
        // a typed steady-state step computes every lane (see below)
        constexpr bool UNMASKED = CAN && FAST;
        constexpr int k = u % PL;  // load slot consumed, then refilled, at this step
        const int eb = s & 1;
        // the wave's level sets: constants for a row type; otherwise re-read
        // at every step so that the per-level tests below stay scalar
        // compares instead of lane masks held (and spilled) across the loop
        uint32_t cm, pm, sm;
        int e1, e2;
        bool hasa, hasb;
        if constexpr (CAN) {
            constexpr int yt = CR::rep(CAN ? TI : 0);
            constexpr uint32_t CM = CR::cmask(yt), PM = CR::pmask(yt), SM = CR::smask(yt);
            constexpr int TA = CR::ta(CAN ? TI : 0), TB = CR::tb(CAN ? TI : 0);
            cm = CM;
            pm = PM;
            sm = SM;
            e1 = TA;
            e2 = TB;
            hasa = TA >= 0;
            hasb = TB >= 0;
        } else {
            cm = (uint32_t)opaque_uniform((int)cmask);
            pm = (uint32_t)opaque_uniform((int)pmask);
            sm = (uint32_t)opaque_uniform((int)smask);
            e1 = opaque_uniform(ea);
            e2 = opaque_uniform(eb_);
            hasa = has_a;
            hasb = has_b;
        }
        qtop_prev = qtop;  // level L's plane s - 1 - LR, for this step's stores
        // plane s - 1 - tau R of level tau (the previous step's), for the stores
        auto qold = [&](auto tc) MWD_INLINE -> T {
            constexpr int tau = decltype(tc)::value;
            if constexpr (tau == L) return qtop_prev;
            else return q[tau][cmod(u - 1 - tau * R, Q)];
        };
        // (1) publish, for every level tau < L, the plane level tau + 1 reads
        //     in-plane neighbours from at this step, and the side row.  In the
        //     steady state a level this row does not hold publishes too: no
        //     other row reads that slot.
        static_for<0, L>([&](auto tc) MWD_INLINE {
            constexpr int tau = decltype(tc)::value;
            const int p = s - (tau + 1) * R;
            const bool held = ((pm >> tau) & 1u) != 0u;
            const bool pub = FAST ? (!CAN || held) : (held && p >= 0 && p < a.nz);
            if (pub) ex[eb][tau][yr + R][xl] = q[tau][cmod(u - (tau + 1) * R, Q)];
        });
        // side row: unconditional, so the wait for its load is the same on
        // every path
        ex[eb][H - 1][side_slot][xl] = sv[k];
        __syncthreads();
        // (2) plane s - tau R of every level that is not computed here:
        //     boundary values, or the edge levels loaded PL steps ago (lanes
        //     that compute below overwrite theirs)
        // edge levels: uniform branches (kept as branches, not lane selects)
        static_for<0, L>([&](auto tc) MWD_INLINE {
            constexpr int tau = decltype(tc)::value;
            if (e1 == tau) {
                keep_branch();
                q[tau][cmod(u - tau * R, Q)] = lea[k];
            } else if (e2 == tau) {
                keep_branch();
                q[tau][cmod(u - tau * R, Q)] = leb[k];
            }
        });
        // boundary values: lanes outside the domain, and, outside the steady
        // state, every lane of a level whose plane is a boundary plane.  Each
        // level copies the level below at the same plane, which is final
        // before this step, so the copy may come before or after the
        // computation: a row type computes every lane (lanes outside the
        // domain compute values nobody reads) and copies afterwards.
        const bool bnd_planes = !FAST && (s - L * R < 0 || s >= a.nz);
        auto boundary = [&]() MWD_INLINE {
          if (wave_bnd || bnd_planes) {
            static_for<0, L + 1>([&](auto tc) MWD_INLINE {
                constexpr int tau = decltype(tc)::value;
                const int p = s - tau * R;
                const bool bnd = !lane_in || (!FAST && (p < 0 || p >= a.nz));
                T bv;
                if constexpr (tau == 0) bv = bzr[k];
                else bv = q[tau - 1][cmod(u - tau * R, Q)];
                if constexpr (tau == L) {
                    if (bnd) qtop = bv;
                } else {
                    if (bnd) q[tau][cmod(u - tau * R, Q)] = bv;
                }
            });
          }
        };
        if constexpr (!UNMASKED) boundary();
        // (3) stores of the previous step (its values are still in the
        //     queues): the last two levels of each point.  Issued before this
        //     step's loads, so waits on those loads stay exact.
        static_for<1, L + 1>([&](auto tc) MWD_INLINE {
            constexpr int tau = decltype(tc)::value;
            const int p = s - 1 - tau * R;
            if constexpr (FAST) {
                // cb[4 + (tau & 1)]: corner of plane sb - 1 - LR of the
                // buffer that holds level tau
                if (((sm >> tau) & 1u) && xout) {
                    char* base = const_cast<char*>(cb[4 + (tau & 1)]);
                    const uint32_t off = colb + opaque_u32((uint32_t)((u + (L - tau) * R) * szb));
                    *reinterpret_cast<T*>(base + off) = qold(tc);
                }
            } else {
                if (((sm >> tau) & 1u) && p >= 0 && p < a.nz && xout)
                    *reinterpret_cast<T*>(const_cast<char*>(plane(dst[tau], p)) + colb) = qold(tc);
            }
        });
        // (4) issue the loads consumed PL steps from now (PD for the
        //     coefficients): side row, edge levels, the boundary plane of
        //     level 0, coefficients.  A wave issues the loads it can need on
        //     every step it can need them; each lane reads its own column
        //     (lanes whose value nobody uses read valid neighbouring data).
        if constexpr (FAST) {
            // cb[0..3]: corners of the chunk's first planes of the side row,
            // edge level a, edge level b and the boundary array; cb[6 + m]:
            // coefficient array m
            const uint32_t du = opaque_u32((uint32_t)(u * szb));
            const uint32_t o = colb + du;
            if (sv_present) sv[k] = ld(cb[0], off_s + du);
            if (hasa) lea[k] = ld(cb[1], o);
            if (hasb) leb[k] = ld(cb[2], o);
            if (wave_bnd) bzr[k] = ld(cb[3], o);
            if constexpr (NARR > 0) {
                constexpr int PD = G::PD;
                if (cm != 0u) {
#pragma unroll
                    for (int m = 0; m < NARR; ++m) cr[m][cmod(u + PD - R, WIN)] = ld(cb[6 + m], o);
                }
            }
        } else {
            // a stream whose plane lies outside its range loads, on every
            // lane, the corner of the nearest plane inside it
            auto gld = [&](const T* arr, int p, int lo, int hi, uint32_t off) MWD_INLINE -> T {
                const bool in = p >= lo && p < hi;
                return ld(plane(arr, min(max(p, lo), hi - 1)), in ? off : 0u);
            };
            const int pl = s + PL;  // level 0's plane at step s + PL
            if (sv_present) sv[k] = gld(sv_src, pl - H * R, 0, a.nz, off_s);
            if (hasa) lea[k] = gld(srca, pl - ta * R, 0, a.nz, colb);
            if (hasb) leb[k] = gld(srcb, pl - tb * R, 0, a.nz, colb);
            // boundary values: at boundary planes every lane needs them, at
            // other planes the lanes outside the domain
            const bool pbnd = pl < 0 || pl >= a.nz;
            if (pm != 0u && (wave_bnd || pbnd)) bzr[k] = gld(a.halo, pl, -R, a.nz + R, colb);
            if constexpr (NARR > 0) {
                constexpr int PD = G::PD;
                const int pc = s + PD - R;
                if (cm != 0u) {
#pragma unroll
                    for (int m = 0; m < NARR; ++m)
                        cr[m][cmod(u + PD - R, WIN)] = gld(a.w.arr[m], pc, 0, a.nz, colb);
                }
            }
        }
        // (5) advance every computed level by one plane, lowest level first:
        //     level tau reads level tau - 1's plane p + R just made
        //     Where registers allow (radius 1 with at most 3 levels, or 7 in
        //     FP32), the in-plane neighbours of every level are read from
        //     LDS up front, so that the levels' chain does not wait on LDS
        //     once per level.  With one wave per diamond row at radius 1,
        //     the x-neighbours come from the neighbouring lanes of the same
        //     wave instead (a lane's own register holds the value it
        //     published), by DPP shifts in wave-uniform control flow.
        constexpr bool XDPP = R == 1 && WPR == 1;
        constexpr bool XYPF = R == 1 && (L <= 3 || (sizeof(T) == 4 && L <= 7));
        T xy[XYPF ? L + 1 : 1][4];
        if constexpr (XYPF) {
            if (UNMASKED || (xl >= R && xl < LX - R)) {
                static_for<1, L + 1>([&](auto tc) MWD_INLINE {
                    constexpr int tau = decltype(tc)::value;
                    if constexpr (!XDPP) {
                        xy[tau][0] = ex[eb][tau - 1][yr + R][xl + 1];
                        xy[tau][1] = ex[eb][tau - 1][yr + R][xl - 1];
                    }
                    xy[tau][2] = ex[eb][tau - 1][yr + R + 1][xl];
                    xy[tau][3] = ex[eb][tau - 1][yr + R - 1][xl];
                });
            }
        }
        static_for<1, L + 1>([&](auto tc) MWD_INLINE {
            constexpr int tau = decltype(tc)::value;
            const int p = s - tau * R;
            if (((cm >> tau) & 1u) && (FAST || (p >= 0 && p < a.nz))) {
                // the x-neighbours by lane shifts, before any per-lane branch
                T xa = T(0), xb = T(0);
                if constexpr (XDPP) {
                    const T c = q[tau - 1][cmod(u - tau * R, Q)];
                    xa = dpp_move<kDppFromAbove>(c);
                    xb = dpp_move<kDppFromBelow>(c);
                }
                // a row type computes every lane: a lane outside the level's
                // x range reads in-bounds LDS and its value is never read
                if (UNMASKED || (xin && xl >= tau * R && xl < LX - tau * R)) {
                    auto nb = [&](int dx, int dy, int dz) MWD_INLINE -> T {
                        if (dz != 0) return q[tau - 1][cmod(u - tau * R + dz, Q)];
                        if constexpr (XDPP) {
                            if (dx > 0) return xa;
                            if (dx < 0) return xb;
                        }
                        if constexpr (XYPF) {
                            if (dx > 0) return xy[tau][0];
                            if (dx < 0) return xy[tau][1];
                            if (dy > 0) return xy[tau][2];
                            if (dy < 0) return xy[tau][3];
                        } else {
                            if (dy != 0) return ex[eb][tau - 1][yr + R + dy][xl];
                            if (dx != 0) return ex[eb][tau - 1][yr + R][xl + dx];
                        }
                        return q[tau - 1][cmod(u - tau * R, Q)];
                    };
                    T v;
                    if constexpr (NARR > 0) {
                        v = apply_stencil<K, T>(nb, [&](int m) MWD_INLINE -> T { return cr[m][cmod(u - tau * R, WIN)]; });
                    } else {
                        v = apply_stencil<K, T>(nb, [&](int m) MWD_INLINE -> T { return a.w.c[m]; });
                    }
                    if constexpr (tau == L) qtop = v;
                    else q[tau][cmod(u - tau * R, Q)] = v;
                }
            }
        });
        if constexpr (UNMASKED) boundary();
    };

    const char* const nocb[1] = {nullptr};
    auto generic_chunks = [&](auto ti, int from, int to) MWD_INLINE {
        for (int sb = from; sb < to; sb += U)
            static_for<0, U>([&](auto uc) MWD_INLINE {
                step(uc, std::false_type{}, ti, opaque_uniform(sb + decltype(uc)::value), nocb);
            });
    };
    auto fast_chunks = [&](auto ti) MWD_INLINE {
      for (int sb = s_fast_begin; sb < s_fast_end; sb += U) {
        const int pl = sb + PL;
        const char* cb[6 + (NARR > 0 ? NARR : 1)];
        cb[0] = plane(sv_src, pl - H * R);
        cb[1] = plane(srca, pl - ta * R);
        cb[2] = plane(srcb, pl - tb * R);
        cb[3] = plane(a.halo, pl);
        cb[4] = plane(a.pair[pair_of_row(row.rho)][par0], sb - 1 - L * R);
        cb[5] = plane(a.pair[pair_of_row(row.rho)][par0 ^ 1], sb - 1 - L * R);
        if constexpr (NARR > 0) {
#pragma unroll
            for (int m = 0; m < NARR; ++m) cb[6 + m] = plane(a.w.arr[m], sb + G::PD - R);
        }
        static_for<0, U>([&](auto uc) MWD_INLINE { step(uc, std::true_type{}, ti, sb + decltype(uc)::value, cb); });
      }
    };
    auto sweep = [&](auto ti) MWD_INLINE {
        generic_chunks(ti, s_first, s_fast_begin);
        fast_chunks(ti);
        generic_chunks(ti, s_fast_end, s_last + 1);
    };
    // the wave's row type, if its level sets are those of an unclipped tile;
    // shapes with more than five types (Dw 16 at radius 1, whose 15 levels
    // do not fit the registers anyway) compile the untyped sweep only
    constexpr int NTYPES = CR::ntypes() <= 5 ? CR::ntypes() : 0;
    int rtype = -1;
    static_for<0, NTYPES>([&](auto ic) MWD_INLINE {
        constexpr int yt = CR::rep(decltype(ic)::value);
        constexpr uint32_t CM = CR::cmask(yt), PM = CR::pmask(yt), SM = CR::smask(yt);
        if (cmask == CM && pmask == PM && smask == SM) rtype = decltype(ic)::value;
    });
    rtype = __builtin_amdgcn_readfirstlane(rtype);
    if (rtype < 0) sweep(std::integral_constant<int, -1>{});
    static_for<0, NTYPES>([&](auto ic) MWD_INLINE {
        if (rtype == decltype(ic)::value) sweep(ic);
    });
}

}  // namespace mwd
