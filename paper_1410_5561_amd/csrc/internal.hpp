// Host-side internal interfaces between the translation units of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

namespace mwd {

enum Kind : int { K7C = 0, K7V = 1, K25C = 2, K25V = 3 };

inline int radius_of(int kind) { return (kind == K7C || kind == K7V) ? 1 : 4; }
inline int narr_of(int kind) { return kind == K7V ? 7 : (kind == K25V ? 13 : 0); }
inline int ndomain_of(int kind) { return kind == K7C ? 2 : kind == K7V ? 9 : kind == K25C ? 2 : 15; }

// The MWD tile kernel addresses a lane's column within a padded plane with a
// 32-bit byte offset: it runs grids whose plane (sz elements) is below 4 GiB.
inline bool mwd_plane_ok(long long sz, int dtype)
{
    return sz >= 0 && sz * (dtype == 0 ? 8LL : 4LL) < (1LL << 32);
}

// A grid as the kernels see it: pointers to the interior origin (element
// (0,0,0)) of each buffer; halo >= R cells exist on every side.
struct DevGrid {
    int nx, ny, nz, halo;
    long long sy, sz;
    int dtype;   // 0 = f64, 1 = f32
    int cur;     // buffer holding the current level
    void* org[2];
};

// Host copy of the weights: constants in double, arrays as interior-origin
// device pointers.
struct HostWeights {
    int kind;
    double c[13];
    const void* org[13];
};

// Optional timing of every kernel a plan launches: an event pair around each
// launch on the launch stream (class 0: the sweep / MWD tile kernels, class 1:
// everything else).  Used by measurement tools through the ABI.
struct Prof {
    bool on = false;
    std::vector<hipEvent_t> start, stop;
    std::vector<int> cls;
    hipEvent_t pending = nullptr;
    void begin(hipStream_t s) {
        if (!on) return;
        pending = nullptr;
        if (hipEventCreate(&pending) == hipSuccess) (void)hipEventRecord(pending, s);
    }
    void end(hipStream_t s, int c) {
        if (!on || !pending) return;
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return;
        (void)hipEventRecord(e, s);
        start.push_back(pending);
        stop.push_back(e);
        cls.push_back(c);
        pending = nullptr;
    }
    // Sum elapsed ms and counts per class, then release the events.
    hipError_t collect(double out[4]) {
        out[0] = out[1] = out[2] = out[3] = 0.0;
        hipError_t err = hipSuccess;
        for (size_t i = 0; i < start.size(); ++i) {
            float ms = 0.f;
            hipError_t e = hipEventSynchronize(stop[i]);
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, start[i], stop[i]);
            if (e != hipSuccess) err = e;
            out[2 * cls[i]] += ms;
            out[2 * cls[i] + 1] += 1.0;
            (void)hipEventDestroy(start[i]);
            (void)hipEventDestroy(stop[i]);
        }
        start.clear();
        stop.clear();
        cls.clear();
        return err;
    }
};

// One full sweep: dst <- op(src) over the interior.
hipError_t naive_sweep(const DevGrid& g, const HostWeights& w, const void* src, void* dst,
                       hipStream_t stream);

// MWD schedule parameters resolved for one (kind, dtype).
struct MwdShape {
    int dw;      // diamond width
    int wpr;     // waves per diamond row (lanes = 64 * wpr)
    int lanes() const { return 64 * wpr; }
};

// True if a compiled MWD kernel exists for (kind, dtype, shape).
bool mwd_supported(int kind, int dtype, const MwdShape& s);
int mwd_levels(int kind, const MwdShape& s);
// All compiled shapes for (kind, dtype); returns how many were written.
int mwd_shapes(int kind, int dtype, MwdShape* out, int cap);
// Whether the shape's row kernel keeps values in scratch memory (register spill).
hipError_t mwd_kernel_scratch(int kind, int dtype, const MwdShape& s, size_t* bytes_per_lane);
// The shape's row kernel: VGPRs per lane, LDS bytes, scratch bytes per lane,
// threads per workgroup, workgroups per CU.
hipError_t mwd_kernel_resources(int kind, int dtype, const MwdShape& s, int out[5]);
int mwd_xtile(int kind, const MwdShape& s);

// Run T steps with MWD.  `scratch` holds two extra grid-sized buffer pairs
// (4 pointers at the interior origin, same strides as g).
hipError_t mwd_run(const DevGrid& g, const HostWeights& w, int T, const MwdShape& s,
                   void* const scratch[4], hipStream_t stream, Prof* prof);
// Rows [rho_lo, rho_hi] of the schedule only, without the boundary fill and
// the gather: for timing (the tuner), not for results.
hipError_t mwd_run_rows(const DevGrid& g, const HostWeights& w, int T, const MwdShape& s, void* const scratch[4],
                        hipStream_t stream, int rho_lo, int rho_hi);

// FP64 norms: which 0 -> of a, which 1 -> of a - b (b may be another dtype).
hipError_t norms_fp64(const DevGrid& ga, const void* a, const DevGrid& gb, const void* b,
                      int which, double out[2], hipStream_t stream);

hipError_t stream_copy(void* dst, const void* src, long long bytes, hipStream_t stream);

void set_last_error(const std::string& s);

}  // namespace mwd
