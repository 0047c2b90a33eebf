// FP64 norms over the interior of a grid (or of a difference of two grids),
// accumulated in FP64 whatever the storage precision: two passes, per-block
// partial sums and maxima, then one block combines them in a fixed order, so
// a result is reproducible run to run.  The max propagates NaN: a NaN
// anywhere in the interior makes the max norm NaN.
//
// Two ways to hold the per-block partials:
//   - norms_fp64: a buffer the library allocates once per device; the call
//     is synchronous (result on the host) and holds a lock from launch to
//     completion, so concurrent calls from several threads do not share it;
//   - norms_fp64_static: a fixed array in the library's device memory
//     (`scratch` below), so the call allocates nothing; the result goes to
//     caller-owned device memory, asynchronously.  Calls that overlap on one
//     device share that array and race.
#include <mutex>

#include "common.hpp"
#include "internal.hpp"
#include "reduce.hpp"

namespace mwd {

constexpr int kNormThreads = 256;
constexpr int kNormMaxBlocks = 2048;
// partial sums and maxima of at most kNormMaxBlocks blocks
constexpr int kNormPartials = 2 * kNormMaxBlocks;

// max(m, |v|) that keeps a NaN once one is seen (fmax would drop it)
__device__ __forceinline__ double nan_max(double m, double v)
{
    return (v > m || v != v) ? v : m;
}

template <typename TA, typename TB, bool DIFF>
__global__ void __launch_bounds__(kNormThreads)
norm_partial_kernel(const TA* __restrict__ a, const TB* __restrict__ b, int nx, int ny, int nz,
                    long long asy, long long asz, long long bsy, long long bsz,
                    double* __restrict__ part)
{
    __shared__ double ssum[kNormThreads];
    __shared__ double smax[kNormThreads];
    double s = 0.0, m = 0.0;
    const long long rows = (long long)ny * nz;
    // one (y, z) row per block iteration; lanes stride along x
    for (long long r = blockIdx.x; r < rows; r += gridDim.x) {
        const int y = (int)(r % ny), z = (int)(r / ny);
        const TA* ar = a + z * asz + (long long)y * asy;
        const TB* br = DIFF ? b + z * bsz + (long long)y * bsy : nullptr;
        for (int x = threadIdx.x; x < nx; x += kNormThreads) {
            double v = (double)ar[x];
            if (DIFF) v = v - (double)br[x];
            s += v * v;
            m = nan_max(m, fabs(v));
        }
    }
    ssum[threadIdx.x] = s;
    smax[threadIdx.x] = m;
    __syncthreads();
    for (int w = kNormThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            ssum[threadIdx.x] += ssum[threadIdx.x + w];
            smax[threadIdx.x] = nan_max(smax[threadIdx.x], smax[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = ssum[0];
        part[2 * blockIdx.x + 1] = smax[0];
    }
}

__global__ void __launch_bounds__(kNormThreads)
norm_final_kernel(const double* __restrict__ part, int nblocks, double* __restrict__ out)
{
    __shared__ double ssum[kNormThreads];
    __shared__ double smax[kNormThreads];
    double s = 0.0, m = 0.0;
    for (int i = threadIdx.x; i < nblocks; i += kNormThreads) {
        s += part[2 * i];
        m = nan_max(m, part[2 * i + 1]);
    }
    ssum[threadIdx.x] = s;
    smax[threadIdx.x] = m;
    __syncthreads();
    for (int w = kNormThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            ssum[threadIdx.x] += ssum[threadIdx.x + w];
            smax[threadIdx.x] = nan_max(smax[threadIdx.x], smax[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = sqrt(ssum[0]);
        out[1] = smax[0];
    }
}

// Partials of the allocation-free entry point: one copy per device, held by
// the loaded library until the process ends (32 KiB).  Host code never uses
// this name as an address: it takes the device address once per device with
// hipGetSymbolAddress and passes that.
static __device__ __align__(256) double scratch[kNormPartials];

constexpr int kMaxDevices = 64;

// The buffer of norms_fp64, one per device, kept for the process.
static std::mutex g_norm_mu;
static double* g_norm_buf[kMaxDevices] = {nullptr};

// Device address of `scratch`, one per device, taken at the first use on
// that device with the device current.
static std::mutex g_static_mu;
static double* g_static_ptr[kMaxDevices] = {nullptr};

static hipError_t norm_buffer(int dev, double** out)
{
    if (!g_norm_buf[dev]) {
        hipError_t e = hipMalloc(&g_norm_buf[dev], sizeof(double) * (kNormPartials + 2));
        if (e != hipSuccess) {
            g_norm_buf[dev] = nullptr;
            return e;
        }
    }
    *out = g_norm_buf[dev];
    return hipSuccess;
}

static hipError_t static_scratch(double** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (!g_static_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_static_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_static_ptr[dev];
    return hipSuccess;
}

template <typename TA, typename TB>
static void launch_norm(const DevGrid& ga, const void* a, const DevGrid& gb, const void* b, bool diff,
                        int nblocks, double* part, hipStream_t stream)
{
    if (diff)
        hipLaunchKernelGGL((norm_partial_kernel<TA, TB, true>), dim3(nblocks), dim3(kNormThreads), 0,
                           stream, static_cast<const TA*>(a), static_cast<const TB*>(b), ga.nx, ga.ny,
                           ga.nz, ga.sy, ga.sz, gb.sy, gb.sz, part);
    else
        hipLaunchKernelGGL((norm_partial_kernel<TA, TB, false>), dim3(nblocks), dim3(kNormThreads), 0,
                           stream, static_cast<const TA*>(a), static_cast<const TB*>(b), ga.nx, ga.ny,
                           ga.nz, ga.sy, ga.sz, gb.sy, gb.sz, part);
}

// Both passes on `stream`: partials into part[0 .. 2 nblocks), the two
// results into out (device memory).  Every partial slot the final pass reads
// is written by this call's first pass, so nothing needs clearing.
static hipError_t norm_passes(const DevGrid& ga, const void* a, const DevGrid& gb, const void* b, int which,
                              double* part, double* out, hipStream_t stream)
{
    const long long rows = (long long)ga.ny * ga.nz;
    const int nblocks = (int)(rows < kNormMaxBlocks ? rows : kNormMaxBlocks);
    const bool diff = which != 0;
    const bool fa = ga.dtype == 0, fb = gb.dtype == 0;
    if (fa && fb) launch_norm<double, double>(ga, a, gb, b, diff, nblocks, part, stream);
    else if (fa && !fb) launch_norm<double, float>(ga, a, gb, b, diff, nblocks, part, stream);
    else if (!fa && fb) launch_norm<float, double>(ga, a, gb, b, diff, nblocks, part, stream);
    else launch_norm<float, float>(ga, a, gb, b, diff, nblocks, part, stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(norm_final_kernel, dim3(1), dim3(kNormThreads), 0, stream, part, nblocks, out);
    return hipGetLastError();
}

hipError_t norms_fp64(const DevGrid& ga, const void* a, const DevGrid& gb, const void* b, int which,
                      double out[2], hipStream_t stream)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    // one buffer per device: held from the first launch until the result is
    // on the host
    std::lock_guard<std::mutex> lk(g_norm_mu);
    double* buf = nullptr;
    e = norm_buffer(dev, &buf);
    if (e != hipSuccess) return e;
    e = norm_passes(ga, a, gb, b, which, buf, buf + kNormPartials, stream);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(out, buf + kNormPartials, 2 * sizeof(double), hipMemcpyDeviceToHost, stream);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(stream);
}

hipError_t norms_fp64_static(const DevGrid& ga, const void* a, const DevGrid& gb, const void* b, int which,
                             double* out_dev, hipStream_t stream)
{
    double* part = nullptr;
    hipError_t e = static_scratch(&part);
    if (e != hipSuccess) return e;
    return norm_passes(ga, a, gb, b, which, part, out_dev, stream);
}

}  // namespace mwd
