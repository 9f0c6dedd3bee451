// stats.hip -- per-bin statistics of replicated runs.
//
// The error of a Monte Carlo detector image is estimated by batch means:
// R independent replicas (runs on disjoint random streams) give R estimates
// I_rb = S_rb / n of each bin's intensity (S_rb the replica's summed
// weight, n its emitted rays); their mean is the image and their sample
// standard deviation over sqrt(R) its standard error.  Unlike the usual
// sqrt(sum w^2) estimate this stays valid for stratified sources and
// importance-weighted rays.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>

#include "mxr.h"

namespace mxr_host {
mxr_status set_error(mxr_status st, const char *msg);
}

namespace {

__global__ void k_batch_means(const double *sums, uint32_t R, uint64_t n_bins, double inv_n, double *mean,
                              double *rel) {
    for (uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; b < n_bins;
         b += (uint64_t)gridDim.x * blockDim.x) {
        double m = 0.0;
        for (uint32_t r = 0; r < R; ++r) m += sums[(uint64_t)r * n_bins + b] * inv_n;
        m /= (double)R;
        double ss = 0.0;
        for (uint32_t r = 0; r < R; ++r) {
            const double d = sums[(uint64_t)r * n_bins + b] * inv_n - m;
            ss += d * d;
        }
        mean[b] = m;
        rel[b] = m > 0.0 ? sqrt(ss / (double)(R - 1)) / (sqrt((double)R) * m) : INFINITY;
    }
}

}  // namespace

extern "C" mxr_status mxr_batch_means(const double *sums, uint32_t R, uint64_t n_bins, uint64_t rays_per_replica,
                                      double *mean, double *rel, void *hip_stream) {
    if (!sums || !mean || !rel) return mxr_host::set_error(MXR_E_INVALID, "null array");
    if (R < 2) return mxr_host::set_error(MXR_E_INVALID, "batch means need at least 2 replicas");
    if (rays_per_replica == 0) return mxr_host::set_error(MXR_E_INVALID, "replicas must trace rays");
    if (n_bins == 0) return MXR_OK;
    // grid-stride: at most 2^22 work-groups (the dispatch counts work-items
    // with 32 bits)
    const unsigned blocks = (unsigned)std::min<uint64_t>((n_bins + 255) / 256, 1ull << 22);
    hipLaunchKernelGGL(k_batch_means, dim3(blocks), dim3(256), 0, (hipStream_t)hip_stream, sums, R, n_bins,
                       1.0 / (double)rays_per_replica, mean, rel);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        char buf[256];
        snprintf(buf, sizeof buf, "batch means launch: %s", hipGetErrorString(e));
        return mxr_host::set_error(MXR_E_HIP, buf);
    }
    return MXR_OK;
}
