// Micro-benchmarks of the MI355X rates the tracing kernels are bound by:
// FP64 fused multiply-add issue, 32-bit multiply-high (the Philox rounds),
// FP64 exp (the attenuation and the spectrum), an HBM read stream, and FP64
// atomic adds against the number of distinct addresses they hit (the
// monitors).  Measurement only: nothing here takes part in tracing.  Each
// kernel's loops are bounded by its arguments; indices stay inside the
// caller's buffer (checked on the host).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "mxr.h"

namespace mxr_host {
mxr_status set_error(mxr_status st, const char *msg);
}

namespace {

constexpr int kPeakBlock = 256;

// eight independent FMA chains per lane; the sink keeps them alive
__global__ __launch_bounds__(kPeakBlock) void k_peak_fma(double *sink, uint64_t iters, double b, double c) {
    const uint64_t t = (uint64_t)blockIdx.x * kPeakBlock + threadIdx.x;
    double a0 = (double)t * 1e-9, a1 = a0 + 1.0, a2 = a0 + 2.0, a3 = a0 + 3.0;
    double a4 = a0 + 4.0, a5 = a0 + 5.0, a6 = a0 + 6.0, a7 = a0 + 7.0;
    for (uint64_t i = 0; i < iters; ++i) {
        a0 = fma(a0, b, c);
        a1 = fma(a1, b, c);
        a2 = fma(a2, b, c);
        a3 = fma(a3, b, c);
        a4 = fma(a4, b, c);
        a5 = fma(a5, b, c);
        a6 = fma(a6, b, c);
        a7 = fma(a7, b, c);
    }
    sink[t] = ((a0 + a1) + (a2 + a3)) + ((a4 + a5) + (a6 + a7));
}

// eight independent multiply-high chains per lane
__global__ __launch_bounds__(kPeakBlock) void k_peak_mulhi(double *sink, uint64_t iters, uint32_t k) {
    const uint32_t t = blockIdx.x * kPeakBlock + threadIdx.x;
    uint32_t x0 = t, x1 = t ^ 0x9E3779B9u, x2 = t + 7u, x3 = t * 3u, x4 = ~t, x5 = t ^ 0xBB67AE85u;
    uint32_t x6 = t + 13u, x7 = t * 5u;
    for (uint64_t i = 0; i < iters; ++i) {
        x0 = __umulhi(x0, k) ^ 0x1u;
        x1 = __umulhi(x1, k) ^ 0x2u;
        x2 = __umulhi(x2, k) ^ 0x3u;
        x3 = __umulhi(x3, k) ^ 0x4u;
        x4 = __umulhi(x4, k) ^ 0x5u;
        x5 = __umulhi(x5, k) ^ 0x6u;
        x6 = __umulhi(x6, k) ^ 0x7u;
        x7 = __umulhi(x7, k) ^ 0x8u;
    }
    sink[t] = (double)((x0 ^ x1) + (x2 ^ x3) + (x4 ^ x5) + (x6 ^ x7));
}

// four independent exp chains per lane (values stay in (0, 1])
__global__ __launch_bounds__(kPeakBlock) void k_peak_exp(double *sink, uint64_t iters) {
    const uint64_t t = (uint64_t)blockIdx.x * kPeakBlock + threadIdx.x;
    double x0 = 1e-3 * (double)(t & 1023u), x1 = x0 + 0.25, x2 = x0 + 0.5, x3 = x0 + 0.75;
    for (uint64_t i = 0; i < iters; ++i) {
        x0 = exp(-x0);
        x1 = exp(-x1);
        x2 = exp(-x2);
        x3 = exp(-x3);
    }
    sink[t] = (x0 + x1) + (x2 + x3);
}

// grid-stride read of n 16-byte elements, four loads in flight per lane;
// one partial sum per lane
__global__ __launch_bounds__(kPeakBlock) void k_peak_read(const double2 *__restrict__ src, uint64_t n, double *sink) {
    const uint64_t t = (uint64_t)blockIdx.x * kPeakBlock + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * kPeakBlock;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    uint64_t i = t;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const double2 v0 = src[i], v1 = src[i + stride], v2 = src[i + 2 * stride], v3 = src[i + 3 * stride];
        s0 += v0.x + v0.y;
        s1 += v1.x + v1.y;
        s2 += v2.x + v2.y;
        s3 += v3.x + v3.y;
    }
    for (; i < n; i += stride) {
        const double2 v = src[i];
        s0 += v.x + v.y;
    }
    sink[t] = (s0 + s1) + (s2 + s3);
}

// each lane adds 1.0 iters times, to address (lane hash + i) mod spread
__global__ __launch_bounds__(kPeakBlock) void k_peak_atomic(double *dst, uint64_t spread, uint64_t iters) {
    const uint64_t t = (uint64_t)blockIdx.x * kPeakBlock + threadIdx.x;
    const uint64_t h = (t * 0x9E3779B97F4A7C15ull) >> 17;
    for (uint64_t i = 0; i < iters; ++i) atomicAdd(dst + (h + i) % spread, 1.0);
}

}  // namespace

extern "C" mxr_status mxr_peak_launch(uint32_t kind, void *buf, uint64_t bytes, uint64_t spread, uint64_t iters,
                                      uint32_t groups, double *work, void *hip_stream) {
    if (!buf || !work) return mxr_host::set_error(MXR_E_INVALID, "null buffer or work pointer");
    if (groups < 1 || groups > (1u << 20)) return mxr_host::set_error(MXR_E_INVALID, "groups must be in [1, 2^20]");
    if (iters < 1 || iters > (1ull << 32)) return mxr_host::set_error(MXR_E_INVALID, "iters must be in [1, 2^32]");
    hipStream_t st = (hipStream_t)hip_stream;
    const uint64_t lanes = (uint64_t)groups * kPeakBlock;
    // every kernel but the read writes one double per lane (the sink) or
    // hits spread doubles of the buffer
    switch (kind) {
        case MXR_PEAK_FP64_FMA:
            if (bytes < lanes * sizeof(double)) return mxr_host::set_error(MXR_E_INVALID, "buffer below one double per lane");
            hipLaunchKernelGGL(k_peak_fma, dim3(groups), dim3(kPeakBlock), 0, st, (double *)buf, iters, 0.999999, 1e-7);
            *work = 2.0 * 8.0 * (double)iters * (double)lanes;
            break;
        case MXR_PEAK_U32_MULHI:
            if (bytes < lanes * sizeof(double)) return mxr_host::set_error(MXR_E_INVALID, "buffer below one double per lane");
            hipLaunchKernelGGL(k_peak_mulhi, dim3(groups), dim3(kPeakBlock), 0, st, (double *)buf, iters, 0xD2511F53u);
            *work = 8.0 * (double)iters * (double)lanes;
            break;
        case MXR_PEAK_FP64_EXP:
            if (bytes < lanes * sizeof(double)) return mxr_host::set_error(MXR_E_INVALID, "buffer below one double per lane");
            hipLaunchKernelGGL(k_peak_exp, dim3(groups), dim3(kPeakBlock), 0, st, (double *)buf, iters);
            *work = 4.0 * (double)iters * (double)lanes;
            break;
        case MXR_PEAK_READ: {
            // the first lanes * 8 bytes are the sink, the rest is read
            const uint64_t sink_bytes = (lanes * sizeof(double) + 255) & ~255ull;
            if (bytes < sink_bytes + 16) return mxr_host::set_error(MXR_E_INVALID, "buffer too small for the read");
            const uint64_t n = (bytes - sink_bytes) / 16;
            hipLaunchKernelGGL(k_peak_read, dim3(groups), dim3(kPeakBlock), 0, st,
                               (const double2 *)((char *)buf + sink_bytes), n, (double *)buf);
            *work = 16.0 * (double)n;
            break;
        }
        case MXR_PEAK_ATOMIC_F64:
            if (spread < 1 || spread > bytes / sizeof(double))
                return mxr_host::set_error(MXR_E_INVALID, "spread must be in [1, bytes / 8]");
            hipLaunchKernelGGL(k_peak_atomic, dim3(groups), dim3(kPeakBlock), 0, st, (double *)buf, spread, iters);
            *work = (double)iters * (double)lanes;
            break;
        default:
            return mxr_host::set_error(MXR_E_INVALID, "unknown peak kind");
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return mxr_host::set_error(MXR_E_HIP, hipGetErrorString(e));
    return MXR_OK;
}
