// mlp.hip -- the learned proposal's network on the matrix cores: a
// 6 -> 128 -> 128 -> 56 MLP (SiLU) in bfloat16 with float32 accumulation,
// the mixture head and its weighted negative log-likelihood in float32,
// split-K weight gradients, Adam with float32 master weights, training-data
// weights and the training loop.
//
// Every product of the network is a dense contraction, so it runs on MFMA:
// v_mfma_f32_16x16x16_bf16 with one wave per 16 x 16 output tile.  Operands
// are read from HBM / L2 through strides, so one kernel serves the forward
// products (activations x W), the input gradients (dZ x W^T) and the weight
// gradients (X^T x dZ, split over row chunks and reduced in a fixed order,
// so a gradient is deterministic).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "mxr.h"

namespace mxr_host {
mxr_status set_error(mxr_status st, const char *msg);
}

namespace {

constexpr int kIn = MXR_MLP_IN, kHid = MXR_MLP_HIDDEN, kOut = MXR_MLP_OUT;
constexpr uint64_t kW1 = 0, kB1 = kW1 + kIn * kHid, kW2 = kB1 + kHid, kB2 = kW2 + kHid * kHid;
constexpr uint64_t kW3 = kB2 + kHid, kB3 = kW3 + kHid * kOut, kParams = kB3 + kOut;
static_assert(kParams == MXR_MLP_PARAMS, "parameter layout");
constexpr uint64_t kSplitRows = 1024;  // rows per split of a weight-gradient product
constexpr int kThreads = 256;

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

mxr_status fail(mxr_status st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
mxr_status fail(mxr_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    return mxr_host::set_error(st, buf);
}

mxr_status launch_check(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(MXR_E_HIP, "%s: %s", what, hipGetErrorString(e));
    return MXR_OK;
}

// ------------------------------------------------------------ bfloat16 --

__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    uint32_t b = __float_as_uint(f);
    if ((b & 0x7F800000u) == 0x7F800000u) return (uint16_t)((b >> 16) | ((b & 0xFFFFu) ? 0x40u : 0u));  // inf/nan
    b += 0x7FFFu + ((b >> 16) & 1u);  // round to nearest, ties to even
    return (uint16_t)(b >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Hardware exponential, logarithm and reciprocal (v_exp_f32, v_log_f32,
// v_rcp_f32: about an ulp each; the argument scaling adds a few ulp): the
// activations they feed are rounded to bfloat16, and the head's float32 loss
// gradient is checked to 3e-4 of a row's scale, so the ten-instruction IEEE
// division and the full-range expf / logf buy nothing here.
__device__ __forceinline__ float fexp(float x) { return __builtin_amdgcn_exp2f(x * 1.4426950408889634f); }
__device__ __forceinline__ float flog(float x) { return __builtin_amdgcn_logf(x) * 0.6931471805599453f; }
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ __forceinline__ float silu(float z) { return z * frcp(1.0f + fexp(-z)); }

__device__ __forceinline__ float silu_grad(float z) {
    const float s = frcp(1.0f + fexp(-z));
    return s * (1.0f + z * (1.0f - s));
}

// ---------------------------------------------------------------- GEMM --

enum Epi { kEpiHidden = 0, kEpiOut, kEpiBackward };

struct GemmArgs {
    const uint16_t *A;  // A(m, k) = A[m * sam + k * sak]
    const uint16_t *B;  // B(k, n) = B[k * sbk + n * sbn]
    int64_t sam, sak, sbk, sbn;
    int64_t M, N, K;
    int64_t kchunk;        // split-K: contraction range per split (blockIdx.z)
    const uint16_t *bias;  // kEpiHidden / kEpiOut: bias[n] (bfloat16)
    float *Z;              // kEpiHidden: pre-activation out; kEpiBackward: pre-activation in
    uint16_t *H;           // kEpiHidden: silu(Z) out; kEpiBackward: dZ (bfloat16) out
    float *C;              // kEpiOut: output; kEpiBackward: dZ (float32) out; split-K: partial base
    int64_t ldc;           // row stride of C / Z / H
    int64_t split_stride;  // split-K: floats between the partials of consecutive splits
    float *colpart;        // strip kEpiBackward: per 16-row tile column sums of dZ (ldc columns)
};

// Split-K products (weight gradients: in x out, contracted over rows): one
// wave per 16 x 16 tile of C, four waves per work-group along M, the
// contraction split over blockIdx.z into chunks of kchunk rows, each split
// writing its own partial (reduced later in a fixed order).  The 16x16x16
// bf16 MFMA takes from lane l the row (A) or column (B) l mod 16 and the four
// consecutive k = 4 (l / 16) .. 4 (l / 16) + 3, and leaves in lane l the four
// outputs of rows 4 (l / 16) .. +3 in column l mod 16.
__global__ __launch_bounds__(kThreads) void k_gemm_splitk(GemmArgs g) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t tm = (int64_t)blockIdx.y * 4 + wave, tn = blockIdx.x;
    if (tm * 16 >= g.M) return;  // whole wave: no barrier in this kernel
    const int64_t k0 = (int64_t)blockIdx.z * g.kchunk;
    const int64_t k1 = std::min<int64_t>(k0 + g.kchunk, g.K);
    const int r = lane & 15, q = lane >> 4;
    const int64_t m = tm * 16 + r, n = tn * 16 + r;
    v4f acc = {0.f, 0.f, 0.f, 0.f};
    // four k-steps per iteration: their loads are in flight together (steps
    // past the end load zeros and add nothing)
    for (int64_t kb = k0; kb < k1; kb += 64) {
        v4s a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int64_t k = kb + 16 * u + 4 * q + j;
                a[u][j] = (m < g.M && k < k1) ? (short)g.A[m * g.sam + k * g.sak] : (short)0;
                b[u][j] = (n < g.N && k < k1) ? (short)g.B[k * g.sbk + n * g.sbn] : (short)0;
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[u], b[u], acc, 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t mm = tm * 16 + 4 * q + j, nn = tn * 16 + r;
        if (mm < g.M && nn < g.N) g.C[(int64_t)blockIdx.z * g.split_stride + mm * g.ldc + nn] = acc[j];
    }
}

// Row-heavy products (n rows x at most 128 columns): one wave per 16-row
// strip and all NT column tiles, so a k-step's A fragment is loaded once for
// NT MFMAs.  AVEC / BVEC: the operand's four consecutive k of a lane are
// contiguous and 8-byte aligned (unit k stride, row stride a multiple of 4),
// read as one 8-byte load; otherwise element loads.
template <int EPI, int NT, bool AVEC, bool BVEC>
__global__ __launch_bounds__(kThreads) void k_gemm_strip(GemmArgs g) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t tm = (int64_t)blockIdx.x * 4 + wave;
    if (tm * 16 >= g.M) return;  // whole wave: no barrier in this kernel
    const int r = lane & 15, q = lane >> 4;
    const int64_t m = tm * 16 + r;
    v4f acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
    for (int64_t kb = 0; kb < g.K; kb += 16) {
        const int64_t k = kb + 4 * q;
        v4s a;
        if (AVEC && m < g.M && k + 3 < g.K) {
            a = *(const v4s *)(g.A + m * g.sam + k);
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                a[j] = (m < g.M && k + j < g.K) ? (short)g.A[m * g.sam + (k + j) * g.sak] : (short)0;
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int64_t n = (int64_t)t * 16 + r;
            v4s b;
            if (BVEC && n < g.N && k + 3 < g.K) {
                b = *(const v4s *)(g.B + n * g.sbn + k);
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    b[j] = (n < g.N && k + j < g.K) ? (short)g.B[(k + j) * g.sbk + n * g.sbn] : (short)0;
            }
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[t], 0, 0, 0);
        }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        float cs = 0.f;  // kEpiBackward: this lane's 4 rows of column t*16 + r
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t mm = tm * 16 + 4 * q + j, nn = (int64_t)t * 16 + r;
            if (mm >= g.M || nn >= g.N) continue;
            const float v = acc[t][j];
            if constexpr (EPI == kEpiHidden) {
                const float z = v + bf16_to_f32(g.bias[nn]);
                g.Z[mm * g.ldc + nn] = z;
                g.H[mm * g.ldc + nn] = f32_to_bf16(silu(z));
            } else if constexpr (EPI == kEpiOut) {
                g.C[mm * g.ldc + nn] = v + bf16_to_f32(g.bias[nn]);
            } else {
                const float dz = v * silu_grad(g.Z[mm * g.ldc + nn]);
                g.C[mm * g.ldc + nn] = dz;
                g.H[mm * g.ldc + nn] = f32_to_bf16(dz);
                cs += dz;
            }
        }
        if constexpr (EPI == kEpiBackward) {
            // the tile's 16 rows: the four row groups of lanes r, r+16, r+32, r+48
            cs += __shfl_xor(cs, 16, 64);
            cs += __shfl_xor(cs, 32, 64);
            const int64_t nn = (int64_t)t * 16 + r;
            if (q == 0 && nn < g.N) g.colpart[tm * g.ldc + nn] = cs;
        }
    }
}

// Bias gradients from per-part column sums: the partial of split z is the
// sum of parts [z pps, (z+1) pps) of a column.  One launch serves the three
// bias vectors (blockIdx.z); a work-group takes 32 columns of one split, its
// 8 sub-lanes per column sum every 8th part, and the 8 sub-sums are added
// in a fixed order (deterministic).
struct ColReduce {
    const float *parts[3];
    int64_t n_parts[3], cols[3], pps[3], off[3];
    int64_t splits;
    float *partial;
};

__global__ __launch_bounds__(256) void k_colpart_reduce(ColReduce a) {
    __shared__ float red[8][32];
    const int b = blockIdx.z;
    const int64_t cols = a.cols[b], pps = a.pps[b], n_parts = a.n_parts[b];
    const int sub = threadIdx.x >> 5, cl = threadIdx.x & 31;
    const int64_t c = (int64_t)blockIdx.x * 32 + cl, z = blockIdx.y;
    float acc = 0.f;
    if (c < cols) {
        const int64_t p1 = std::min<int64_t>((z + 1) * pps, n_parts);
        for (int64_t p = z * pps + sub; p < p1; p += 8) acc += a.parts[b][p * cols + c];
    }
    red[sub][cl] = acc;
    __syncthreads();
    if (sub == 0 && c < cols) {
        float sum = 0.f;
        for (int u = 0; u < 8; ++u) sum += red[u][cl];
        a.partial[z * (int64_t)kParams + a.off[b] + c] = sum;
    }
}

bool vec_ok(const uint16_t *p, int64_t s_k, int64_t s_row) {
    return s_k == 1 && s_row % 4 == 0 && ((uintptr_t)p & 7) == 0;
}

// strip product with N <= 128 (8 tiles) or N <= 64 (4 tiles)
template <int EPI>
mxr_status gemm_strip(const GemmArgs &g, hipStream_t st) {
    if (g.M == 0 || g.N == 0) return MXR_OK;
    const bool av = vec_ok(g.A, g.sak, g.sam), bv = vec_ok(g.B, g.sbk, g.sbn);
    const dim3 grid((unsigned)((g.M + 63) / 64));
    if (g.N <= 64) {
        if (av && bv) hipLaunchKernelGGL((k_gemm_strip<EPI, 4, true, true>), grid, dim3(kThreads), 0, st, g);
        else hipLaunchKernelGGL((k_gemm_strip<EPI, 4, false, false>), grid, dim3(kThreads), 0, st, g);
    } else {
        if (av && bv) hipLaunchKernelGGL((k_gemm_strip<EPI, 8, true, true>), grid, dim3(kThreads), 0, st, g);
        else hipLaunchKernelGGL((k_gemm_strip<EPI, 8, false, false>), grid, dim3(kThreads), 0, st, g);
    }
    return launch_check("MLP strip product");
}

// W^T copies of the three weight matrices (out x in, row-major), for the
// forward products' unit-stride B operand.
__global__ void k_transpose_weights(const uint16_t *w, uint16_t *wt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kIn * kHid) {  // W1: in 6 x out 128
        const int a = i / kHid, b = i % kHid;
        wt[kW1 + b * kIn + a] = w[kW1 + i];
    }
    if (i < kHid * kHid) {
        const int a = i / kHid, b = i % kHid;
        wt[kW2 + b * kHid + a] = w[kW2 + i];
    }
    if (i < kHid * kOut) {
        const int a = i / kOut, b = i % kOut;
        wt[kW3 + b * kHid + a] = w[kW3 + i];
    }
}

mxr_status gemm_splitk(const GemmArgs &g, int64_t splits, hipStream_t st) {
    if (g.M == 0 || g.N == 0) return MXR_OK;
    const dim3 grid((unsigned)((g.N + 15) / 16), (unsigned)((g.M + 63) / 64), (unsigned)splits);
    hipLaunchKernelGGL(k_gemm_splitk, grid, dim3(kThreads), 0, st, g);
    return launch_check("MLP split-K product");
}

// ------------------------------------------------------ small kernels --

// Rows of a batch: row i of the batch is dataset row (a i + b) mod n_data
// (a coprime to n_data: a bijection, a cheap shuffle per epoch; a, b and
// the row index below n_data < 2^32); the identity is a = 1, b = 0.  Contexts go to bfloat16, targets and weights
// are copied.
__global__ void k_gather(const float *ctx, const double *y, const double *omega, uint64_t n_data, uint64_t a,
                         uint64_t b, uint64_t first, uint64_t n, uint16_t *X, double *Yb, double *Wb) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t src = ((a * (first + i)) % n_data + b) % n_data;  // n_data < 2^32: no overflow
        for (int j = 0; j < kIn; ++j) X[i * kIn + j] = f32_to_bf16(ctx[src * kIn + j]);
        if (Yb) {
            for (int j = 0; j < 3; ++j) Yb[i * 3 + j] = y[src * 3 + j];
            Wb[i] = omega[src];
        }
    }
}

// Deterministic sums: each work-group sums its stride of the input into one
// partial; a second launch with one work-group sums the partials in order.
__global__ void k_sum_f64(const double *x, uint64_t n, double *partial) {
    __shared__ double red[kThreads];
    double s = 0.0;
    for (uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kThreads)
        s += x[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

constexpr unsigned kSumBlocks = 256;

mxr_status sum_f64(const double *x, uint64_t n, double *scratch, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_sum_f64, dim3(kSumBlocks), dim3(kThreads), 0, st, x, n, scratch);
    hipLaunchKernelGGL(k_sum_f64, dim3(1), dim3(kThreads), 0, st, (const double *)scratch, (uint64_t)kSumBlocks, out);
    return launch_check("sum");
}

// The mixture head and the weighted negative log-likelihood of one row per
// thread, in float32.  Head: pi = softmax(logits), mu = centre + half tanh,
// sigma = half (1e-3 + softplus).  -log q = -logsumexp_k(log pi_k +
// sum_d log N(y_d; mu, sigma)) + log sum_k pi_k Z_k.  Writes dL/do scaled by
// a_i = omega_i / sum omega (float32 and bfloat16) and a_i (-log q_i).
struct HeadArgs {
    const float *O;  // n x 56
    const double *Y;
    const double *W;
    const double *wsum;
    uint64_t n;
    float lo[3], hi[3];
    float *dO;
    uint16_t *dOh;
    double *row_loss;
    float *colpart;  // per wave (8 rows) column sums of dO, 56 per wave
};

__device__ __forceinline__ float phi_pdf(float z) { return 0.3989422804014327f * fexp(-0.5f * z * z); }

// mass of a standard normal in [za, zb], from the side that does not cancel
__device__ __forceinline__ float box_mass(float za, float zb) {
    if (za > 0.f) return 0.5f * (erfcf(za * 0.70710678f) - erfcf(zb * 0.70710678f));
    if (zb < 0.f) return 0.5f * (erfcf(-zb * 0.70710678f) - erfcf(-za * 0.70710678f));
    return 1.0f - 0.5f * (erfcf(-za * 0.70710678f) + erfcf(zb * 0.70710678f));
}

// Eight lanes per row, lane k of the group holding mixture component k;
// row-level maxima and sums are butterflies over the group (xor 1, 2, 4).
__device__ __forceinline__ float group8_max(float v) {
    v = fmaxf(v, __shfl_xor(v, 1, 64));
    v = fmaxf(v, __shfl_xor(v, 2, 64));
    return fmaxf(v, __shfl_xor(v, 4, 64));
}
__device__ __forceinline__ float group8_sum(float v) {
    v += __shfl_xor(v, 1, 64);
    v += __shfl_xor(v, 2, 64);
    return v + __shfl_xor(v, 4, 64);
}

// The head and loss gradient of one row, component k = this lane's index in
// its group of eight (the eight lanes of a row are consecutive and take part
// together).  o: the row's 56 outputs; y: its target; a: its loss weight
// omega_i / sum omega.  g: dL/do of component k's seven outputs, scaled by a;
// loss: a (-log q) of the row (every lane of the group).
__device__ __forceinline__ void head_row(const float *o_row, const double *y_row, float a, const float lo[3],
                                         const float hi[3], int k, float g[7], float &loss) {
    const float *o = o_row + 7 * k;
    const float lg = o[0];
    const float mx = group8_max(lg);
    const float lse_logit = mx + flog(group8_sum(fexp(lg - mx)));
    const float pi = fexp(lg - lse_logit);
    float c = lg - lse_logit, zk = 1.f;
    float t[3], sg[3], z[3], za[3], zb[3], F[3], raw_s[3];
    for (int d = 0; d < 3; ++d) {
        const float cen = 0.5f * (lo[d] + hi[d]), half = 0.5f * (hi[d] - lo[d]);
        t[d] = tanhf(o[1 + d]);
        const float mu = cen + half * t[d];
        raw_s[d] = o[4 + d];
        const float sp = raw_s[d] > 20.f ? raw_s[d] : log1pf(fexp(raw_s[d]));
        sg[d] = half * (1e-3f + sp);
        const float is = frcp(sg[d]);
        z[d] = ((float)y_row[d] - mu) * is;
        za[d] = (lo[d] - mu) * is;
        zb[d] = (hi[d] - mu) * is;
        F[d] = box_mass(za[d], zb[d]);
        c += -0.5f * z[d] * z[d] - flog(sg[d]) - 0.91893853f;
        zk *= F[d];
    }
    const float cmax = group8_max(c);
    const float lse = cmax + flog(group8_sum(fexp(c - cmax)));
    const float S = group8_sum(pi * zk);
    loss = a * (flog(S) - lse);
    const float r = fexp(c - lse);
    const float s = pi * zk * frcp(S);
    g[0] = a * (s - r);
    for (int d = 0; d < 3; ++d) {
        const float half = 0.5f * (hi[d] - lo[d]);
        const float pa = phi_pdf(za[d]), pb = phi_pdf(zb[d]);
        const float is = frcp(sg[d]), iF = frcp(F[d]);
        const float dF_mu = -(pb - pa) * is;
        const float dF_sg = -(zb[d] * pb - za[d] * pa) * is;
        const float g_mu = -r * z[d] * is + s * dF_mu * iF;
        const float g_sg = -r * (z[d] * z[d] - 1.f) * is + s * dF_sg * iF;
        g[1 + d] = a * (g_mu * half * (1.f - t[d] * t[d]));
        g[4 + d] = a * (g_sg * half * frcp(1.f + fexp(-raw_s[d])));
    }
}

__global__ __launch_bounds__(kThreads) void k_head_loss_grad(HeadArgs h) {
    const uint64_t gt = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    const uint64_t gi = gt >> 3;
    const int k = (int)(gt & 7);
    const bool live = gi < h.n;
    const uint64_t i = live ? gi : 0;  // groups past the end compute row 0 with weight 0
    const float a = live ? (float)(h.W[i] / *h.wsum) : 0.f;
    float g[7], loss;
    head_row(h.O + i * kOut, h.Y + i * 3, a, h.lo, h.hi, k, g, loss);
    if (live && k == 0) h.row_loss[i] = (double)loss;
    const uint64_t wave = gt >> 6;  // 8 rows per wave
    const bool writer = (threadIdx.x & 63) < 8 && (wave << 3) < h.n;
    for (int j = 0; j < 7; ++j) {
        const float v = g[j];
        if (live) {
            h.dO[i * kOut + 7 * k + j] = v;
            h.dOh[i * kOut + 7 * k + j] = f32_to_bf16(v);
        }
        // the wave's 8 rows of this column: lanes k, k + 8, ..., k + 56
        float cs = v;
        cs += __shfl_xor(cs, 8, 64);
        cs += __shfl_xor(cs, 16, 64);
        cs += __shfl_xor(cs, 32, 64);
        if (writer) h.colpart[wave * kOut + 7 * k + j] = cs;
    }
}

// Mixture tables for the tracer from head outputs: per row and component
// (pi, mu_u, mu_v, mu_E, sigma_u, sigma_v, sigma_E), computed in float32
// like the training head and stored as float64.
__global__ void k_head_params(const float *O, uint64_t n, float lo0, float lo1, float lo2, float hi0, float hi1,
                              float hi2, double *gmm) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const float lo[3] = {lo0, lo1, lo2}, hi[3] = {hi0, hi1, hi2};
        const float *o = O + i * kOut;
        float mx = -INFINITY;
        for (int k = 0; k < 8; ++k) mx = fmaxf(mx, o[7 * k]);
        float se = 0.f;
        for (int k = 0; k < 8; ++k) se += expf(o[7 * k] - mx);
        const float lse = mx + logf(se);
        for (int k = 0; k < 8; ++k) {
            double *g = gmm + i * kOut + 7 * k;
            g[0] = (double)expf(o[7 * k] - lse);
            for (int d = 0; d < 3; ++d) {
                const float cen = 0.5f * (lo[d] + hi[d]), half = 0.5f * (hi[d] - lo[d]);
                const float raw = o[7 * k + 4 + d];
                const float sp = raw > 20.f ? raw : log1pf(expf(raw));
                g[1 + d] = (double)(cen + half * tanhf(o[7 * k + 1 + d]));
                g[4 + d] = (double)(half * (1e-3f + sp));
            }
        }
    }
}

// gradient[p] = sum over splits, in split order
__global__ void k_reduce_partials(const float *partial, int64_t splits, float *grad) {
    const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kParams) return;
    float s = 0.f;
    for (int64_t z = 0; z < splits; ++z) s += partial[z * (int64_t)kParams + p];
    grad[p] = s;
}

__global__ void k_adam(float *theta, uint16_t *wb, const float *g, float *m, float *v, uint64_t n, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float t = theta[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
        theta[i] = t;
        wb[i] = f32_to_bf16(t);
    }
}

__global__ void k_to_bf16(const float *x, uint64_t n, uint16_t *y) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        y[i] = f32_to_bf16(x[i]);
}

// ----------------------------------------------- fused training step --
// One launch computes a whole Adam step's gradient: work-group g takes the
// 32-row strips g, g + G, g + 2G, ... of the batch and, per strip, gathers
// its rows, runs the three layers forward, the head and its loss gradient,
// and the backward products, with the bfloat16 weights staged once in LDS
// and every layer value of the strip in LDS (nothing but the rows goes to
// or comes from memory).  The weight gradients accumulate across the
// group's strips in the MFMA accumulators; the group then writes one
// partial gradient, and k_fused_reduce_adam sums the G partials in order
// (deterministic) and takes the Adam step.  The products, operands and
// roundings are those of the layer-by-layer path (bf16 operands, f32
// accumulation, f32 pre-activations, bf16 copies of activations and
// gradients), only the order of the float32 sums differs.
constexpr int kStripRows = 32;
static_assert(kStripRows % 32 == 0, "weight-gradient products take K = 32 rows per instruction");
constexpr int kFusedGroups = 256;

struct FusedArgs {
    const float *ctx;
    const double *y, *omega;
    uint64_t n_data, a, b, first, cnt;  // batch row i = data row (a (first + i) mod n_data + b) mod n_data
    const double *wsum;                 // sum of the batch's omega
    const uint16_t *w;                  // bfloat16 parameters
    float lo[3], hi[3];
    float *part;                        // gridDim.x x kParams partial gradients
    double *loss_part;                  // gridDim.x partial losses
};

__device__ __forceinline__ v4s frag_c(const uint16_t *p) { return *(const v4s *)p; }
__device__ __forceinline__ v4s frag_s(const uint16_t *p, int stride) {
    v4s r;
    r[0] = (short)p[0];
    r[1] = (short)p[stride];
    r[2] = (short)p[2 * stride];
    r[3] = (short)p[3 * stride];
    return r;
}
__device__ __forceinline__ v4f mfma16(v4s a, v4s b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// gfx950's 16 x 16 x 32 bfloat16 product (twice the K of one instruction):
// lane l holds row (A) or column (B) l % 16 and eight values of k, the same
// eight for A and B (here k = 8 (l / 16) + j); the accumulator layout is the
// 16 x 16 x 16 product's.
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
__device__ __forceinline__ v8bf frag8_c(const uint16_t *p) { return __builtin_bit_cast(v8bf, *(const uint4 *)p); }
__device__ __forceinline__ v8bf frag8_s(const uint16_t *p, int stride) {
    uint4 u;
    u.x = (uint32_t)p[0] | ((uint32_t)p[stride] << 16);
    u.y = (uint32_t)p[2 * stride] | ((uint32_t)p[3 * stride] << 16);
    u.z = (uint32_t)p[4 * stride] | ((uint32_t)p[5 * stride] << 16);
    u.w = (uint32_t)p[6 * stride] | ((uint32_t)p[7 * stride] << 16);
    return __builtin_bit_cast(v8bf, u);
}
__device__ __forceinline__ v4f mfma32(v8bf a, v8bf b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

constexpr int kFusedThreads = 512;  // eight waves: two per SIMD

__global__ __launch_bounds__(kFusedThreads, 1) void k_train_fused(FusedArgs f) {
    constexpr int R = kStripRows, H = kHid, O64 = 64, X16 = 16;
    __shared__ __attribute__((aligned(16))) uint16_t sW1t[H * X16];  // W1 transposed (out x in), in >= 6 zero
    __shared__ __attribute__((aligned(16))) uint16_t sW2[H * H];     // W2 (in x out)
    __shared__ __attribute__((aligned(16))) uint16_t sW3[H * O64];   // W3 (in x out), out >= 56 zero
    __shared__ __attribute__((aligned(16))) float sB1[H], sB2[H], sB3[O64];
    __shared__ __attribute__((aligned(16))) uint16_t sX[R * X16];
    __shared__ __attribute__((aligned(16))) double sY[R * 3];
    __shared__ __attribute__((aligned(16))) float sA[R];
    __shared__ __attribute__((aligned(16))) float sZ1[R * H];  // pre-activations of layer 1
    __shared__ __attribute__((aligned(16))) uint16_t sH1[R * H];
    __shared__ __attribute__((aligned(16))) float sZ2[R * H];  // layer 2; then dZ1 (bf16) in its first half
    __shared__ __attribute__((aligned(16))) uint16_t sH2[R * H];
    __shared__ __attribute__((aligned(16))) float sO[R * O64];  // outputs; then dZ2 (bf16 R x H) in the same bytes
    __shared__ __attribute__((aligned(16))) uint16_t sdO[R * O64];
    __shared__ __attribute__((aligned(16))) uint64_t sSrc[R];
    __shared__ __attribute__((aligned(16))) float sRed[4 * 64];
    __shared__ __attribute__((aligned(16))) double sLoss[kFusedThreads];
    uint16_t *sdZ2 = (uint16_t *)sO;
    uint16_t *sdZ1 = (uint16_t *)sZ2;

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, r = lane & 15, q = lane >> 4;
    // weights and biases, once
    for (int i = tid; i < H * X16; i += kFusedThreads) {
        const int n = i / X16, k = i % X16;
        sW1t[i] = k < kIn ? f.w[kW1 + k * H + n] : (uint16_t)0;
    }
    for (int i = tid; i < H * H; i += kFusedThreads) sW2[i] = f.w[kW2 + i];
    for (int i = tid; i < H * O64; i += kFusedThreads) {
        const int k = i / O64, n = i % O64;
        sW3[i] = n < kOut ? f.w[kW3 + k * kOut + n] : (uint16_t)0;
    }
    for (int i = tid; i < H; i += kFusedThreads) {
        sB1[i] = bf16_to_f32(f.w[kB1 + i]);
        sB2[i] = bf16_to_f32(f.w[kB2 + i]);
    }
    for (int i = tid; i < O64; i += kFusedThreads) sB3[i] = i < kOut ? bf16_to_f32(f.w[kB3 + i]) : 0.f;
    for (int i = tid; i < R * O64; i += kFusedThreads) sdO[i] = 0;  // columns >= 56 stay zero
    const double wsum = *f.wsum;
    // wave w owns column tile w of the row-strip products and row tile w of
    // the weight-gradient products
    v4f acc1 = {0.f, 0.f, 0.f, 0.f}, acc2[8], acc3[4];
    for (int t = 0; t < 8; ++t) acc2[t] = v4f{0.f, 0.f, 0.f, 0.f};
    for (int t = 0; t < 4; ++t) acc3[t] = v4f{0.f, 0.f, 0.f, 0.f};
    float db1 = 0.f, db2 = 0.f, db3[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    double loss_acc = 0.0;
    const uint64_t n_strips = (f.cnt + R - 1) / R;
    const int nt = wave;
    __syncthreads();

    for (uint64_t strip = blockIdx.x; strip < n_strips; strip += gridDim.x) {
        // rows of the strip (rows past the batch repeat its first row with
        // weight 0): their data rows, then one element per thread
        if (tid < R) {
            const uint64_t i = strip * R + tid;
            const bool live = i < f.cnt;
            sSrc[tid] = ((f.a * (f.first + (live ? i : 0))) % f.n_data + f.b) % f.n_data;
        }
        __syncthreads();
        for (int e = tid; e < R * 10; e += kFusedThreads) {
            const int row = e / 10, item = e % 10;
            const uint64_t src = sSrc[row];
            if (item < kIn) sX[row * X16 + item] = f32_to_bf16(f.ctx[src * kIn + item]);
            else if (item < kIn + 3) sY[row * 3 + item - kIn] = f.y[src * 3 + item - kIn];
            else sA[row] = (strip * R + row < f.cnt) ? (float)(f.omega[src] / wsum) : 0.f;
        }
        for (int e = tid; e < R * (X16 - kIn); e += kFusedThreads)
            sX[(e / (X16 - kIn)) * X16 + kIn + e % (X16 - kIn)] = 0;
        __syncthreads();
        // layer 1: Z1 = X W1 + b1 (K = 6, padded to 16)
        {
            const v4s b = frag_c(sW1t + (nt * 16 + r) * X16 + 4 * q);
            v4f c[2];
            for (int mt = 0; mt < 2; ++mt)
                c[mt] = mfma16(frag_c(sX + (mt * 16 + r) * X16 + 4 * q), b, v4f{0.f, 0.f, 0.f, 0.f});
            for (int mt = 0; mt < 2; ++mt)
                for (int j = 0; j < 4; ++j) {
                    const int m = mt * 16 + 4 * q + j, n = nt * 16 + r;
                    const float z = c[mt][j] + sB1[n];
                    sZ1[m * H + n] = z;
                    sH1[m * H + n] = f32_to_bf16(silu(z));
                }
        }
        __syncthreads();
        // layer 2: Z2 = H1 W2 + b2 (the two row tiles' chains interleaved)
        {
            v4f c[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
#pragma unroll
            for (int k0 = 0; k0 < H; k0 += 32) {
                const v8bf b = frag8_s(sW2 + (k0 + 8 * q) * H + nt * 16 + r, H);
                c[0] = mfma32(frag8_c(sH1 + r * H + k0 + 8 * q), b, c[0]);
                c[1] = mfma32(frag8_c(sH1 + (16 + r) * H + k0 + 8 * q), b, c[1]);
            }
            for (int mt = 0; mt < 2; ++mt)
                for (int j = 0; j < 4; ++j) {
                    const int m = mt * 16 + 4 * q + j, n = nt * 16 + r;
                    const float z = c[mt][j] + sB2[n];
                    sZ2[m * H + n] = z;
                    sH2[m * H + n] = f32_to_bf16(silu(z));
                }
        }
        __syncthreads();
        // layer 3: O = H2 W3 + b3 (outputs 56..63 are zero): 8 tiles, one per wave
        {
            const int mt = wave >> 2, ot = wave & 3;
            v4f c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int k0 = 0; k0 < H; k0 += 32)
                c = mfma32(frag8_c(sH2 + (mt * 16 + r) * H + k0 + 8 * q),
                           frag8_s(sW3 + (k0 + 8 * q) * O64 + ot * 16 + r, O64), c);
            for (int j = 0; j < 4; ++j) {
                const int m = mt * 16 + 4 * q + j, n = ot * 16 + r;
                sO[m * O64 + n] = c[j] + sB3[n];
            }
        }
        __syncthreads();
        // head: eight lanes per row (lane k = component k), waves 0-3
        if (tid < R * 8) {
            const int i = tid >> 3, k = tid & 7;
            float g[7], loss;
            head_row(sO + i * O64, sY + i * 3, sA[i], f.lo, f.hi, k, g, loss);
            if (k == 0) loss_acc += (double)loss;
            for (int j = 0; j < 7; ++j) {
                sdO[i * O64 + 7 * k + j] = f32_to_bf16(g[j]);
                // this wave's 8 rows of the column: lanes k, k + 8, ..., k + 56
                float cs = g[j];
                cs += __shfl_xor(cs, 8, 64);
                cs += __shfl_xor(cs, 16, 64);
                cs += __shfl_xor(cs, 32, 64);
                db3[j] += cs;
            }
        }
        __syncthreads();
        // dZ2 = (dO W3^T) * silu'(Z2), its column sums (bias 2)
        {
            v4f c[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
#pragma unroll
            for (int k0 = 0; k0 < O64; k0 += 32) {
                const v8bf b = frag8_c(sW3 + (nt * 16 + r) * O64 + k0 + 8 * q);
                c[0] = mfma32(frag8_c(sdO + r * O64 + k0 + 8 * q), b, c[0]);
                c[1] = mfma32(frag8_c(sdO + (16 + r) * O64 + k0 + 8 * q), b, c[1]);
            }
            float cs = 0.f;
            for (int mt = 0; mt < 2; ++mt)
                for (int j = 0; j < 4; ++j) {
                    const int m = mt * 16 + 4 * q + j, n = nt * 16 + r;
                    const float dz = c[mt][j] * silu_grad(sZ2[m * H + n]);
                    cs += dz;
                    sdZ2[m * H + n] = f32_to_bf16(dz);
                }
            cs += __shfl_xor(cs, 16, 64);
            cs += __shfl_xor(cs, 32, 64);
            db2 += cs;
        }
        __syncthreads();
        // dW3 += H2^T dO (in x out over the strip's rows): row tile = wave
        {
            const int mt = wave;
#pragma unroll
            for (int k0 = 0; k0 < R; k0 += 32) {
                const v8bf a = frag8_s(sH2 + (k0 + 8 * q) * H + mt * 16 + r, H);
#pragma unroll
                for (int ot = 0; ot < 4; ++ot)
                    acc3[ot] = mfma32(a, frag8_s(sdO + (k0 + 8 * q) * O64 + ot * 16 + r, O64), acc3[ot]);
            }
        }
        // dZ1 = (dZ2 W2^T) * silu'(Z1), its column sums (bias 1); Z2 is no
        // longer read, its bytes take dZ1
        {
            v4f c[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
#pragma unroll
            for (int k0 = 0; k0 < H; k0 += 32) {
                const v8bf b = frag8_c(sW2 + (nt * 16 + r) * H + k0 + 8 * q);
                c[0] = mfma32(frag8_c(sdZ2 + r * H + k0 + 8 * q), b, c[0]);
                c[1] = mfma32(frag8_c(sdZ2 + (16 + r) * H + k0 + 8 * q), b, c[1]);
            }
            float cs = 0.f;
            for (int mt = 0; mt < 2; ++mt)
                for (int j = 0; j < 4; ++j) {
                    const int m = mt * 16 + 4 * q + j, n = nt * 16 + r;
                    const float dz = c[mt][j] * silu_grad(sZ1[m * H + n]);
                    cs += dz;
                    sdZ1[m * H + n] = f32_to_bf16(dz);
                }
            cs += __shfl_xor(cs, 16, 64);
            cs += __shfl_xor(cs, 32, 64);
            db1 += cs;
        }
        __syncthreads();
        // dW2 += H1^T dZ2 (row tile = wave), dW1 += X^T dZ1 (column tile = wave)
        {
            const int mt = wave;
#pragma unroll
            for (int k0 = 0; k0 < R; k0 += 32) {
                const v8bf a = frag8_s(sH1 + (k0 + 8 * q) * H + mt * 16 + r, H);
#pragma unroll
                for (int t = 0; t < 8; ++t)
                    acc2[t] = mfma32(a, frag8_s(sdZ2 + (k0 + 8 * q) * H + t * 16 + r, H), acc2[t]);
                acc1 = mfma32(frag8_s(sX + (k0 + 8 * q) * X16 + r, X16),
                              frag8_s(sdZ1 + (k0 + 8 * q) * H + nt * 16 + r, H), acc1);
            }
        }
        __syncthreads();
    }

    // the group's partial gradient, in the parameter layout
    float *P = f.part + (uint64_t)blockIdx.x * kParams;
    {
        const int mt = wave;
        for (int t = 0; t < 8; ++t)
            for (int j = 0; j < 4; ++j) P[kW2 + (mt * 16 + 4 * q + j) * H + t * 16 + r] = acc2[t][j];
        for (int ot = 0; ot < 4; ++ot)
            for (int j = 0; j < 4; ++j) {
                const int n = ot * 16 + r;
                if (n < kOut) P[kW3 + (mt * 16 + 4 * q + j) * kOut + n] = acc3[ot][j];
            }
        for (int j = 0; j < 4; ++j) {
            const int m = 4 * q + j;
            if (m < kIn) P[kW1 + m * H + nt * 16 + r] = acc1[j];
        }
        if (q == 0) {
            P[kB1 + nt * 16 + r] = db1;
            P[kB2 + nt * 16 + r] = db2;
        }
    }
    // bias 3: lanes 0..7 of waves 0-3 hold their waves' column sums
    if (wave < 4 && lane < 8)
        for (int j = 0; j < 7; ++j) sRed[wave * 64 + 7 * lane + j] = db3[j];
    sLoss[tid] = loss_acc;
    __syncthreads();
    if (tid < kOut) P[kB3 + tid] = ((sRed[tid] + sRed[64 + tid]) + sRed[128 + tid]) + sRed[192 + tid];
    if (tid == 0) {
        double s = 0.0;
        for (int i = 0; i < kFusedThreads; ++i) s += sLoss[i];
        f.loss_part[blockIdx.x] = s;
    }
}

// Sum of the batch's omega over the shuffled rows (the gathered order of the
// layer-by-layer path; each work-group sums its stride into one partial).
__global__ void k_batch_wsum(const double *omega, uint64_t n_data, uint64_t a, uint64_t b, uint64_t first,
                             uint64_t cnt, double *partial) {
    __shared__ double red[kThreads];
    double s = 0.0;
    for (uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x; i < cnt; i += (uint64_t)gridDim.x * kThreads)
        s += omega[((a * (first + i)) % n_data + b) % n_data];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// gradient = the groups' partials summed in a fixed order (eight threads
// per parameter each sum every eighth group, then their eight sums in
// order), then one Adam step; the loss (nullable) = the partial losses
// summed in order
constexpr int kReduceParams = 32;  // parameters per work-group of 256 threads

__global__ __launch_bounds__(256) void k_fused_reduce_adam(const float *part, int groups, float *grad, float *theta,
                                                           uint16_t *wb, float *m, float *v, float lr, float b1,
                                                           float b2, float eps, float c1, float c2,
                                                           const double *loss_part, double *loss) {
    __shared__ float red[8][kReduceParams];
    const int sub = threadIdx.x >> 5, c = threadIdx.x & 31;
    const uint64_t p = (uint64_t)blockIdx.x * kReduceParams + c;
    if (loss && blockIdx.x == 0 && threadIdx.x == 0) {
        double s = 0.0;
        for (int g = 0; g < groups; ++g) s += loss_part[g];
        *loss = s;
    }
    float acc = 0.f;
    if (p < kParams)
        for (int g = sub; g < groups; g += 8) acc += part[(uint64_t)g * kParams + p];
    red[sub][c] = acc;
    __syncthreads();
    if (sub != 0 || p >= kParams) return;
    float gi = 0.f;
    for (int u = 0; u < 8; ++u) gi += red[u][c];
    grad[p] = gi;
    const float mi = b1 * m[p] + (1.f - b1) * gi;
    const float vi = b2 * v[p] + (1.f - b2) * gi * gi;
    m[p] = mi;
    v[p] = vi;
    const float t = theta[p] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    theta[p] = t;
    wb[p] = f32_to_bf16(t);
}

// Training weights omega_i = w_i / max(I_b, floor), I_b = sum_w[b] / n_emitted
// the bin's estimated intensity, floor = floor_frac * (mean I over bins with
// hits): every live bin gets equal total weight, the proposal that makes the
// per-bin relative errors equal when weights within a bin are alike.
__global__ void k_bin_stats(const double *sum_w, uint64_t n_bins, double *partial) {
    __shared__ double rs[kThreads], rc[kThreads];
    double s = 0.0, c = 0.0;
    for (uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x; i < n_bins; i += (uint64_t)gridDim.x * kThreads) {
        if (sum_w[i] > 0.0) {
            s += sum_w[i];
            c += 1.0;
        }
    }
    rs[threadIdx.x] = s;
    rc[threadIdx.x] = c;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            rs[threadIdx.x] += rs[threadIdx.x + w];
            rc[threadIdx.x] += rc[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = rs[0];
        partial[2 * blockIdx.x + 1] = rc[0];
    }
}

__global__ void k_bin_stats_final(const double *partial, unsigned n_part, double *out) {
    if (threadIdx.x != 0) return;
    double s = 0.0, c = 0.0;
    for (unsigned i = 0; i < n_part; ++i) {
        s += partial[2 * i];
        c += partial[2 * i + 1];
    }
    out[0] = c > 0.0 ? s / c : 0.0;  // mean sum_w over bins with hits
}

__global__ void k_train_weights(const double *w, const int64_t *bin, uint64_t n, const double *sum_w, uint64_t n_bins,
                                const double *mean_live, double floor_frac, double *omega) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const int64_t b = bin[i];
        const double Ib = (b >= 0 && (uint64_t)b < n_bins) ? sum_w[b] : 0.0;
        const double den = fmax(Ib, floor_frac * *mean_live);
        omega[i] = den > 0.0 ? w[i] / den : 0.0;
    }
}

// Work-groups for n items of a grid-stride kernel: at most 2^22 (the HSA
// dispatch counts a grid's work-items with 32 bits), each item reached by the
// kernel's stride loop.
unsigned blocks_for(uint64_t n) {
    return (unsigned)std::min<uint64_t>(1ull << 22, std::max<uint64_t>(1, (n + kThreads - 1) / kThreads));
}
// Work-groups for exactly n items, one per lane (n below 2^32 - kThreads).
unsigned blocks_exact(uint64_t n) { return (unsigned)std::max<uint64_t>(1, (n + kThreads - 1) / kThreads); }

// ------------------------------------------------------------ workspace --

struct Layout {
    uint64_t off[MXR_MLP_WS_REGIONS];
    uint64_t bytes;
};

uint64_t splits_for(uint64_t n) { return std::max<uint64_t>(1, (n + kSplitRows - 1) / kSplitRows); }
constexpr uint64_t kFusedGroupsMax = 256;  // the fused step's work-groups (kFusedGroups)
static_assert(kFusedGroupsMax == (uint64_t)kFusedGroups, "partial region of the fused step");

Layout layout_for(uint64_t n) {
    const uint64_t sizes[MXR_MLP_WS_REGIONS] = {
        n * kIn * 2,                    // X (bf16)
        n * kHid * 4, n * kHid * 2,     // Z1, H1
        n * kHid * 4, n * kHid * 2,     // Z2, H2
        n * kOut * 4,                   // O
        n * kOut * 4, n * kOut * 2,     // dO, dO (bf16)
        n * kHid * 4, n * kHid * 2,     // dZ2, dZ2 (bf16)
        n * kHid * 4, n * kHid * 2,     // dZ1, dZ1 (bf16)
        std::max<uint64_t>(splits_for(n), kFusedGroupsMax) * kParams * 4,  // split / group partials of the gradient
        n * 3 * 8, n * 8, n * 8,        // gathered targets, weights, per-row loss
        (kSumBlocks + 2) * 8,           // reduction scratch + sum of weights + loss
        kParams * 2,                    // W^T copies (bf16), same offsets as W
        ((n + 15) / 16 * kHid * 2 + (n + 7) / 8 * kOut) * 4,  // per-part column sums (bias gradients)
    };
    Layout L;
    uint64_t o = 0;
    for (int i = 0; i < MXR_MLP_WS_REGIONS; ++i) {
        L.off[i] = o;
        o += (sizes[i] + 255) / 256 * 256;
    }
    L.bytes = o;
    return L;
}

// Layout of a forward pass alone: the context, the layer values, the
// outputs and the transposed weights; the training regions are empty.
Layout layout_forward(uint64_t n) {
    uint64_t sizes[MXR_MLP_WS_REGIONS] = {0};
    sizes[MXR_MLP_WS_X] = n * kIn * 2;
    sizes[MXR_MLP_WS_Z1] = n * kHid * 4;
    sizes[MXR_MLP_WS_H1] = n * kHid * 2;
    sizes[MXR_MLP_WS_Z2] = n * kHid * 4;
    sizes[MXR_MLP_WS_H2] = n * kHid * 2;
    sizes[MXR_MLP_WS_O] = n * kOut * 4;
    sizes[MXR_MLP_WS_WT] = kParams * 2;
    Layout L;
    uint64_t o = 0;
    for (int i = 0; i < MXR_MLP_WS_REGIONS; ++i) {
        L.off[i] = o;
        o += (sizes[i] + 255) / 256 * 256;
    }
    L.bytes = o;
    return L;
}

// Scratch of mxr_mlp_forward_noalloc: the layer values of up to
// kScratchRows rows, in a device array the library holds on every device it
// runs on until the process ends.  Host code reaches it only through the
// address hipGetSymbolAddress gives on that device.
constexpr uint64_t kScratchRows = MXR_MLP_NOALLOC_ROWS;
constexpr uint64_t kScratchBytes = 8ull << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The current device's address of `scratch`, looked up once per device.
mxr_status scratch_address(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(MXR_E_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(MXR_E_UNSUPPORTED, "device %d: at most %d devices", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return fail(MXR_E_HIP, "address of the static scratch: %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return MXR_OK;
}

template <class T>
T *at(void *ws, const Layout &L, int region) {
    return (T *)((char *)ws + L.off[region]);
}

mxr_status check_device_ptrs(std::initializer_list<const void *> ps) {
    for (const void *p : ps)
        if (!p) return fail(MXR_E_INVALID, "null array");
    return MXR_OK;
}

// forward of the n rows already gathered into the workspace (X)
mxr_status forward_ws(const uint16_t *w, uint64_t n, void *ws, const Layout &L, hipStream_t st) {
    uint16_t *wt = at<uint16_t>(ws, L, MXR_MLP_WS_WT);
    hipLaunchKernelGGL(k_transpose_weights, dim3((kHid * kHid + kThreads - 1) / kThreads), dim3(kThreads), 0, st, w, wt);
    mxr_status s = launch_check("weight transpose");
    if (s != MXR_OK) return s;
    GemmArgs g{};
    g.M = (int64_t)n;
    // layer 1: X (n x 6) W1; B(k, n) = W1^T[n][k]
    g.A = at<uint16_t>(ws, L, MXR_MLP_WS_X), g.sam = kIn, g.sak = 1;
    g.B = wt + kW1, g.sbk = 1, g.sbn = kIn;
    g.N = kHid, g.K = kIn, g.bias = w + kB1;
    g.Z = at<float>(ws, L, MXR_MLP_WS_Z1), g.H = at<uint16_t>(ws, L, MXR_MLP_WS_H1), g.ldc = kHid;
    if ((s = gemm_strip<kEpiHidden>(g, st)) != MXR_OK) return s;
    // layer 2: H1 W2
    g.A = at<uint16_t>(ws, L, MXR_MLP_WS_H1), g.sam = kHid, g.sak = 1;
    g.B = wt + kW2, g.sbk = 1, g.sbn = kHid;
    g.N = kHid, g.K = kHid, g.bias = w + kB2;
    g.Z = at<float>(ws, L, MXR_MLP_WS_Z2), g.H = at<uint16_t>(ws, L, MXR_MLP_WS_H2);
    if ((s = gemm_strip<kEpiHidden>(g, st)) != MXR_OK) return s;
    // layer 3: H2 W3 + b3 -> O
    g.A = at<uint16_t>(ws, L, MXR_MLP_WS_H2);
    g.B = wt + kW3, g.sbk = 1, g.sbn = kHid;
    g.N = kOut, g.K = kHid, g.bias = w + kB3;
    g.C = at<float>(ws, L, MXR_MLP_WS_O), g.ldc = kOut;
    return gemm_strip<kEpiOut>(g, st);
}

// loss and gradient of the n rows gathered into the workspace
mxr_status loss_grad_ws(const uint16_t *w, uint64_t n, const float lo[3], const float hi[3], float *grad,
                        double *loss, void *ws, const Layout &L, hipStream_t st) {
    // the head launches one lane per row and component
    if (n > ((1ull << 32) - kThreads) / 8)
        return fail(MXR_E_UNSUPPORTED, "%llu rows: at most 2^29 - 32 rows per gradient", (unsigned long long)n);
    mxr_status s = forward_ws(w, n, ws, L, st);
    if (s != MXR_OK) return s;
    double *red = at<double>(ws, L, MXR_MLP_WS_SCALARS);
    double *wsum = red + kSumBlocks;
    s = sum_f64(at<double>(ws, L, MXR_MLP_WS_W), n, red, wsum, st);
    if (s != MXR_OK) return s;
    HeadArgs h;
    h.O = at<float>(ws, L, MXR_MLP_WS_O);
    h.Y = at<double>(ws, L, MXR_MLP_WS_Y);
    h.W = at<double>(ws, L, MXR_MLP_WS_W);
    h.wsum = wsum;
    h.n = n;
    for (int d = 0; d < 3; ++d) {
        h.lo[d] = lo[d];
        h.hi[d] = hi[d];
    }
    h.dO = at<float>(ws, L, MXR_MLP_WS_DO);
    h.dOh = at<uint16_t>(ws, L, MXR_MLP_WS_DOH);
    h.row_loss = at<double>(ws, L, MXR_MLP_WS_ROWLOSS);
    const int64_t tiles16 = ((int64_t)n + 15) / 16, groups8 = ((int64_t)n + 7) / 8;
    float *cp2 = at<float>(ws, L, MXR_MLP_WS_COLS), *cp1 = cp2 + tiles16 * kHid, *cp3 = cp1 + tiles16 * kHid;
    h.colpart = cp3;
    hipLaunchKernelGGL(k_head_loss_grad, dim3(blocks_exact(8 * n)), dim3(kThreads), 0, st, h);
    if ((s = launch_check("head")) != MXR_OK) return s;
    if (loss) {
        s = sum_f64(h.row_loss, n, red, loss, st);
        if (s != MXR_OK) return s;
    }
    const int64_t splits = (int64_t)splits_for(n);
    float *part = at<float>(ws, L, MXR_MLP_WS_PARTIAL);
    GemmArgs g{};
    g.kchunk = kSplitRows;
    g.K = (int64_t)n;
    g.C = part;
    g.split_stride = kParams;
    // dW3 = H2^T dO  (128 x 56)
    g.A = at<uint16_t>(ws, L, MXR_MLP_WS_H2), g.sam = 1, g.sak = kHid;
    g.B = h.dOh, g.sbk = kOut, g.sbn = 1;
    g.M = kHid, g.N = kOut, g.ldc = kOut;
    g.C = part + kW3;
    if ((s = gemm_splitk(g, splits, st)) != MXR_OK) return s;
    // dZ2 = (dO W3^T) * silu'(Z2); B(k = out, n = in) = W3[in][out]
    GemmArgs b{};
    b.M = (int64_t)n, b.N = kHid, b.K = kOut;
    b.A = h.dOh, b.sam = kOut, b.sak = 1;
    b.B = w + kW3, b.sbk = 1, b.sbn = kOut;
    b.Z = at<float>(ws, L, MXR_MLP_WS_Z2);
    b.C = at<float>(ws, L, MXR_MLP_WS_DZ2), b.H = at<uint16_t>(ws, L, MXR_MLP_WS_DZ2H), b.ldc = kHid;
    b.colpart = cp2;
    if ((s = gemm_strip<kEpiBackward>(b, st)) != MXR_OK) return s;
    // dW2 = H1^T dZ2
    g.A = at<uint16_t>(ws, L, MXR_MLP_WS_H1), g.sam = 1, g.sak = kHid;
    g.B = at<uint16_t>(ws, L, MXR_MLP_WS_DZ2H), g.sbk = kHid, g.sbn = 1;
    g.M = kHid, g.N = kHid, g.ldc = kHid;
    g.C = part + kW2;
    if ((s = gemm_splitk(g, splits, st)) != MXR_OK) return s;
    // dZ1 = (dZ2 W2^T) * silu'(Z1)
    b.K = kHid;
    b.A = at<uint16_t>(ws, L, MXR_MLP_WS_DZ2H), b.sam = kHid, b.sak = 1;
    b.B = w + kW2, b.sbk = 1, b.sbn = kHid;
    b.Z = at<float>(ws, L, MXR_MLP_WS_Z1);
    b.C = at<float>(ws, L, MXR_MLP_WS_DZ1), b.H = at<uint16_t>(ws, L, MXR_MLP_WS_DZ1H);
    b.colpart = cp1;
    if ((s = gemm_strip<kEpiBackward>(b, st)) != MXR_OK) return s;
    // dW1 = X^T dZ1
    g.A = at<uint16_t>(ws, L, MXR_MLP_WS_X), g.sam = 1, g.sak = kIn;
    g.B = at<uint16_t>(ws, L, MXR_MLP_WS_DZ1H), g.sbk = kHid, g.sbn = 1;
    g.M = kIn, g.N = kHid, g.ldc = kHid;
    g.C = part + kW1;
    if ((s = gemm_splitk(g, splits, st)) != MXR_OK) return s;
    // bias gradients: per-split sums of the fused per-part column sums
    ColReduce cr;
    cr.parts[0] = cp3, cr.n_parts[0] = groups8, cr.cols[0] = kOut, cr.pps[0] = kSplitRows / 8, cr.off[0] = kB3;
    cr.parts[1] = cp2, cr.n_parts[1] = tiles16, cr.cols[1] = kHid, cr.pps[1] = kSplitRows / 16, cr.off[1] = kB2;
    cr.parts[2] = cp1, cr.n_parts[2] = tiles16, cr.cols[2] = kHid, cr.pps[2] = kSplitRows / 16, cr.off[2] = kB1;
    cr.splits = splits;
    cr.partial = part;
    hipLaunchKernelGGL(k_colpart_reduce, dim3((kHid + 31) / 32, (unsigned)splits, 3), dim3(256), 0, st, cr);
    hipLaunchKernelGGL(k_reduce_partials, dim3(blocks_for(kParams)), dim3(kThreads), 0, st, (const float *)part,
                       splits, grad);
    return launch_check("gradient reduction");
}

mxr_status box_ok(const double lo[3], const double hi[3], float flo[3], float fhi[3]) {
    if (!lo || !hi) return fail(MXR_E_INVALID, "null box");
    for (int d = 0; d < 3; ++d) {
        if (!std::isfinite(lo[d]) || !std::isfinite(hi[d]) || !(hi[d] > lo[d]))
            return fail(MXR_E_INVALID, "box edge %d: need finite lo < hi", d);
        flo[d] = (float)lo[d];
        fhi[d] = (float)hi[d];
    }
    return MXR_OK;
}

}  // namespace

extern "C" {

uint64_t mxr_mlp_workspace_bytes(uint64_t batch) { return layout_for(batch).bytes; }

mxr_status mxr_mlp_workspace_layout(uint64_t batch, uint64_t *offsets) {
    if (!offsets) return fail(MXR_E_INVALID, "null offsets");
    const Layout L = layout_for(batch);
    for (int i = 0; i < MXR_MLP_WS_REGIONS; ++i) offsets[i] = L.off[i];
    return MXR_OK;
}

mxr_status mxr_mlp_to_bf16(const float *x, uint64_t n, uint16_t *y, void *hip_stream) {
    if (n == 0) return MXR_OK;
    if (!x || !y) return fail(MXR_E_INVALID, "null array");
    hipLaunchKernelGGL(k_to_bf16, dim3(blocks_for(n)), dim3(kThreads), 0, (hipStream_t)hip_stream, x, n, y);
    return launch_check("bfloat16 conversion");
}

mxr_status mxr_mlp_forward(const uint16_t *w, const float *ctx, uint64_t n, float *out, void *ws, uint64_t ws_bytes,
                           void *hip_stream) {
    if (n == 0) return MXR_OK;
    mxr_status s = check_device_ptrs({w, ctx, out, ws});
    if (s != MXR_OK) return s;
    const Layout L = layout_for(n);
    if (ws_bytes < L.bytes) return fail(MXR_E_INVALID, "workspace of %llu bytes, %llu needed", (unsigned long long)ws_bytes, (unsigned long long)L.bytes);
    hipStream_t st = (hipStream_t)hip_stream;
    hipLaunchKernelGGL(k_gather, dim3(blocks_for(n)), dim3(kThreads), 0, st, ctx, (const double *)nullptr,
                       (const double *)nullptr, n, (uint64_t)1, (uint64_t)0, (uint64_t)0, n,
                       at<uint16_t>(ws, L, MXR_MLP_WS_X), (double *)nullptr, (double *)nullptr);
    if ((s = launch_check("gather")) != MXR_OK) return s;
    if ((s = forward_ws(w, n, ws, L, st)) != MXR_OK) return s;
    hipError_t e = hipMemcpyAsync(out, at<float>(ws, L, MXR_MLP_WS_O), n * kOut * sizeof(float),
                                  hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return fail(MXR_E_HIP, "copy of the outputs: %s", hipGetErrorString(e));
    return MXR_OK;
}

mxr_status mxr_mlp_forward_noalloc(const uint16_t *w, const float *ctx, uint64_t n, float *out, void *hip_stream) {
    if (n == 0) return MXR_OK;
    mxr_status s = check_device_ptrs({w, ctx, out});
    if (s != MXR_OK) return s;
    if (n > kScratchRows)
        return fail(MXR_E_INVALID, "%llu rows: the allocation-free forward takes at most %llu rows per call",
                    (unsigned long long)n, (unsigned long long)kScratchRows);
    const Layout L = layout_forward(n);
    if (L.bytes > kScratchBytes) return fail(MXR_E_INVALID, "the forward's layer values exceed the static scratch");
    void *ws = nullptr;
    if ((s = scratch_address(&ws)) != MXR_OK) return s;
    hipStream_t st = (hipStream_t)hip_stream;
    hipLaunchKernelGGL(k_gather, dim3(blocks_for(n)), dim3(kThreads), 0, st, ctx, (const double *)nullptr,
                       (const double *)nullptr, n, (uint64_t)1, (uint64_t)0, (uint64_t)0, n,
                       at<uint16_t>(ws, L, MXR_MLP_WS_X), (double *)nullptr, (double *)nullptr);
    if ((s = launch_check("gather")) != MXR_OK) return s;
    if ((s = forward_ws(w, n, ws, L, st)) != MXR_OK) return s;
    hipError_t e = hipMemcpyAsync(out, at<float>(ws, L, MXR_MLP_WS_O), n * kOut * sizeof(float),
                                  hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return fail(MXR_E_HIP, "copy of the outputs: %s", hipGetErrorString(e));
    return MXR_OK;
}

mxr_status mxr_mlp_mixture(const float *out, uint64_t n, const double lo[3], const double hi[3], double *gmm,
                           void *hip_stream) {
    if (n == 0) return MXR_OK;
    float flo[3], fhi[3];
    mxr_status s = box_ok(lo, hi, flo, fhi);
    if (s != MXR_OK) return s;
    if ((s = check_device_ptrs({out, gmm})) != MXR_OK) return s;
    hipLaunchKernelGGL(k_head_params, dim3(blocks_for(n)), dim3(kThreads), 0, (hipStream_t)hip_stream, out, n,
                       flo[0], flo[1], flo[2], fhi[0], fhi[1], fhi[2], gmm);
    return launch_check("mixture head");
}

mxr_status mxr_mlp_loss_grad(const uint16_t *w, const float *ctx, const double *y, const double *omega, uint64_t n,
                             const double lo[3], const double hi[3], float *grad, double *loss, void *ws,
                             uint64_t ws_bytes, void *hip_stream) {
    if (n == 0) return fail(MXR_E_INVALID, "empty batch");
    float flo[3], fhi[3];
    mxr_status s = box_ok(lo, hi, flo, fhi);
    if (s != MXR_OK) return s;
    if ((s = check_device_ptrs({w, ctx, y, omega, grad, ws})) != MXR_OK) return s;
    const Layout L = layout_for(n);
    if (ws_bytes < L.bytes) return fail(MXR_E_INVALID, "workspace of %llu bytes, %llu needed", (unsigned long long)ws_bytes, (unsigned long long)L.bytes);
    hipStream_t st = (hipStream_t)hip_stream;
    hipLaunchKernelGGL(k_gather, dim3(blocks_for(n)), dim3(kThreads), 0, st, ctx, y, omega, n, (uint64_t)1,
                       (uint64_t)0, (uint64_t)0, n, at<uint16_t>(ws, L, MXR_MLP_WS_X), at<double>(ws, L, MXR_MLP_WS_Y),
                       at<double>(ws, L, MXR_MLP_WS_W));
    if ((s = launch_check("gather")) != MXR_OK) return s;
    return loss_grad_ws(w, n, flo, fhi, grad, loss, ws, L, st);
}

mxr_status mxr_adam_step(float *master, uint16_t *w, const float *grad, float *m, float *v, uint64_t n_params,
                         uint32_t step, float lr, float beta1, float beta2, float eps, void *hip_stream) {
    if (n_params == 0) return MXR_OK;
    mxr_status s = check_device_ptrs({master, w, grad, m, v});
    if (s != MXR_OK) return s;
    if (step < 1) return fail(MXR_E_INVALID, "Adam steps count from 1");
    if (!(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps >= 0.f))
        return fail(MXR_E_INVALID, "bad Adam hyper-parameters");
    const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, (double)step)));
    const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, (double)step)));
    hipLaunchKernelGGL(k_adam, dim3(blocks_for(n_params)), dim3(kThreads), 0, (hipStream_t)hip_stream, master, w, grad,
                       m, v, n_params, lr, beta1, beta2, eps, c1, c2);
    return launch_check("Adam");
}

mxr_status mxr_train_weights(const double *w, const int64_t *bin, uint64_t n, const double *sum_w, uint64_t n_bins,
                             double floor_frac, double *omega, double *scratch, void *hip_stream) {
    if (n == 0) return MXR_OK;
    mxr_status s = check_device_ptrs({w, bin, sum_w, omega, scratch});
    if (s != MXR_OK) return s;
    if (!(floor_frac >= 0.0) || !std::isfinite(floor_frac)) return fail(MXR_E_INVALID, "bad floor fraction");
    hipStream_t st = (hipStream_t)hip_stream;
    hipLaunchKernelGGL(k_bin_stats, dim3(kSumBlocks), dim3(kThreads), 0, st, sum_w, n_bins, scratch);
    hipLaunchKernelGGL(k_bin_stats_final, dim3(1), dim3(64), 0, st, (const double *)scratch, kSumBlocks,
                       scratch + 2 * kSumBlocks);
    hipLaunchKernelGGL(k_train_weights, dim3(blocks_for(n)), dim3(kThreads), 0, st, w, bin, n, sum_w, n_bins,
                       (const double *)(scratch + 2 * kSumBlocks), floor_frac, omega);
    return launch_check("training weights");
}

mxr_status mxr_mlp_train(const float *ctx, const double *y, const double *omega, uint64_t n_rows,
                         const mxr_train_cfg *cfg, const double lo[3], const double hi[3], float *master, uint16_t *w,
                         float *m, float *v, float *grad, void *ws, uint64_t ws_bytes, double *loss_log,
                         void *hip_stream) {
    if (!cfg) return fail(MXR_E_INVALID, "null configuration");
    if (n_rows == 0) return fail(MXR_E_INVALID, "no training rows");
    if (cfg->batch == 0 || cfg->epochs == 0) return fail(MXR_E_INVALID, "batch and epochs must be positive");
    if (n_rows >= (1ull << 32)) return fail(MXR_E_UNSUPPORTED, "at most 2^32 - 1 training rows");
    float flo[3], fhi[3];
    mxr_status s = box_ok(lo, hi, flo, fhi);
    if (s != MXR_OK) return s;
    if ((s = check_device_ptrs({ctx, y, omega, master, w, m, v, grad, ws})) != MXR_OK) return s;
    const uint64_t B = std::min<uint64_t>(cfg->batch, n_rows);
    const Layout L = layout_for(B);
    if (ws_bytes < L.bytes) return fail(MXR_E_INVALID, "workspace of %llu bytes, %llu needed", (unsigned long long)ws_bytes, (unsigned long long)L.bytes);
    hipStream_t st = (hipStream_t)hip_stream;
    const uint64_t steps_per_epoch = (n_rows + B - 1) / B;
    // per-epoch bijections i -> (a i + b) mod n_rows from a splitmix64 sequence
    uint64_t state = cfg->seed;
    auto next = [&state]() {
        uint64_t z = (state += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    };
    auto gcd = [](uint64_t a, uint64_t b) {
        while (b) {
            const uint64_t t = a % b;
            a = b;
            b = t;
        }
        return a;
    };
    uint32_t step = cfg->first_step;
    for (uint32_t e = 0; e < cfg->epochs; ++e) {
        uint64_t a = 1, b = 0;
        if (n_rows > 1) {
            a = next() % n_rows;
            while (a == 0 || gcd(a, n_rows) != 1) a = (a + 1) % n_rows;
            b = next() % n_rows;
        }
        for (uint64_t k = 0; k < steps_per_epoch; ++k) {
            const uint64_t first = k * B, cnt = std::min<uint64_t>(B, n_rows - first);
            double *lp = loss_log ? loss_log + (uint64_t)e * steps_per_epoch + k : nullptr;
            ++step;
            if (!(cfg->lr > 0.f) || !(cfg->beta1 >= 0.f && cfg->beta1 < 1.f) ||
                !(cfg->beta2 >= 0.f && cfg->beta2 < 1.f) || !(cfg->eps >= 0.f))
                return fail(MXR_E_INVALID, "bad Adam hyper-parameters");
            // one fused launch per step: the batch's weight sum, the
            // gradient partials of every strip, their ordered sum and Adam
            double *red = at<double>(ws, L, MXR_MLP_WS_SCALARS), *wsum = red + kSumBlocks;
            hipLaunchKernelGGL(k_batch_wsum, dim3(kSumBlocks), dim3(kThreads), 0, st, omega, n_rows, a, b, first, cnt,
                               red);
            hipLaunchKernelGGL(k_sum_f64, dim3(1), dim3(kThreads), 0, st, (const double *)red, (uint64_t)kSumBlocks,
                               wsum);
            FusedArgs fa;
            fa.ctx = ctx;
            fa.y = y;
            fa.omega = omega;
            fa.n_data = n_rows;
            fa.a = a;
            fa.b = b;
            fa.first = first;
            fa.cnt = cnt;
            fa.wsum = wsum;
            fa.w = w;
            for (int d = 0; d < 3; ++d) {
                fa.lo[d] = flo[d];
                fa.hi[d] = fhi[d];
            }
            fa.part = at<float>(ws, L, MXR_MLP_WS_PARTIAL);
            fa.loss_part = at<double>(ws, L, MXR_MLP_WS_ROWLOSS);
            const uint64_t strips = (cnt + kStripRows - 1) / kStripRows;
            const int groups = (int)std::min<uint64_t>(kFusedGroups, strips);
            hipLaunchKernelGGL(k_train_fused, dim3(groups), dim3(kFusedThreads), 0, st, fa);
            const float c1 = (float)(1.0 / (1.0 - std::pow((double)cfg->beta1, (double)step)));
            const float c2 = (float)(1.0 / (1.0 - std::pow((double)cfg->beta2, (double)step)));
            hipLaunchKernelGGL(k_fused_reduce_adam, dim3((unsigned)((kParams + kReduceParams - 1) / kReduceParams)),
                               dim3(256), 0, st,
                               (const float *)fa.part, groups, grad, master, w, m, v, cfg->lr, cfg->beta1, cfg->beta2,
                               cfg->eps, c1, c2, (const double *)fa.loss_part, lp);
            if ((s = launch_check("fused training step")) != MXR_OK) return s;
        }
    }
    return MXR_OK;
}

mxr_status mxr_proposal_train(const mxr_instrument *ins, const mxr_train_rows *rows, const mxr_train_cfg *cfg,
                              float *master, uint16_t *w, float *m, float *v, float *grad, double *omega, void *ws,
                              uint64_t ws_bytes, double *loss_log, void *hip_stream) {
    if (!rows || !cfg) return fail(MXR_E_INVALID, "null rows or configuration");
    double lo[3], hi[3];
    mxr_status s = mxr_proposal_box(ins, lo, hi);
    if (s != MXR_OK) return s;
    const mxr_train_rows &R = *rows;
    if (R.n_rows == 0) return fail(MXR_E_INVALID, "no training rows");
    if (R.n_runs == 0 || !R.run_first || !R.run_image) return fail(MXR_E_INVALID, "no run table");
    if (R.run_first[0] != 0 || R.run_first[R.n_runs] != R.n_rows)
        return fail(MXR_E_INVALID, "the run table must cover rows [0, n_rows)");
    if ((s = check_device_ptrs({R.ctx, R.y, R.w, R.bin, omega, ws})) != MXR_OK) return s;
    if (ws_bytes < (2 * kSumBlocks + 1) * sizeof(double))
        return fail(MXR_E_INVALID, "workspace of %llu bytes is too small", (unsigned long long)ws_bytes);
    for (uint32_t r = 0; r < R.n_runs; ++r) {
        const uint64_t a = R.run_first[r], b = R.run_first[r + 1];
        if (b < a || b > R.n_rows) return fail(MXR_E_INVALID, "run %u: rows [%llu, %llu) out of order", r,
                                               (unsigned long long)a, (unsigned long long)b);
        if (b == a) continue;
        if (!R.run_image[r]) return fail(MXR_E_INVALID, "run %u: null image", r);
        // the weight statistics use the start of the workspace; the training
        // below overwrites it only after these kernels (same stream)
        if ((s = mxr_train_weights(R.w + a, R.bin + a, b - a, R.run_image[r], R.n_bins, R.floor_frac, omega + a,
                                   (double *)ws, hip_stream)) != MXR_OK)
            return s;
    }
    return mxr_mlp_train(R.ctx, R.y, omega, R.n_rows, cfg, lo, hi, master, w, m, v, grad, ws, ws_bytes, loss_log,
                         hip_stream);
}

mxr_status mxr_proposal_apply(mxr_instrument *ins, const uint16_t *w, const float context[6], double alpha, void *ws,
                              uint64_t ws_bytes, void *hip_stream) {
    double lo[3], hi[3];
    mxr_status s = mxr_proposal_box(ins, lo, hi);
    if (s != MXR_OK) return s;
    if (!w || !context || !ws) return fail(MXR_E_INVALID, "null parameters, context or workspace");
    const uint64_t net_bytes = layout_for(1).bytes;
    if (ws_bytes < net_bytes + 1024)
        return fail(MXR_E_INVALID, "workspace of %llu bytes, %llu needed", (unsigned long long)ws_bytes,
                    (unsigned long long)(net_bytes + 1024));
    // after the network's workspace: the context (6 floats), the outputs
    // (56 floats) and the mixture (56 doubles)
    char *tail = (char *)ws + net_bytes;
    float *ctx = (float *)tail, *out = (float *)(tail + 64);
    double *gmm = (double *)(tail + 512);
    hipStream_t st = (hipStream_t)hip_stream;
    hipError_t e = hipMemcpyAsync(ctx, context, kIn * sizeof(float), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return fail(MXR_E_HIP, "copy of the context: %s", hipGetErrorString(e));
    if ((s = mxr_mlp_forward(w, ctx, 1, out, ws, net_bytes, hip_stream)) != MXR_OK) return s;
    if ((s = mxr_mlp_mixture(out, 1, lo, hi, gmm, hip_stream)) != MXR_OK) return s;
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(MXR_E_HIP, "network forward: %s", hipGetErrorString(e));
    return mxr_proposal_set(ins, gmm, alpha);
}

}  // extern "C"
