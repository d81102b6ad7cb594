// Precision and measurement helpers: FP32 -> BF16 and FP64 -> BF16 rounding and a STREAM-style
// triad.
#include "spt_internal.h"

namespace spt {

__global__ __launch_bounds__(kBlock) void k_f32_to_bf16(const float *__restrict__ in,
                                                        uint16_t *__restrict__ out, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride)
        out[i] = f32_to_bf16_rne(in[i]);
}

__global__ __launch_bounds__(kBlock) void k_f64_to_bf16(const double *__restrict__ in,
                                                        uint16_t *__restrict__ out, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride)
        out[i] = f64_to_bf16_rne(in[i]);
}

// Each thread handles kTriadUnroll float4 elements, strided by the block size so every load and
// store instruction of a wave covers 1 KiB of contiguous memory; the output is written with
// non-temporal stores (it is not read again).
constexpr int kTriadUnroll = 4;

__global__ __launch_bounds__(kBlock) void k_triad(float4 *__restrict__ a,
                                                  const float4 *__restrict__ b,
                                                  const float4 *__restrict__ c, float s,
                                                  int64_t nq) {
    const int64_t base = (int64_t)blockIdx.x * kBlock * kTriadUnroll + threadIdx.x;
    float4 x[kTriadUnroll], y[kTriadUnroll];
#pragma unroll
    for (int k = 0; k < kTriadUnroll; ++k) {
        const int64_t i = base + (int64_t)k * kBlock;
        if (i < nq) {
            x[k] = b[i];
            y[k] = c[i];
        }
    }
#pragma unroll
    for (int k = 0; k < kTriadUnroll; ++k) {
        const int64_t i = base + (int64_t)k * kBlock;
        if (i < nq) {
            float4 r = make_float4(x[k].x + s * y[k].x, x[k].y + s * y[k].y, x[k].z + s * y[k].z,
                                   x[k].w + s * y[k].w);
            __builtin_nontemporal_store(r.x, &a[i].x);
            __builtin_nontemporal_store(r.y, &a[i].y);
            __builtin_nontemporal_store(r.z, &a[i].z);
            __builtin_nontemporal_store(r.w, &a[i].w);
        }
    }
}

__global__ void k_triad_tail(float *a, const float *b, const float *c, float s, int64_t lo,
                             int64_t n) {
    int64_t i = lo + threadIdx.x;
    if (i < n) a[i] = b[i] + s * c[i];
}

}  // namespace spt

using namespace spt;

extern "C" int spt_f32_to_bf16(const float *in, uint16_t *out, int64_t n, void *stream) {
    if (n < 0 || (n > 0 && (in == nullptr || out == nullptr))) return SPT_EINVAL;
    if (n == 0) return SPT_OK;
    int64_t blocks = ceil_div(n, kBlock);
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_f32_to_bf16, dim3((unsigned)blocks), dim3(kBlock), 0,
                       static_cast<hipStream_t>(stream), in, out, n);
    return hipGetLastError() == hipSuccess ? SPT_OK : SPT_EHIP;
}

extern "C" int spt_f64_to_bf16(const double *in, uint16_t *out, int64_t n, void *stream) {
    if (n < 0 || (n > 0 && (in == nullptr || out == nullptr))) return SPT_EINVAL;
    if (n == 0) return SPT_OK;
    int64_t blocks = ceil_div(n, kBlock);
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_f64_to_bf16, dim3((unsigned)blocks), dim3(kBlock), 0,
                       static_cast<hipStream_t>(stream), in, out, n);
    return hipGetLastError() == hipSuccess ? SPT_OK : SPT_EHIP;
}

extern "C" int spt_stream_triad(float *a, const float *b, const float *c, float s, int64_t n,
                                void *stream) {
    if (n < 0 || (n > 0 && (a == nullptr || b == nullptr || c == nullptr))) return SPT_EINVAL;
    if ((((uintptr_t)a) | ((uintptr_t)b) | ((uintptr_t)c)) & 15u) return SPT_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t nq = n / 4;
    if (nq > 0) {
        const int64_t blocks = ceil_div(nq, (int64_t)kBlock * kTriadUnroll);
        hipLaunchKernelGGL(k_triad, dim3((unsigned)blocks), dim3(kBlock), 0, st,
                           reinterpret_cast<float4 *>(a), reinterpret_cast<const float4 *>(b),
                           reinterpret_cast<const float4 *>(c), s, nq);
    }
    if (nq * 4 < n)
        hipLaunchKernelGGL(k_triad_tail, dim3(1), dim3(64), 0, st, a, b, c, s, nq * 4, n);
    return hipGetLastError() == hipSuccess ? SPT_OK : SPT_EHIP;
}
