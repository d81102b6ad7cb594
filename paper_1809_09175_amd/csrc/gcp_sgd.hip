// Stochastic generalized CP (GCP-SGD): the stratified sample of an iteration drawn on the device
// with the Philox4x64-10 counter-based generator (Salmon et al., SC'11), and the Adam update of
// the factors.  Generalized CP is the workload Sec. 8 names next; the sampled loss and gradient
// come from the existing GCP entry points.
#include "spt_internal.h"

namespace spt {

__device__ __forceinline__ void philox4x64(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                           uint64_t k0, uint64_t k1, uint64_t out[4]) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t lo0 = 0xD2E7470EE14C6C93ull * c0, hi0 = __umul64hi(0xD2E7470EE14C6C93ull, c0);
        const uint64_t lo1 = 0xCA5A826395121157ull * c2, hi1 = __umul64hi(0xCA5A826395121157ull, c2);
        const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B97F4A7C15ull;
        k1 += 0xBB67AE8584CAA73Bull;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

// floor(r * n / 2^64)
__device__ __forceinline__ int64_t scale_index(uint64_t r, int64_t n) {
    return (int64_t)__umul64hi(r, (uint64_t)n);
}

template <int RW, class VT, class OT>
__global__ __launch_bounds__(kBlock) void k_gcp_sample(const int4 *__restrict__ rec, int d,
                                                       int64_t P, int64_t dim0, int64_t dim1,
                                                       int64_t dim2, int64_t dim3, int64_t dim4,
                                                       uint64_t seed, int64_t iter, int64_t s_nz,
                                                       int64_t s_z, double w_nz, double w_z,
                                                       int32_t *__restrict__ osubs,
                                                       OT *__restrict__ ovals,
                                                       OT *__restrict__ ow) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= s_nz + s_z) return;
    const int64_t dims[SPT_MAX_ORDER] = {dim0, dim1, dim2, dim3, dim4};
    uint64_t r[8];
    if (e < s_nz) {
        philox4x64((uint64_t)e, (uint64_t)iter, 0, 0, seed, 0, r);
        const int64_t p = scale_index(r[0], P);
        const int *w = reinterpret_cast<const int *>(rec + p * (RW / 4));
#pragma unroll
        for (int m = 0; m < SPT_MAX_ORDER; ++m)
            if (m < d) osubs[e * d + m] = w[m];
        VT x;
        if constexpr (sizeof(VT) == 8)
            x = __hiloint2double(w[RW - 1], w[RW - 2]);
        else
            x = __int_as_float(w[RW - 1]);
        ovals[e] = (OT)x;
        ow[e] = (OT)w_nz;
    } else {
        const int64_t k = e - s_nz;
        philox4x64((uint64_t)k, (uint64_t)iter, 1, 0, seed, 0, r);
        if (d > 4) philox4x64((uint64_t)k, (uint64_t)iter, 1, 1, seed, 0, r + 4);
#pragma unroll
        for (int m = 0; m < SPT_MAX_ORDER; ++m)
            if (m < d) osubs[e * d + m] = (int32_t)scale_index(r[m], dims[m]);
        ovals[e] = (OT)0;
        ow[e] = (OT)w_z;
    }
}

// one Adam step; the bias corrections c1 = 1 - beta1^t, c2 = 1 - beta2^t come from the host
template <class T>
__global__ __launch_bounds__(kBlock) void k_adam(T *__restrict__ x, const T *__restrict__ g,
                                                 T *__restrict__ m, T *__restrict__ v, int64_t n,
                                                 double lr, double b1, double b2, double eps,
                                                 double c1, double c2, double lower) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        const double gi = (double)g[i];
        const double mi = b1 * (double)m[i] + (1.0 - b1) * gi;
        const double vi = b2 * (double)v[i] + (1.0 - b2) * gi * gi;
        m[i] = (T)mi;
        v[i] = (T)vi;
        double xi = (double)x[i] - lr * (mi / c1) / (sqrt(vi / c2) + eps);
        x[i] = (T)(xi < lower ? lower : xi);
    }
}

}  // namespace spt

using namespace spt;

extern "C" {

int spt_gcp_sample(const spt_tensor *X, uint64_t seed, int64_t iter, int64_t s_nz, int64_t s_z,
                   int32_t *subs, void *vals, void *w, int dtype, void *stream) {
    if (X == nullptr || s_nz < 0 || s_z < 0 || iter < 0 || (s_nz > 0 && X->P == 0)) return SPT_EINVAL;
    if (s_nz + s_z > INT32_MAX) return SPT_EINVAL;
    if (s_nz + s_z > 0 && (subs == nullptr || vals == nullptr || w == nullptr)) return SPT_EINVAL;
    if (dtype != SPT_F32 && dtype != SPT_F64) return SPT_EINVAL;
    if (s_nz + s_z == 0) return SPT_OK;
    double cells = 1.0;
    for (int m = 0; m < X->d; ++m) cells *= (double)X->dims[m];
    const double w_nz = s_nz > 0 ? (double)X->P / (double)s_nz : 0.0;
    const double w_z = (s_z > 0 && cells > (double)X->P) ? (cells - (double)X->P) / (double)s_z : 0.0;
    const int64_t *dd = X->dims;
    dim3 g((unsigned)ceil_div(s_nz + s_z, kBlock)), b(kBlock);
    hipStream_t s = static_cast<hipStream_t>(stream);
#define SPT_SAMPLE(RW_, VT_, OT_)                                                                \
    hipLaunchKernelGGL((k_gcp_sample<RW_, VT_, OT_>), g, b, 0, s, X->rec, X->d, X->P, dd[0],     \
                       dd[1], dd[2], dd[3], dd[4], seed, iter, s_nz, s_z, w_nz, w_z, subs,       \
                       static_cast<OT_ *>(vals), static_cast<OT_ *>(w))
    const bool f64v = X->vdtype == SPT_F64;
    if (X->rec_words == 4) {
        if (f64v) {
            if (dtype == SPT_F64) SPT_SAMPLE(4, double, double); else SPT_SAMPLE(4, double, float);
        } else {
            if (dtype == SPT_F64) SPT_SAMPLE(4, float, double); else SPT_SAMPLE(4, float, float);
        }
    } else {
        if (f64v) {
            if (dtype == SPT_F64) SPT_SAMPLE(8, double, double); else SPT_SAMPLE(8, double, float);
        } else {
            if (dtype == SPT_F64) SPT_SAMPLE(8, float, double); else SPT_SAMPLE(8, float, float);
        }
    }
#undef SPT_SAMPLE
    return hipGetLastError() == hipSuccess ? SPT_OK : SPT_EHIP;
}

int spt_adam_step(void *x, const void *g, void *m, void *v, int64_t n, int dtype, double lr,
                  double beta1, double beta2, double eps, int64_t t, double lower, void *stream) {
    if (n < 0 || t < 1 || (n > 0 && (x == nullptr || g == nullptr || m == nullptr || v == nullptr)))
        return SPT_EINVAL;
    if (dtype != SPT_F32 && dtype != SPT_F64) return SPT_EINVAL;
    if (n == 0) return SPT_OK;
    const double c1 = 1.0 - pow(beta1, (double)t), c2 = 1.0 - pow(beta2, (double)t);
    int64_t blocks = ceil_div(n, kBlock);
    if (blocks > 4096) blocks = 4096;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (dtype == SPT_F64)
        hipLaunchKernelGGL(k_adam<double>, dim3((unsigned)blocks), dim3(kBlock), 0, s,
                           static_cast<double *>(x), static_cast<const double *>(g),
                           static_cast<double *>(m), static_cast<double *>(v), n, lr, beta1,
                           beta2, eps, c1, c2, lower);
    else
        hipLaunchKernelGGL(k_adam<float>, dim3((unsigned)blocks), dim3(kBlock), 0, s,
                           static_cast<float *>(x), static_cast<const float *>(g),
                           static_cast<float *>(m), static_cast<float *>(v), n, lr, beta1,
                           beta2, eps, c1, c2, lower);
    return hipGetLastError() == hipSuccess ? SPT_OK : SPT_EHIP;
}

}  // extern "C"
