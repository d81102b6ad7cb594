// Generalized CP with the Poisson log-link loss (Sec. 8 names generalized CP as the next
// workload): loss sum_i w_i (exp(m_i) - x_i m_i) over the stored entries, and its gradient with
// respect to every factor, which is an MTTKRP of the elementwise derivative tensor
// y_i = w_i (exp(m_i) - x_i) sharing the tensor's subscripts and permutations.
#include "mttkrp_kernels.h"

namespace spt {

int gcp_forward_impl(const spt_tensor *X, int R, const void *const *factors, int fdtype,
                     int loss_kind, const void *w, void *m, double *loss, double *part,
                     hipStream_t s);


// y_i = g * w_i * df(x_i, m_i), g the upstream gradient (device scalar, NULL = 1)
template <int RW, class T>
__global__ __launch_bounds__(kBlock) void k_gcp_deriv(const int4 *__restrict__ rec, int64_t P,
                                                      const T *__restrict__ w,
                                                      const T *__restrict__ m,
                                                      const double *__restrict__ gscale,
                                                      T *__restrict__ y, int loss) {
    const T g = gscale != nullptr ? (T)*gscale : (T)1;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < P; i += stride) {
        const int *rw = reinterpret_cast<const int *>(rec + i * (RW / 4));
        const T x = rec_value<T, RW>(rw);
        const T wi = (w != nullptr) ? w[i] : (T)1;
        y[i] = g * wi * gcp_dloss<T>(loss, x, m[i]);
    }
}

template <class T>
static int launch_deriv(const spt_tensor *X, const T *w, const T *m, const double *gscale, T *y,
                        hipStream_t s, int loss) {
    int64_t blocks = ceil_div(X->P, kBlock);
    if (blocks > 8192) blocks = 8192;
    if (X->rec_words == 4)
        hipLaunchKernelGGL((k_gcp_deriv<4, T>), dim3((unsigned)blocks), dim3(kBlock), 0, s, X->rec,
                           X->P, w, m, gscale, y, loss);
    else
        hipLaunchKernelGGL((k_gcp_deriv<8, T>), dim3((unsigned)blocks), dim3(kBlock), 0, s, X->rec,
                           X->P, w, m, gscale, y, loss);
    return hipGetLastError() == hipSuccess ? SPT_OK : SPT_EHIP;
}

}  // namespace spt

using namespace spt;

extern "C" {

static int gcp_dtype_ok(const spt_tensor *X, int fdtype) {
    if (fdtype == SPT_F64) return X->vdtype == SPT_F64 ? SPT_OK : SPT_EUNSUPPORTED;
    if (fdtype == SPT_F32) return X->vdtype == SPT_F32 ? SPT_OK : SPT_EUNSUPPORTED;
    return fdtype == SPT_BF16 ? SPT_EUNSUPPORTED : SPT_EINVAL;
}

int spt_gcp_forward(const spt_tensor *X, int R, const void *const *factors, int fdtype,
                    int loss_kind, const void *w, void *m, double *loss, void *ws,
                    size_t ws_bytes, void *stream) {
    if (X == nullptr || R < 1 || R > 256 || m == nullptr || loss == nullptr) return SPT_EINVAL;
    if (loss_kind < SPT_GCP_POISSON || loss_kind > SPT_GCP_GAMMA) return SPT_EINVAL;
    if (int e = gcp_dtype_ok(X, fdtype)) return e;
    int rc = check_factors(X, -1, factors);
    if (rc == SPT_OK) rc = check_factor_extent(X, -1, R, fdtype);
    if (rc) return rc;
    if (ws == nullptr || ((uintptr_t)ws & 255u) || ws_bytes < 2 * 2048 * sizeof(double))
        return SPT_EWORKSPACE;
    return gcp_forward_impl(X, R, factors, fdtype, loss_kind, w, m, loss,
                            static_cast<double *>(ws), static_cast<hipStream_t>(stream));
}

int spt_gcp_poisson_forward(const spt_tensor *X, int R, const void *const *factors, int fdtype,
                            const void *w, void *m, double *loss, void *ws, size_t ws_bytes,
                            void *stream) {
    return spt_gcp_forward(X, R, factors, fdtype, SPT_GCP_POISSON, w, m, loss, ws, ws_bytes,
                           stream);
}

int spt_gcp_backward(const spt_tensor *X, int R, const void *const *factors, int fdtype,
                     int loss_kind, const void *w, const void *m, const double *gscale, void *y,
                     void *const *grads, const spt_tune *tune, void *stream) {
    if (X == nullptr || R < 1 || R > 256 || m == nullptr || y == nullptr || grads == nullptr)
        return SPT_EINVAL;
    if (loss_kind < SPT_GCP_POISSON || loss_kind > SPT_GCP_GAMMA) return SPT_EINVAL;
    if (int e = gcp_dtype_ok(X, fdtype)) return e;
    int rc = check_factors(X, -1, factors);
    if (rc == SPT_OK) rc = check_factor_extent(X, -1, R, fdtype);
    if (rc) return rc;
    for (int n = 0; n < X->d; ++n)
        if (grads[n] == nullptr) return SPT_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (X->P > 0) {
        rc = (fdtype == SPT_F64)
                 ? launch_deriv<double>(X, static_cast<const double *>(w),
                                        static_cast<const double *>(m), gscale,
                                        static_cast<double *>(y), s, loss_kind)
                 : launch_deriv<float>(X, static_cast<const float *>(w),
                                       static_cast<const float *>(m), gscale,
                                       static_cast<float *>(y), s, loss_kind);
        if (rc) return rc;
    }
    for (int n = 0; n < X->d; ++n) {
        spt_tune t;
        rc = resolve_tune(X, n, R, fdtype, tune, &t);
        if (rc) return rc;
        if (t.algo == SPT_ALGO_PERMUTED && !X->permuted[n]) t.algo = SPT_ALGO_ATOMIC;
        if (t.algo == SPT_ALGO_PERMUTED_COPY && X->srec[n] == nullptr)
            t.algo = X->permuted[n] ? SPT_ALGO_PERMUTED : SPT_ALGO_ATOMIC;
        rc = launch_mttkrp(X, n, R, factors, fdtype, nullptr, y, grads[n], t, s);
        if (rc) return rc;
    }
    return SPT_OK;
}

int spt_gcp_poisson_backward(const spt_tensor *X, int R, const void *const *factors, int fdtype,
                             const void *w, const void *m, const double *gscale, void *y,
                             void *const *grads, const spt_tune *tune, void *stream) {
    return spt_gcp_backward(X, R, factors, fdtype, SPT_GCP_POISSON, w, m, gscale, y, grads, tune,
                            stream);
}

}  // extern "C"
