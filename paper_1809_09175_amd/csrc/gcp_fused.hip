// Fused generalized-CP loss and gradient (Sec. 8 names generalized CP as the next workload).
// One pass per mode n over the entries in mode-n order (the sorted record copy, or the records
// gathered through the permutation) computes each entry's model value, the loss derivative y
// and y's contribution to the mode-n gradient row, an MTTKRP of the derivative tensor with the
// same segmented reduction as the permuted MTTKRP.  The derivative tensor is never written, and
// the only gathers are the factor rows the MTTKRP reads anyway plus the mode-n row, which a lane
// group loads once per run of equal mode-n subscripts.
// The pass over mode 0 also sums the loss.
#include "mttkrp_kernels.h"

namespace spt {

int device_cus();  // compute units of the current device (mttkrp.hip)

template <int D, int G, int CPL, class FT>
__global__ __launch_bounds__(kBlock) void k_gcp_fused(const int4 *__restrict__ rec,
                                                      const int32_t *__restrict__ perm,
                                                      const int4 *__restrict__ srec, int64_t P,
                                                      int n, int R, FactorSet<FT> A,
                                                      FT *__restrict__ V, int chunk, int loss,
                                                      double *__restrict__ loss_part) {
    __shared__ PermShared<D, G, CPL, FT, FT> sm[kBlock / kWave];
    const int wave = threadIdx.x >> 6;
    const int64_t c0 = ((int64_t)blockIdx.x * (kBlock / kWave) + wave) * chunk;
    if (c0 >= P) return;  // whole wavefront leaves together
    // one entry at a time per lane group: the fused entry holds d factor rows and the model
    // butterfly, and deeper unrolling cost occupancy (1e8 entries, R = 32: 9.7 ms for the three
    // passes against 11.7-15.9 ms with 2-8 entries in flight)
    perm_wave_chunk<D, G, CPL, FT, FT, FT, 1, true>(sm[wave], rec, perm, srec, P, n, R, A, nullptr,
                                                     nullptr, V, chunk, c0, nullptr, nullptr, loss,
                                                     loss_part);
}

// loss = sum of the per-wave partials: lane l adds partials l, l + 64, ... in order, then a
// fixed butterfly (one wavefront, reproducible)
__global__ __launch_bounds__(kWave) void k_sum_loss(const double *__restrict__ part, int64_t n,
                                                    double *__restrict__ loss) {
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kWave) s += part[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (threadIdx.x == 0) *loss = s;
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_scale(const T *src, T *dst, int64_t n,
                                                  const double *__restrict__ g) {
    const T s = (T)*g;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride)
        dst[i] = src[i] * s;
}

struct FusedArgs {
    const int4 *rec;
    const int32_t *perm;
    const int4 *srec;
    int64_t P;
    int n, R, chunk, loss;
    int auto_chunk, min_chunk, cus;
    void *V;
    double *loss_part;
    int64_t *nparts;  // out: wave chunks of the launch (loss partials of mode 0)
    hipStream_t s;
};

template <int D, int G, int CPL, class FT>
static int launch_fused_cfg(const FusedArgs &a, const FactorSet<FT> &A) {
    int chunk = a.chunk;
    // the sorted-copy MTTKRP's rule for the default chunk (capacity_chunk), with this kernel's
    // occupancy; never below the chunk the loss partials need (8.19 ms instead of 8.34 for the
    // three passes over 1e8 entries at R = 32)
    if (a.auto_chunk && a.srec != nullptr && CPL >= 4) {
        static const int per_cu = [] {
            int nb = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_gcp_fused<D, G, CPL, FT>,
                                                             kBlock, 0) != hipSuccess)
                nb = 0;
            return nb * (kBlock / kWave);
        }();
        chunk = capacity_chunk(a.P, (int64_t)per_cu * a.cus, chunk);
        if (chunk < a.min_chunk) chunk = a.min_chunk;
    }
    *a.nparts = ceil_div(a.P, chunk);
    const unsigned grid = (unsigned)ceil_div(a.P, (int64_t)chunk * (kBlock / kWave));
    if (grid == 0) return SPT_OK;
    hipLaunchKernelGGL((k_gcp_fused<D, G, CPL, FT>), dim3(grid), dim3(kBlock), 0, a.s, a.rec,
                       a.perm, a.srec, a.P, a.n, a.R, A, static_cast<FT *>(a.V), chunk, a.loss,
                       a.loss_part);
    return hipGetLastError() == hipSuccess ? SPT_OK : SPT_EHIP;
}

template <int D, class FT>
static int launch_fused_d(const FusedArgs &a, const FactorSet<FT> &A, int G, int CPL) {
    switch (G * 16 + CPL) {
        case 4 * 16 + 4: return launch_fused_cfg<D, 4, 4, FT>(a, A);
        case 4 * 16 + 8: return launch_fused_cfg<D, 4, 8, FT>(a, A);
        case 8 * 16 + 1: return launch_fused_cfg<D, 8, 1, FT>(a, A);
        case 8 * 16 + 2: return launch_fused_cfg<D, 8, 2, FT>(a, A);
        case 8 * 16 + 4: return launch_fused_cfg<D, 8, 4, FT>(a, A);
        case 8 * 16 + 8: return launch_fused_cfg<D, 8, 8, FT>(a, A);
        case 16 * 16 + 1: return launch_fused_cfg<D, 16, 1, FT>(a, A);
        case 16 * 16 + 2: return launch_fused_cfg<D, 16, 2, FT>(a, A);
        case 16 * 16 + 4: return launch_fused_cfg<D, 16, 4, FT>(a, A);
        case 16 * 16 + 8: return launch_fused_cfg<D, 16, 8, FT>(a, A);
        case 32 * 16 + 1: return launch_fused_cfg<D, 32, 1, FT>(a, A);
        case 32 * 16 + 2: return launch_fused_cfg<D, 32, 2, FT>(a, A);
        case 32 * 16 + 4: return launch_fused_cfg<D, 32, 4, FT>(a, A);
        case 32 * 16 + 8: return launch_fused_cfg<D, 32, 8, FT>(a, A);
        case 64 * 16 + 1: return launch_fused_cfg<D, 64, 1, FT>(a, A);
        case 64 * 16 + 2: return launch_fused_cfg<D, 64, 2, FT>(a, A);
        case 64 * 16 + 4: return launch_fused_cfg<D, 64, 4, FT>(a, A);
        default: return SPT_EUNSUPPORTED;
    }
}

template <class FT>
static int launch_fused(const FusedArgs &a, int d, const void *const *factors, int G, int CPL) {
    FactorSet<FT> A{};
    for (int m = 0; m < d; ++m) A.p[m] = static_cast<const FT *>(factors[m]);
    switch (d) {
        case 2: return launch_fused_d<2, FT>(a, A, G, CPL);
        case 3: return launch_fused_d<3, FT>(a, A, G, CPL);
        case 4: return launch_fused_d<4, FT>(a, A, G, CPL);
        case 5: return launch_fused_d<5, FT>(a, A, G, CPL);
        default: return SPT_EUNSUPPORTED;
    }
}

// Default lane layout of the fused pass: the fewest lanes per entry (at least 4, at most 8
// columns each), since every entry ends in a butterfly over its lane group.  Measured on the
// 1e8-entry count tensor at R = 32: 4 x 8 lanes x columns 8.5 ms, 8 x 4 9.8 ms, 16 x 2 16.9 ms.
static bool gcp_layout(int R, int *G, int *CPL) {
    static const int ok[][2] = {{4, 4},  {4, 8},  {8, 1},  {8, 2},  {8, 4},  {8, 8},
                                {16, 1}, {16, 2}, {16, 4}, {16, 8}, {32, 1}, {32, 2},
                                {32, 4}, {32, 8}, {64, 1}, {64, 2}, {64, 4}};
    for (int c = 8; c >= 1; c >>= 1) {
        if (R % c != 0 || R / c < 4) continue;
        int g = 1;
        while (g < R / c) g <<= 1;
        for (const auto &e : ok)
            if (e[0] == g && e[1] == c) {
                *G = g;
                *CPL = c;
                return true;
            }
    }
    return false;
}

}  // namespace spt

using namespace spt;

extern "C" {

int spt_gcp_fused(const spt_tensor *X, int R, const void *const *factors, int fdtype,
                  int loss_kind, double *loss, void *const *grads, const double *gscale,
                  const spt_tune *tune, void *stream) {
    if (X == nullptr || R < 1 || R > 256 || loss == nullptr || grads == nullptr) return SPT_EINVAL;
    if (loss_kind < SPT_GCP_POISSON || loss_kind > SPT_GCP_GAMMA) return SPT_EINVAL;
    if (fdtype == SPT_F64) {
        if (X->vdtype != SPT_F64) return SPT_EUNSUPPORTED;
    } else if (fdtype == SPT_F32) {
        if (X->vdtype != SPT_F32) return SPT_EUNSUPPORTED;
    } else {
        return fdtype == SPT_BF16 ? SPT_EUNSUPPORTED : SPT_EINVAL;
    }
    int rc = check_factors(X, -1, factors);
    if (rc == SPT_OK) rc = check_factor_extent(X, -1, R, fdtype);
    if (rc) return rc;
    for (int n = 0; n < X->d; ++n) {
        if (grads[n] == nullptr) return SPT_EINVAL;
        if (!X->permuted[n]) return SPT_ESTATE;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int at = (fdtype == SPT_F64) ? 8 : 4;
    int64_t nparts = 0;
    for (int n = 0; n < X->d; ++n) {
        // the permuted layouts whatever algorithm the tune names (the pass is a permuted one)
        spt_tune tin = tune ? *tune : spt_tune{0, 0, 0, 0, 0, 0}, t;
        tin.algo = (X->srec[n] != nullptr) ? SPT_ALGO_PERMUTED_COPY : SPT_ALGO_PERMUTED;
        if (tin.flags & SPT_TUNE_DETERMINISTIC) return SPT_EUNSUPPORTED;
        if (tin.lanes_per_nnz == 0 && tin.cols_per_lane == 0) {
            int G, CPL;
            if (gcp_layout(R, &G, &CPL)) {
                tin.lanes_per_nnz = G;
                tin.cols_per_lane = CPL;
            }
        }
        rc = resolve_tune(X, n, R, fdtype, &tin, &t);
        if (rc) return rc;
        rc = zero_words(grads[n], X->dims[n] * (int64_t)R * at / 4, s);
        if (rc) return rc;
        if (X->P == 0) continue;
        int64_t chunk = t.nnz_per_wave;
        // one loss partial per wave chunk of mode 0, in the tensor's reduction scratch
        const int64_t minc = (ceil_div(X->P, (int64_t)kRedSlots) + 63) / 64 * 64;
        if (n == 0 && chunk < minc) chunk = minc;
        int64_t np = 0;
        FusedArgs a;
        a.auto_chunk = tune == nullptr || tune->nnz_per_wave == 0;
        a.min_chunk = (n == 0) ? (int)minc : 64;
        a.cus = device_cus();
        a.nparts = &np;
        a.rec = X->rec;
        a.srec = (t.algo == SPT_ALGO_PERMUTED_COPY) ? X->srec[n] : nullptr;
        a.perm = (a.srec != nullptr) ? X->sperm[n] : X->perm[n];
        a.P = X->P;
        a.n = n;
        a.R = R;
        a.chunk = (int)chunk;
        a.loss = loss_kind;
        a.V = grads[n];
        a.loss_part = (n == 0) ? X->red : nullptr;
        a.s = s;
        rc = (fdtype == SPT_F64) ? launch_fused<double>(a, X->d, factors, t.lanes_per_nnz, t.cols_per_lane)
                                 : launch_fused<float>(a, X->d, factors, t.lanes_per_nnz, t.cols_per_lane);
        if (rc) return rc;
        if (n == 0) nparts = np;
        if (gscale != nullptr) {
            const int64_t len = X->dims[n] * (int64_t)R;
            int64_t blocks = ceil_div(len, kBlock);
            if (blocks > 4096) blocks = 4096;
            if (fdtype == SPT_F64)
                hipLaunchKernelGGL(k_scale<double>, dim3((unsigned)blocks), dim3(kBlock), 0, s,
                                   static_cast<const double *>(grads[n]),
                                   static_cast<double *>(grads[n]), len, gscale);
            else
                hipLaunchKernelGGL(k_scale<float>, dim3((unsigned)blocks), dim3(kBlock), 0, s,
                                   static_cast<const float *>(grads[n]),
                                   static_cast<float *>(grads[n]), len, gscale);
            SPT_LAUNCH_CHECK();
        }
    }
    if (X->P == 0) return zero_words(loss, 2, s);
    hipLaunchKernelGGL(k_sum_loss, dim3(1), dim3(kWave), 0, s, X->red, nparts, loss);
    SPT_LAUNCH_CHECK();
    return SPT_OK;
}

int spt_scale_values(const void *src, void *dst, int64_t n, int dtype, const double *g,
                     void *stream) {
    if (n < 0 || g == nullptr || (n > 0 && (src == nullptr || dst == nullptr))) return SPT_EINVAL;
    if (dtype != SPT_F32 && dtype != SPT_F64) return SPT_EINVAL;
    if (n == 0) return SPT_OK;
    int64_t blocks = ceil_div(n, kBlock);
    if (blocks > 4096) blocks = 4096;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (dtype == SPT_F64)
        hipLaunchKernelGGL(k_scale<double>, dim3((unsigned)blocks), dim3(kBlock), 0, s,
                           static_cast<const double *>(src), static_cast<double *>(dst), n, g);
    else
        hipLaunchKernelGGL(k_scale<float>, dim3((unsigned)blocks), dim3(kBlock), 0, s,
                           static_cast<const float *>(src), static_cast<float *>(dst), n, g);
    return hipGetLastError() == hipSuccess ? SPT_OK : SPT_EHIP;
}

}  // extern "C"
