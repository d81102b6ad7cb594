// Batched MTTKRP: many (tensor, mode) products, each with its own launch parameters, in one
// persistent kernel that workgroups feed from a global work counter, captured with the output
// zeroing in one HIP graph.  Plus the autotuner that picks each product's parameters by timing
// the candidates on the device.
#include <string.h>

#include <new>
#include <vector>

#include "mttkrp_kernels.h"

namespace spt {

struct BatchItem {
    const int4 *rec;
    const int32_t *perm;
    const int4 *srec;   // mode-sorted record copy or null
    const void *A[SPT_MAX_ORDER];
    void *V;
    int64_t P;
    int64_t unit0;   // first work unit of this item (a unit = 4 wave chunks = one workgroup)
    int64_t vwords;  // 32-bit words of V
    int32_t n, R, cfg, chunk;
};

// (algo, order, lanes per entry, columns per lane) combinations compiled into the batched
// kernel; each product's tuned parameters are mapped onto one of them
#define SPT_BATCH_CONFIGS(X)                 \
    X(0, SPT_ALGO_PERMUTED, 3, 4, 4)         \
    X(1, SPT_ALGO_PERMUTED, 3, 8, 2)         \
    X(2, SPT_ALGO_PERMUTED, 3, 8, 4)         \
    X(3, SPT_ALGO_PERMUTED, 3, 16, 2)        \
    X(4, SPT_ALGO_PERMUTED, 3, 16, 4)        \
    X(5, SPT_ALGO_ATOMIC, 3, 8, 2)           \
    X(6, SPT_ALGO_ATOMIC, 3, 8, 4)           \
    X(7, SPT_ALGO_ATOMIC, 3, 16, 2)          \
    X(8, SPT_ALGO_ATOMIC, 3, 16, 4)          \
    X(9, SPT_ALGO_PERMUTED, 3, 8, 1)         \
    X(10, SPT_ALGO_PERMUTED, 3, 16, 1)

struct BatchCfg {
    int algo, d, G, CPL;
};
static const BatchCfg kBatchCfgs[] = {
#define SPT_CFG_ROW(i, a, d, g, c) {a, d, g, c},
    SPT_BATCH_CONFIGS(SPT_CFG_ROW)
#undef SPT_CFG_ROW
};
constexpr int kNumBatchCfgs = sizeof(kBatchCfgs) / sizeof(kBatchCfgs[0]);

// The batched kernel holds every configuration's code, so its register allocation is the
// largest of them.  It runs with an unroll of 2 under a 4-waves-per-SIMD register cap (128
// VGPRs): on the 64-tensor batch that beat unrolls 1 and 4, capped or not (1.13 ms against
// 1.25-1.50 ms), the few spills it costs included.
constexpr int kBatchUnroll = 2;

template <int ALGO, int D, int G, int CPL, class FT>
__device__ __forceinline__ void batch_unit(int4 *smem4, const BatchItem &it, int64_t u) {
    FactorSet<FT> A{};
#pragma unroll
    for (int m = 0; m < D; ++m) A.p[m] = static_cast<const FT *>(it.A[m]);
    const int64_t bc0 = (u - it.unit0) * (kBlock / kWave) * it.chunk;
    float *V = static_cast<float *>(it.V);
    if constexpr (ALGO == SPT_ALGO_PERMUTED) {
        using SM = PermShared<D, G, CPL, float, float>;
        static_assert(sizeof(SM) == perm_shared_bytes(G, CPL, SM::RQ, 4),
                      "the dynamic LDS is sized with perm_shared_bytes");
        SM *sm = reinterpret_cast<SM *>(smem4);
        const int wave = threadIdx.x >> 6;
        const int64_t c0 = bc0 + (int64_t)wave * it.chunk;
        if (c0 < it.P)
            perm_wave_chunk<D, G, CPL, FT, float, float, kBatchUnroll>(sm[wave], it.rec, it.perm, it.srec, it.P, it.n,
                                                         it.R, A, nullptr, nullptr, V, it.chunk, c0);
    } else {
        using SM = AtomicTileShared<D, G, CPL, float, float>;
        const int64_t bc1 = bc0 + (int64_t)(kBlock / kWave) * it.chunk;
        atomic_tile_range<D, G, CPL, FT, float, float, kBatchUnroll>(
            *reinterpret_cast<SM *>(smem4), it.rec, it.n, it.R, A, nullptr, nullptr, V, bc0,
            bc1 < it.P ? bc1 : it.P);
    }
}

// ATOMIC = false compiles the permuted configurations only: the atomic path's tile sort raises
// the kernel's register demand, so a batch whose products are all permuted runs the lighter
// kernel (4 waves per SIMD); with the atomic path the kernel may take 2 waves per SIMD's
// registers instead of spilling.
template <class FT, bool ATOMIC>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(ATOMIC ? 2 : 4, 8))) void k_mttkrp_batched(const BatchItem *__restrict__ items,
                                                           int nitems, int64_t total_units,
                                                           unsigned long long *counter) {
    extern __shared__ int4 smem4[];
    __shared__ long long s_unit;
    for (;;) {
        if (threadIdx.x == 0) s_unit = (long long)atomicAdd(counter, 1ull);
        __syncthreads();
        const int64_t u = s_unit;
        if (u >= total_units) break;  // uniform: every thread read the same unit
        int lo = 0, hi = nitems - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (items[mid].unit0 <= u) lo = mid;
            else hi = mid - 1;
        }
        lo = __builtin_amdgcn_readfirstlane(lo);
        const BatchItem &it = items[lo];
        switch (it.cfg) {
#define SPT_CFG_CASE(i, a, d, g, c)                                   \
    case i:                                                           \
        if constexpr (ATOMIC || (a) == SPT_ALGO_PERMUTED)               \
            batch_unit<a, d, g, c, FT>(smem4, it, u);                 \
        break;
            SPT_BATCH_CONFIGS(SPT_CFG_CASE)
#undef SPT_CFG_CASE
            default: break;
        }
        __syncthreads();
    }
}

// zero every output and the work counter (a kernel, not a memset node, so replays are exact)
__global__ __launch_bounds__(kBlock) void k_batch_zero(const BatchItem *__restrict__ items,
                                                       unsigned long long *counter) {
    const BatchItem &it = items[blockIdx.y];
    uint32_t *p = static_cast<uint32_t *>(it.V);
    const int64_t n = it.vwords;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        p[i] = 0u;
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *counter = 0ull;
}

}  // namespace spt

using namespace spt;

struct spt_batch {
    int nitems;
    int fdtype;
    int64_t total_units;
    BatchItem *d_items;
    unsigned long long *d_counter;
    size_t smem;
    int zero_blocks;
    hipStream_t capture_stream;
    hipGraph_t graph;
    hipGraphExec_t exec;
};

static int batch_cfg_index(int algo, int d, int G, int CPL) {
    for (int i = 0; i < kNumBatchCfgs; ++i)
        if (kBatchCfgs[i].algo == algo && kBatchCfgs[i].d == d && kBatchCfgs[i].G == G &&
            kBatchCfgs[i].CPL == CPL)
            return i;
    return -1;
}

static size_t batch_smem_for(int cfg) {
    switch (cfg) {
#define SPT_CFG_SMEM(i, a, d, g, c)                                                       \
    case i:                                                                               \
        return (a) == SPT_ALGO_PERMUTED                                                   \
                   ? (size_t)(kBlock / kWave) * perm_shared_bytes(g, c, 1, 4)             \
                   : atomic_tile_smem_bytes<d, g, c, float, float>();
        SPT_BATCH_CONFIGS(SPT_CFG_SMEM)
#undef SPT_CFG_SMEM
        default: return 0;
    }
}

extern "C" {

int spt_batch_supported_tune(int d, int fdtype, int algo, int lanes_per_nnz, int cols_per_lane) {
    if (fdtype != SPT_F32 && fdtype != SPT_BF16) return 0;
    if (algo == SPT_ALGO_PERMUTED_COPY) algo = SPT_ALGO_PERMUTED;
    return batch_cfg_index(algo, d, lanes_per_nnz, cols_per_lane) >= 0;
}

size_t spt_batch_workspace_bytes(int nitems) {
    if (nitems < 1) return 0;
    return align256((size_t)nitems * sizeof(BatchItem)) + 256;
}

int spt_batch_create(spt_batch **out, int nitems, const spt_tensor *const *tensors,
                     const int *modes, const int *ranks, const void *const *const *factors,
                     int fdtype, void *const *outputs, const spt_tune *tunes, void *ws,
                     size_t ws_bytes, void *stream) {
    if (out == nullptr) return SPT_EINVAL;
    *out = nullptr;
    if (nitems < 1 || tensors == nullptr || modes == nullptr || ranks == nullptr ||
        factors == nullptr || outputs == nullptr || tunes == nullptr)
        return SPT_EINVAL;
    if (fdtype != SPT_F32 && fdtype != SPT_BF16) return SPT_EUNSUPPORTED;
    if (ws == nullptr || ((uintptr_t)ws & 255u) || ws_bytes < spt_batch_workspace_bytes(nitems))
        return SPT_EWORKSPACE;
    std::vector<BatchItem> h(nitems);
    int64_t units = 0;
    bool any_atomic = false;
    size_t smem = 0;
    for (int i = 0; i < nitems; ++i) {
        const spt_tensor *X = tensors[i];
        const int n = modes[i], R = ranks[i];
        int rc = check_mttkrp_args(X, n, R, factors[i], fdtype, outputs[i]);
        if (rc) return rc;
        spt_tune t;
        rc = resolve_tune(X, n, R, fdtype, &tunes[i], &t);
        if (rc) return rc;
        if (t.algo == SPT_ALGO_PERMUTED && !X->permuted[n]) return SPT_ESTATE;
        if (t.algo == SPT_ALGO_PERMUTED_COPY && X->srec[n] == nullptr) return SPT_ESTATE;
        if (t.flags & SPT_TUNE_DETERMINISTIC) return SPT_EUNSUPPORTED;
        const int kalgo = (t.algo == SPT_ALGO_PERMUTED_COPY) ? SPT_ALGO_PERMUTED : t.algo;
        const int cfg = batch_cfg_index(kalgo, X->d, t.lanes_per_nnz, t.cols_per_lane);
        any_atomic = any_atomic || kalgo == SPT_ALGO_ATOMIC;
        if (cfg < 0) return SPT_EUNSUPPORTED;
        BatchItem &b = h[i];
        memset(&b, 0, sizeof b);
        b.rec = X->rec;
        b.srec = (t.algo == SPT_ALGO_PERMUTED_COPY) ? X->srec[n] : nullptr;
        b.perm = (b.srec != nullptr) ? X->sperm[n] : X->perm[n];
        for (int m = 0; m < X->d; ++m) b.A[m] = factors[i][m];
        b.V = outputs[i];
        b.P = X->P;
        b.unit0 = units;
        b.vwords = X->dims[n] * (int64_t)R;
        b.n = n;
        b.R = R;
        b.cfg = cfg;
        b.chunk = t.nnz_per_wave;
        const size_t sm = batch_smem_for(cfg);
        smem = sm > smem ? sm : smem;
        units += ceil_div(X->P, (int64_t)(kBlock / kWave) * t.nnz_per_wave);
    }
    spt_batch *B = new (std::nothrow) spt_batch;
    if (!B) return SPT_EINVAL;
    memset(B, 0, sizeof *B);
    B->nitems = nitems;
    B->fdtype = fdtype;
    B->total_units = units;
    B->d_items = static_cast<BatchItem *>(ws);
    B->d_counter = reinterpret_cast<unsigned long long *>(
        static_cast<uint8_t *>(ws) + align256((size_t)nitems * sizeof(BatchItem)));
    B->smem = smem;
    B->zero_blocks = 64;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int rc = SPT_EHIP;
    if (hipMemcpyAsync(B->d_items, h.data(), (size_t)nitems * sizeof(BatchItem),
                       hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess ||
        hipStreamCreateWithFlags(&B->capture_stream, hipStreamNonBlocking) != hipSuccess) {
        delete B;
        return SPT_EHIP;
    }
    // capture: zero outputs and counter, then the persistent kernel
    int dev = 0, cus = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    int per_cu = 0;
    hipError_t oe = hipSuccess;
    const void *kfn = fdtype == SPT_F32
                          ? (any_atomic ? (const void *)k_mttkrp_batched<float, true>
                                        : (const void *)k_mttkrp_batched<float, false>)
                          : (any_atomic ? (const void *)k_mttkrp_batched<uint16_t, true>
                                        : (const void *)k_mttkrp_batched<uint16_t, false>);
    oe = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, kBlock, smem);
    if (oe != hipSuccess || per_cu < 1) per_cu = 1;
    int64_t grid = (int64_t)cus * per_cu;
    if (grid > units) grid = units;
    if (grid < 1) grid = 1;
    if (hipStreamBeginCapture(B->capture_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
        goto fail;
    hipLaunchKernelGGL(k_batch_zero, dim3(B->zero_blocks, nitems), dim3(kBlock), 0,
                       B->capture_stream, B->d_items, B->d_counter);
    {
        void *args[] = {&B->d_items, &nitems, &units, &B->d_counter};
        if (hipLaunchKernel(kfn, dim3((unsigned)grid), dim3(kBlock), args, smem,
                            B->capture_stream) != hipSuccess)
            goto fail;
    }
    if (hipStreamEndCapture(B->capture_stream, &B->graph) != hipSuccess) goto fail;
    if (hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0) != hipSuccess) goto fail;
    *out = B;
    return SPT_OK;
fail:
    if (B->graph) hipGraphDestroy(B->graph);
    hipStreamDestroy(B->capture_stream);
    delete B;
    return rc;
}

int spt_batch_launch(spt_batch *B, void *stream) {
    if (B == nullptr) return SPT_EINVAL;
    return hipGraphLaunch(B->exec, static_cast<hipStream_t>(stream)) == hipSuccess ? SPT_OK
                                                                                    : SPT_EHIP;
}

int spt_batch_info(const spt_batch *B, int64_t *units, int *grid_smem_bytes) {
    if (B == nullptr) return SPT_EINVAL;
    if (units) *units = B->total_units;
    if (grid_smem_bytes) *grid_smem_bytes = (int)B->smem;
    return SPT_OK;
}

int spt_batch_destroy(spt_batch *B) {
    if (B == nullptr) return SPT_OK;
    if (B->exec) hipGraphExecDestroy(B->exec);
    if (B->graph) hipGraphDestroy(B->graph);
    if (B->capture_stream) hipStreamDestroy(B->capture_stream);
    delete B;
    return SPT_OK;
}

}  // extern "C"
