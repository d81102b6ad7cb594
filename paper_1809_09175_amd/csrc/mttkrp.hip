// Public MTTKRP entry point: argument checks, launch-parameter choice, output zeroing and
// dispatch to the per-dtype kernel instantiations.
#include <algorithm>

#include "mttkrp_kernels.h"

namespace spt {

// Zero n bytes (n a multiple of 4) with a kernel rather than a memset node, so the call can be
// captured in a HIP graph.
__global__ __launch_bounds__(kBlock) void k_zero(uint32_t *__restrict__ p, int64_t nwords) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    const int64_t nq = nwords / 4;
    uint4 *q = reinterpret_cast<uint4 *>(p);
    for (int64_t k = i; k < nq; k += stride) q[k] = make_uint4(0, 0, 0, 0);
    for (int64_t k = nq * 4 + i; k < nwords; k += stride) p[k] = 0;
}

int zero_words(void *p, int64_t nwords, hipStream_t s) {
    if (nwords <= 0) return SPT_OK;
    int64_t blocks = ceil_div(ceil_div(nwords, 4), kBlock);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(kBlock), 0, s,
                       static_cast<uint32_t *>(p), nwords);
    return hipGetLastError() == hipSuccess ? SPT_OK : SPT_EHIP;
}

// (lanes per entry, columns per lane) pairs with compiled kernels
static bool cfg_supported(int G, int CPL) {
    switch (G * 16 + CPL) {
        case 4 * 16 + 4: case 4 * 16 + 8:
        case 8 * 16 + 1: case 8 * 16 + 2: case 8 * 16 + 4: case 8 * 16 + 8:
        case 16 * 16 + 1: case 16 * 16 + 2: case 16 * 16 + 4: case 16 * 16 + 8:
        case 32 * 16 + 1: case 32 * 16 + 2: case 32 * 16 + 4: case 32 * 16 + 8:
        case 64 * 16 + 1: case 64 * 16 + 2: case 64 * 16 + 4:
            return true;
        default:
            return false;
    }
}

constexpr size_t kPrivatizedLds = 64 * 1024;

int device_cus() {
    static int cus = 0;
    if (cus == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus < 1)
            cus = 256;
    }
    return cus;
}

static int pow2_at_least(int x) {
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

// Default lane layout (lanes per entry x columns per lane), from measurements on MI355X
// (1e8-entry Zipf tensor, all three modes, each layout at its best unroll and chunk):
//   FP32  16 x 1 at R = 16, then four columns (sixteen bytes per lane): 8 x 4, 16 x 4, 32 x 4,
//         64 x 4 at R = 32, 64, 128, 256 (R = 128 / 256: 12.4 / 25.6 ms against 14.0 / 28.1
//         with 16 x 8 / 32 x 8);
//   BF16  one column below R = 16, two up to 32, then eight (sixteen bytes per lane): 8 x 2,
//         16 x 2, 8 x 8, 16 x 8, 32 x 8 at R = 16, 32, 64, 128, 256 (R = 16 / 64 / 128:
//         2.65 / 4.47 / 7.5 ms against 2.75-2.85 / 4.82 / 9.0 with 16 x 1 / 32 x 2 / 64 x 2);
//   FP64  four columns (32 bytes per lane) from R = 16: 4 x 4, 8 x 4, 16 x 4, 32 x 4 at R = 16,
//         32, 64, 128 (4.53 / 7.30 / 13.8 / 28.2 ms against 7.84 / 7.61 / 14.6 / 36.1 with
//         16 x 1 and the FP32 chunk rules at R <= 64, 16 x 8 at R = 128);
// over as many lanes as cover R.  The atomic kernel is fastest with one column per lane (its
// LDS and global atomics are per column either way).  Columns per lane must divide R.
static void default_layout(int R, int fdtype, int algo, int *G_out, int *cpl_out) {
    int cpl = 1, G = 8;
    if (algo == SPT_ALGO_PERMUTED) {
        int c = (fdtype == SPT_BF16)  ? (R < 16 ? 1 : (R <= 32 ? 2 : 8))
                : (fdtype == SPT_F64) ? (R < 16 ? 1 : 4)
                                      : (R < 32 ? 1 : 4);
        while (c > 1 && R % c != 0) c >>= 1;
        int g = pow2_at_least((R + c - 1) / c);
        const int gmin = (fdtype == SPT_F64 && c == 4) ? 4 : 8;
        if (g < gmin) g = gmin;
        if (cfg_supported(g, c)) {
            *G_out = g;
            *cpl_out = c;
            return;
        }
        const int opts[] = {8, 4, 2, 1};
        for (int c2 : opts) {
            if (R % c2 != 0 || R / c2 < 4) continue;
            g = pow2_at_least(R / c2);
            if (cfg_supported(g, c2)) {
                *G_out = g;
                *cpl_out = c2;
                return;
            }
        }
    }
    // one column per lane up to 64 columns, then wider lanes (R must then be even, and a
    // multiple of 4 above 128; other ranks are rejected by resolve_tune)
    if (R <= 64) {
        cpl = 1;
        G = pow2_at_least(R);
        if (G < 8) G = 8;
    } else if (R <= 128 && R % 8 == 0) {
        cpl = 8;
        G = 16;
    } else if (R <= 128) {
        cpl = 2;
        G = 64;
    } else {
        cpl = 4;
        G = 64;
    }
    *G_out = G;
    *cpl_out = cpl;
}

int resolve_tune(const spt_tensor *X, int mode, int R, int fdtype, const spt_tune *in,
                 spt_tune *out) {
    spt_tune t = in ? *in : spt_tune{0, 0, 0, 0, 0, 0};
    if (t.algo == SPT_ALGO_AUTO)
        t.algo = X->srec[mode] != nullptr ? SPT_ALGO_PERMUTED_COPY
                                          : (X->permuted[mode] ? SPT_ALGO_PERMUTED : SPT_ALGO_ATOMIC);
    if (t.algo != SPT_ALGO_ATOMIC && t.algo != SPT_ALGO_PERMUTED &&
        t.algo != SPT_ALGO_PERMUTED_COPY && t.algo != SPT_ALGO_PRIVATIZED)
        return SPT_EINVAL;
    const int lalgo = (t.algo == SPT_ALGO_ATOMIC || t.algo == SPT_ALGO_PRIVATIZED)
                          ? SPT_ALGO_ATOMIC : SPT_ALGO_PERMUTED;
    int G = t.lanes_per_nnz, cpl = t.cols_per_lane;
    if (G == 0 && cpl == 0) {
        default_layout(R, fdtype, lalgo, &G, &cpl);
    } else if (cpl == 0) {
        cpl = (R + G - 1) / G;
        while (cpl & (cpl - 1)) ++cpl;
    } else if (G == 0) {
        G = pow2_at_least((R + cpl - 1) / cpl);
        if (G < 4) G = 4;
    }
    if (cpl != 1 && cpl != 2 && cpl != 4 && cpl != 8) return SPT_EINVAL;
    if (R % cpl != 0) return SPT_EUNSUPPORTED;
    if (G * cpl < R || !cfg_supported(G, cpl)) return SPT_EUNSUPPORTED;
    if (t.nnz_per_wave == 0) {
        // long chunks amortise the chunk-boundary work, but a small tensor needs enough
        // wavefronts to occupy the GPU: aim for at least ~2048 wave chunks (the permuted launch
        // may then match the chunk to the device's resident wavefronts: capacity_chunk)
        t.flags |= kTuneChunkDefaulted;
        const int64_t cap = (lalgo != SPT_ALGO_PERMUTED) ? 2048
                            : (fdtype == SPT_F64 && R <= 32) ? 8192 : 4096;
        int64_t c = (X->P / 2048) & ~int64_t(63);
        t.nnz_per_wave = (int)(c < 256 ? 256 : (c > cap ? cap : c));
    }
    if (t.nnz_per_wave < 64 || t.nnz_per_wave % 64 != 0 || t.nnz_per_wave > (1 << 20))
        return SPT_EINVAL;
    if (t.lds_kib < 0 || t.lds_kib > 64) return SPT_EINVAL;
    if (t.algo == SPT_ALGO_PRIVATIZED) {
        // the whole output must fit one workgroup's LDS next to the record staging buffer,
        // within 64 KiB so two workgroups share a CU
        const size_t at = (fdtype == SPT_F64) ? 8 : 4;
        const size_t need =
            (size_t)(kBlock / kWave) * (kWave / G) * staged_group_stride(G, X->rec_words / 4) * 16 +
            (size_t)X->dims[mode] * G * cpl * at;
        if (need > kPrivatizedLds) return SPT_EUNSUPPORTED;
    }
    t.lanes_per_nnz = G;
    t.cols_per_lane = cpl;
    *out = t;
    return SPT_OK;
}

int launch_mttkrp(const spt_tensor *X, int mode, int R, const void *const *factors, int fdtype,
                  const double *lambda, const void *vals, void *V, const spt_tune &t,
                  hipStream_t s) {
    const int at_bytes = (fdtype == SPT_F64) ? 8 : 4;
    int rc = zero_words(V, X->dims[mode] * (int64_t)R * at_bytes / 4, s);
    if (rc) return rc;
    if (X->P == 0) return SPT_OK;
    MttkrpArgs a;
    a.rec = X->rec;
    a.srec = (t.algo == SPT_ALGO_PERMUTED_COPY) ? X->srec[mode] : nullptr;
    a.perm = (a.srec != nullptr) ? X->sperm[mode] : X->perm[mode];
    a.P = X->P;
    a.n = mode;
    a.R = R;
    a.lambda = lambda;
    a.vovr = vals;
    a.V = V;
    a.chunk = t.nnz_per_wave;
    a.algo = t.algo;
    a.slot_keys = nullptr;
    a.slot_vals = nullptr;
    a.In = (int)X->dims[mode];
    a.auto_chunk = (t.flags & kTuneChunkDefaulted) != 0;
    a.cus = device_cus();
    a.query_chunk = nullptr;
    a.privatized = 0;
    if (t.algo == SPT_ALGO_PRIVATIZED) {
        // privatised output: about two workgroups per CU, each adding a long contiguous range
        // into its LDS copy of V, so every row is flushed to HBM only once per workgroup
        a.algo = SPT_ALGO_ATOMIC;
        a.privatized = 1;
        int64_t blocks = 2 * (int64_t)device_cus();
        const int64_t minb = ceil_div(X->P, (int64_t)(kBlock / kWave) * 64);
        if (blocks > minb) blocks = minb;
        int64_t ch = ceil_div(ceil_div(X->P, blocks * (kBlock / kWave)), 64) * 64;
        a.chunk = (int)(ch < 64 ? 64 : ch);
    }
    if ((t.flags & SPT_TUNE_DETERMINISTIC) &&
        (t.algo == SPT_ALGO_PERMUTED || t.algo == SPT_ALGO_PERMUTED_COPY)) {
        // the boundary slots live in the radix-sort scratch (two P-entry int32 arrays), free
        // once the permutations exist; chunks are lengthened until they fit
        const size_t avail = 2 * align256((size_t)X->P * 4);
        int64_t chunk = a.chunk;
        for (;;) {
            const int64_t ns = 2 * ceil_div(X->P, chunk);
            if (align256((size_t)ns * 4) + (size_t)ns * R * at_bytes <= avail) break;
            chunk *= 2;
        }
        a.chunk = (int)chunk;
        const int64_t ns = 2 * ceil_div(X->P, chunk);
        a.slot_keys = X->tmp_keys;
        a.slot_vals = reinterpret_cast<uint8_t *>(X->tmp_keys) + align256((size_t)ns * 4);
    }
    a.stream = s;
    switch (fdtype) {
        case SPT_F64: return launch_mttkrp_f64(a, X->d, factors, t.lanes_per_nnz, t.cols_per_lane);
        case SPT_F32: return launch_mttkrp_f32(a, X->d, factors, t.lanes_per_nnz, t.cols_per_lane);
        case SPT_BF16:
            return launch_mttkrp_bf16(a, X->d, factors, t.lanes_per_nnz, t.cols_per_lane);
        default: return SPT_EINVAL;
    }
}

static int check_dtypes(const spt_tensor *X, int fdtype) {
    if (fdtype == SPT_F64) return X->vdtype == SPT_F64 ? SPT_OK : SPT_EUNSUPPORTED;
    if (fdtype == SPT_F32 || fdtype == SPT_BF16)
        return X->vdtype == SPT_F32 ? SPT_OK : SPT_EUNSUPPORTED;
    return SPT_EINVAL;
}

int check_factors(const spt_tensor *X, int skip_mode, const void *const *factors) {
    if (factors == nullptr) return SPT_EINVAL;
    if (X->appended != X->P) return SPT_ESTATE;  // entries still to be appended
    for (int m = 0; m < X->d; ++m)
        if (m != skip_mode && factors[m] == nullptr) return SPT_EINVAL;
    return SPT_OK;
}

// The kernels address factor rows with 32-bit byte offsets from the matrix base, so every
// matrix they gather from (all but skip_mode's; -1 = all) must be smaller than 4 GiB.
int check_factor_extent(const spt_tensor *X, int skip_mode, int R, int fdtype) {
    const uint64_t fbytes = fdtype == SPT_F64 ? 8 : (fdtype == SPT_BF16 ? 2 : 4);
    for (int m = 0; m < X->d; ++m)
        if (m != skip_mode && (uint64_t)X->dims[m] * (uint64_t)R * fbytes >= (1ull << 32))
            return SPT_EUNSUPPORTED;
    return SPT_OK;
}

int check_mttkrp_args(const spt_tensor *X, int mode, int R, const void *const *factors,
                      int fdtype, const void *V) {
    if (X == nullptr || mode < 0 || mode >= X->d || R < 1 || R > 256 || V == nullptr)
        return SPT_EINVAL;
    int rc = check_factors(X, mode, factors);
    if (rc) return rc;
    rc = check_dtypes(X, fdtype);
    if (rc) return rc;
    return check_factor_extent(X, mode, R, fdtype);
}

}  // namespace spt

using namespace spt;

extern "C" int spt_mttkrp(const spt_tensor *X, int mode, int R, const void *const *factors,
                          int fdtype, const double *lambda, const void *vals, void *V,
                          const spt_tune *tune, void *stream) {
    int rc = check_mttkrp_args(X, mode, R, factors, fdtype, V);
    if (rc) return rc;
    spt_tune t;
    rc = resolve_tune(X, mode, R, fdtype, tune, &t);
    if (rc) return rc;
    if (t.algo == SPT_ALGO_PERMUTED && !X->permuted[mode]) return SPT_ESTATE;
    if (t.algo == SPT_ALGO_PERMUTED_COPY && X->srec[mode] == nullptr) return SPT_ESTATE;
    return launch_mttkrp(X, mode, R, factors, fdtype, lambda, vals, V, t,
                         static_cast<hipStream_t>(stream));
}

extern "C" int spt_mttkrp_default_tune(const spt_tensor *X, int mode, int R, int fdtype,
                                       int algo, spt_tune *out) {
    if (X == nullptr || out == nullptr || mode < 0 || mode >= X->d || R < 1 || R > 256)
        return SPT_EINVAL;
    spt_tune in{algo, 0, 0, 0, 0};
    int rc = resolve_tune(X, mode, R, fdtype, &in, out);
    if (rc) return rc;
    if ((out->flags & kTuneChunkDefaulted) && X->P > 0 && out->algo == SPT_ALGO_PERMUTED_COPY) {
        // report the chunk the launch will use (no launch: a query of the dispatch)
        MttkrpArgs a{};
        int chunk = out->nnz_per_wave;
        a.P = X->P;
        a.R = R;
        a.n = mode;
        a.chunk = out->nnz_per_wave;
        a.algo = out->algo;
        a.auto_chunk = 1;
        a.cus = device_cus();
        a.query_chunk = &chunk;
        a.srec = X->srec[mode];
        const void *none[SPT_MAX_ORDER] = {nullptr, nullptr, nullptr, nullptr, nullptr};
        switch (fdtype) {
            case SPT_F64: rc = launch_mttkrp_f64(a, X->d, none, out->lanes_per_nnz, out->cols_per_lane); break;
            case SPT_F32: rc = launch_mttkrp_f32(a, X->d, none, out->lanes_per_nnz, out->cols_per_lane); break;
            case SPT_BF16: rc = launch_mttkrp_bf16(a, X->d, none, out->lanes_per_nnz, out->cols_per_lane); break;
            default: rc = SPT_EINVAL;
        }
        if (rc) return rc;
        out->nnz_per_wave = chunk;
    }
    out->flags &= ~kTuneChunkDefaulted;
    return SPT_OK;
}

// ------------------------------------------------------------------------------------------
// autotuner: time every candidate launch configuration on the device and keep the fastest
// ------------------------------------------------------------------------------------------

extern "C" int spt_batch_supported_tune(int d, int fdtype, int algo, int lanes_per_nnz,
                                        int cols_per_lane);

extern "C" int spt_paper_block_sizes(int R, int *vector_size, int *fbs) {
    // GPU vector and factor block sizes by rank for the register-array MTTKRP (Tab. sizes)
    static const int lo[] = {1, 2, 3, 4, 5, 8, 9, 17, 25, 48, 49, 96, 97};
    static const int vs[] = {1, 2, 2, 4, 4, 8, 8, 8, 8, 16, 16, 32, 32};
    static const int fb[] = {1, 2, 4, 4, 8, 8, 16, 24, 32, 48, 64, 96, 128};
    if (R < 1 || vector_size == nullptr || fbs == nullptr) return SPT_EINVAL;
    int k = 0;
    for (int i = 0; i < 13; ++i)
        if (R >= lo[i]) k = i;
    *vector_size = vs[k];
    *fbs = fb[k];
    return SPT_OK;
}

constexpr int kTuneDefaultReps = 7;
constexpr int kTuneMaxReps = 64;

// Median time of `reps` individually timed launches of configuration r (after one untimed
// launch): single launches of a small MTTKRP last microseconds, so one slow launch (a cold
// cache, a clock step) must not decide the choice.
static int time_config(const spt_tensor *X, int mode, int R, const void *const *factors,
                       int fdtype, void *V, const spt_tune &r, int reps, hipEvent_t *ev,
                       hipStream_t s, float *ms_out) {
    int rc = launch_mttkrp(X, mode, R, factors, fdtype, nullptr, nullptr, V, r, s);
    if (rc) return rc;
    float t[kTuneMaxReps];
    for (int k = 0; k < reps; ++k) {
        if (hipEventRecord(ev[2 * k], s) != hipSuccess) return SPT_EHIP;
        rc = launch_mttkrp(X, mode, R, factors, fdtype, nullptr, nullptr, V, r, s);
        if (rc) return rc;
        if (hipEventRecord(ev[2 * k + 1], s) != hipSuccess) return SPT_EHIP;
    }
    if (hipEventSynchronize(ev[2 * reps - 1]) != hipSuccess) return SPT_EHIP;
    for (int k = 0; k < reps; ++k)
        if (hipEventElapsedTime(&t[k], ev[2 * k], ev[2 * k + 1]) != hipSuccess) return SPT_EHIP;
    std::sort(t, t + reps);
    *ms_out = (reps % 2) ? t[reps / 2] : 0.5f * (t[reps / 2 - 1] + t[reps / 2]);
    return SPT_OK;
}

extern "C" int spt_mttkrp_autotune(const spt_tensor *X, int mode, int R,
                                   const void *const *factors, int fdtype, void *V, int flags,
                                   int reps, spt_tune *best, float *best_ms, void *stream) {
    int rc = check_mttkrp_args(X, mode, R, factors, fdtype, V);
    if (rc) return rc;
    if (best == nullptr) return SPT_EINVAL;
    if (reps < 1) reps = kTuneDefaultReps;
    if (reps > kTuneMaxReps) reps = kTuneMaxReps;
    hipStream_t s = static_cast<hipStream_t>(stream);
    static const int cfgs[][2] = {{4, 4},  {4, 8},  {8, 1},  {8, 2},  {8, 4},  {8, 8},
                                  {16, 1}, {16, 2}, {16, 4}, {16, 8}, {32, 1}, {32, 2},
                                  {32, 4}, {32, 8}, {64, 1}, {64, 2}, {64, 4}};
    static const int chunks[] = {512, 1024, 2048, 4096};
    const bool batch_only = (flags & SPT_TUNE_BATCH_CONFIGS) != 0;
    hipEvent_t ev[2 * kTuneMaxReps];
    int nev = 0;
    for (; nev < 2 * reps; ++nev)
        if (hipEventCreate(&ev[nev]) != hipSuccess) break;
    if (nev < 2 * reps) {
        for (int k = 0; k < nev; ++k) hipEventDestroy(ev[k]);
        return SPT_EHIP;
    }
    float bms = 1e30f;
    spt_tune bt{0, 0, 0, 0, 0};
    int tried = 0;
    rc = SPT_OK;
    auto consider = [&](const spt_tune &r) {
        float ms = 0.f;
        rc = time_config(X, mode, R, factors, fdtype, V, r, reps, ev, s, &ms);
        if (rc) return;
        ++tried;
        if (ms < bms) {
            bms = ms;
            bt = r;
        }
    };
    // the library's own default first: its layout and the chunk its launch really uses (which
    // may be matched to the device's resident wavefronts), whenever the flags allow it
    {
        spt_tune r;
        if (spt_mttkrp_default_tune(X, mode, R, fdtype, SPT_ALGO_AUTO, &r) == SPT_OK) {
            const bool is_perm = r.algo != SPT_ALGO_ATOMIC && r.algo != SPT_ALGO_PRIVATIZED;
            const bool allowed =
                !(is_perm && (flags & SPT_TUNE_NO_PERMUTED)) &&
                !(!is_perm && (flags & SPT_TUNE_NO_ATOMIC)) &&
                !(batch_only && !spt_batch_supported_tune(X->d, fdtype, r.algo, r.lanes_per_nnz,
                                                          r.cols_per_lane));
            if (allowed) consider(r);
        }
    }
    for (int algo = SPT_ALGO_ATOMIC; algo <= SPT_ALGO_PRIVATIZED && rc == SPT_OK; ++algo) {
        if (algo == SPT_ALGO_PRIVATIZED && (batch_only || (flags & SPT_TUNE_NO_ATOMIC))) continue;
        if (algo == SPT_ALGO_PERMUTED && (!X->permuted[mode] || (flags & SPT_TUNE_NO_PERMUTED)))
            continue;
        if (algo == SPT_ALGO_PERMUTED_COPY &&
            (X->srec[mode] == nullptr || (flags & SPT_TUNE_NO_PERMUTED)))
            continue;
        if (algo == SPT_ALGO_ATOMIC && (flags & SPT_TUNE_NO_ATOMIC)) continue;
        for (const auto &c : cfgs) {
            const int G = c[0], CPL = c[1];
            // lanes must cover R; skip layouts that leave more than half the lanes idle
            if (G * CPL < R || R % CPL != 0) continue;
            if (G * CPL >= 2 * R && G * CPL > 16) continue;
            if (batch_only && !spt_batch_supported_tune(X->d, fdtype, algo, G, CPL)) continue;
            for (int chunk : chunks) {
                if (algo == SPT_ALGO_PRIVATIZED && chunk != chunks[0]) break;  // chunk is derived
                spt_tune t{algo, G, CPL, chunk, 0}, r;
                if (resolve_tune(X, mode, R, fdtype, &t, &r) != SPT_OK) continue;
                consider(r);
                if (rc) break;
            }
            if (rc) break;
        }
    }
    for (int k = 0; k < nev; ++k) hipEventDestroy(ev[k]);
    if (rc) return rc;
    if (tried == 0) return SPT_EUNSUPPORTED;
    *best = bt;
    if (best_ms) *best_ms = bms;
    return SPT_OK;
}
