// Internal declarations shared by the HIP translation units of libspt (never installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spt.h"

#define SPT_MAX_ORDER 5

// Device status word block at the start of every tensor workspace.
struct SptStatusBlock {
    int32_t code;       // 0 or a negative spt_status raised on the device
    int32_t pad;
    int64_t bad_entry;  // smallest entry index with an out-of-range subscript (INT64_MAX: none)
};

struct spt_tensor {
    int d;
    int64_t dims[SPT_MAX_ORDER];
    int64_t P;
    int vdtype;          // SPT_F64 or SPT_F32
    int rec_words;       // 4 (16-byte records) or 8 (32-byte records)
    uint8_t *ws;
    size_t ws_bytes;
    SptStatusBlock *status;
    int4 *rec;           // P packed records: subscripts in words 0..d-1, value in the last word(s)
    int32_t *perm[SPT_MAX_ORDER];
    int32_t *skey[SPT_MAX_ORDER];
    int4 *srec[SPT_MAX_ORDER];  // optional mode-sorted record copies (caller workspace)
    const int32_t *sperm[SPT_MAX_ORDER];  // storage position of each record of srec[n]
    int32_t *tmp_keys;   // radix-sort ping-pong buffers
    int32_t *tmp_vals;
    uint32_t *hist;      // 256 x ntiles digit counts, scanned in place
    uint32_t *scan_part; // per-segment partial sums of the counts scan
    double *red;         // reduction scratch (fit, loss): kRedSlots doubles
    int permuted[SPT_MAX_ORDER];
    uint32_t *hist0;     // first-pass digit counts of every mode (256 x ntiles each), filled
                         // while packing
    int64_t appended;    // entries packed so far (spt_tensor_append); all P once created
    double xx;           // ||X||^2 of the stored values, once xx_valid (the values never change)
    int xx_valid;
};

namespace spt {

constexpr int kWave = 64;
constexpr int kBlock = 256;            // 4 waves
constexpr int kSortItems = 8;                       // keys per thread and sub-tile
constexpr int kSortSub = kBlock * kSortItems;        // elements of one sub-tile
constexpr int kSortSubs = 4;                         // sub-tiles one workgroup walks in order
constexpr int kSortTile = kSortSub * kSortSubs;      // elements per workgroup (one digit-count column)
constexpr int kScanSeg = kBlock * 8;
constexpr int kRedSlots = 8192;

inline int rec_words_for(int d, int vdtype) {
    int vbytes = (vdtype == SPT_F64) ? 8 : 4;
    return (d * 4 + vbytes <= 16) ? 4 : 8;
}

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// factor matrix pointers passed by value to kernels
template <class FT>
struct FactorSet {
    const FT *p[SPT_MAX_ORDER];
};

// status helpers
#define SPT_HIP(call)                                  \
    do {                                               \
        hipError_t e_ = (call);                        \
        if (e_ != hipSuccess) return SPT_EHIP;         \
    } while (0)

#define SPT_LAUNCH_CHECK() SPT_HIP(hipGetLastError())

// ------------------------------------------------------------------------------------------
// device helpers
// ------------------------------------------------------------------------------------------

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ float bf16_bits_to_f32(uint32_t h) {
    return __uint_as_float(h << 16);
}

// FP32 -> BF16, round to nearest even; NaN -> quiet NaN keeping sign and top payload bits.
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
    uint32_t x = __float_as_uint(f);
    if ((x & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((x >> 16) | 0x0040u);
    uint32_t lsb = (x >> 16) & 1u;
    return (uint16_t)((x + 0x7fffu + lsb) >> 16);
}

// FP64 -> BF16, round to nearest even in one rounding.  The value is first narrowed to FP32
// with round-to-odd (toward zero, then the last bit set when anything was cut off); FP32 carries
// 16 more bits than BF16 at every exponent, subnormals included, so the following
// round-to-nearest-even to BF16 gives the correctly rounded result of the original double
// (Boldo and Melquiond's round-to-odd rule).  NaN -> the quiet NaN 0x7fc0 with the sign.
__device__ __forceinline__ uint16_t f64_to_bf16_rne(double v) {
    if (v != v) return (uint16_t)(((uint64_t)__double_as_longlong(v) >> 48 & 0x8000u) | 0x7fc0u);
    uint32_t b = __float_as_uint((float)v);
    if (fabs((double)__uint_as_float(b)) > fabs(v)) b -= 1u;  // magnitude one step toward zero
    if ((double)__uint_as_float(b) != v) b |= 1u;
    return f32_to_bf16_rne(__uint_as_float(b));
}

__device__ __forceinline__ void atomic_add_f(float *p, float v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void atomic_add_f(double *p, double v) { unsafeAtomicAdd(p, v); }

__device__ __forceinline__ void raise_status(SptStatusBlock *s, int code) {
    atomicCAS(&s->code, 0, code);
}

// ------------------------------------------------------------------------------------------
// host-side entry points implemented in the individual translation units
// ------------------------------------------------------------------------------------------

int launch_mttkrp(const spt_tensor *X, int mode, int R, const void *const *factors, int fdtype,
                  const double *lambda, const void *vals, void *V, const spt_tune &tune,
                  hipStream_t s);
int resolve_tune(const spt_tensor *X, int mode, int R, int fdtype, const spt_tune *in,
                 spt_tune *out);
int zero_words(void *p, int64_t nwords, hipStream_t s);
int check_factors(const spt_tensor *X, int skip_mode, const void *const *factors);
int check_factor_extent(const spt_tensor *X, int skip_mode, int R, int fdtype);
int check_mttkrp_args(const spt_tensor *X, int mode, int R, const void *const *factors,
                      int fdtype, const void *V);

}  // namespace spt
