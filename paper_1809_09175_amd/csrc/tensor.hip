// COO tensor storage for libspt: packing of the caller's subscripts and values into records,
// and the per-mode permutations of Sec. 6 built by a stable LSD radix sort (8-bit digits,
// reduce-then-scan, LDS ranking with wavefront ballots).
#include <string.h>

#include <new>

#include "spt_internal.h"

namespace spt {

// ------------------------------------------------------------------------------------------
// packing: P x d int32 subscripts + values -> records {l_0 .. l_{d-1}, pad, value}
// ------------------------------------------------------------------------------------------

// Packing of whole sort tiles (kSortTile entries per workgroup, the element order of the radix
// kernels) that also counts the first radix digit (bits 0-7) of every mode's subscript, so the
// first sort pass of each mode needs no histogram pass of its own: counts[m][digit][tile] for
// the tiles tile0 .. tile0 + gridDim.x - 1.  Out-of-range subscripts are packed (and counted) as
// 0 and reported, as by k_pack.
template <class VT, int RW>
__global__ __launch_bounds__(kBlock) void k_pack_tiles(const int32_t *__restrict__ subs,
                                                        const VT *__restrict__ vals, int d,
                                                        int64_t P, int64_t first, int64_t tile0,
                                                        int64_t ntiles, int4 *__restrict__ rec,
                                                        uint32_t *__restrict__ counts,
                                                        SptStatusBlock *st, int64_t dim0,
                                                        int64_t dim1, int64_t dim2, int64_t dim3,
                                                        int64_t dim4) {
    __shared__ uint32_t h[SPT_MAX_ORDER][256];
    const int tid = threadIdx.x, lane = tid & 63;
    const int64_t dims[SPT_MAX_ORDER] = {dim0, dim1, dim2, dim3, dim4};
#pragma unroll
    for (int m = 0; m < SPT_MAX_ORDER; ++m) h[m][tid] = 0;
    __syncthreads();
    const int64_t tile = tile0 + blockIdx.x;
    int64_t bad_min = INT64_MAX;
    for (int sub = 0; sub < kSortSubs; ++sub) {
        const int64_t base = tile * kSortTile + (int64_t)sub * kSortSub;
        // every item's loads first (kSortItems entries per thread in flight), then the packing
        // and the digit counts
        int32_t l[kSortItems][SPT_MAX_ORDER];
        VT v[kSortItems];
#pragma unroll
        for (int it = 0; it < kSortItems; ++it) {
            const int64_t e = base + it * kBlock + tid;
            const int64_t i = e - first;  // position in the caller's chunk
#pragma unroll
            for (int m = 0; m < SPT_MAX_ORDER; ++m) l[it][m] = 0;
            v[it] = 0;
            if (e < P) {
#pragma unroll
                for (int m = 0; m < SPT_MAX_ORDER; ++m)
                    if (m < d) l[it][m] = subs[i * d + m];
                v[it] = vals[i];
            }
        }
#pragma unroll
        for (int it = 0; it < kSortItems; ++it) {
            const int64_t e = base + it * kBlock + tid;
            const bool valid = e < P;
            int32_t w[RW];
#pragma unroll
            for (int k = 0; k < RW; ++k) w[k] = 0;
            if (valid) {
#pragma unroll
                for (int m = 0; m < SPT_MAX_ORDER; ++m) {
                    if (m < d) {
                        int32_t lm = l[it][m];
                        if (lm < 0 || (int64_t)lm >= dims[m]) {
                            bad_min = e < bad_min ? e : bad_min;
                            lm = 0;  // keep every later access in bounds
                        }
                        w[m] = lm;
                    }
                }
                if constexpr (sizeof(VT) == 8) {
                    const uint64_t b = __double_as_longlong(v[it]);
                    w[RW - 2] = (int32_t)(uint32_t)b;
                    w[RW - 1] = (int32_t)(uint32_t)(b >> 32);
                } else {
                    w[RW - 1] = __float_as_int(v[it]);
                }
                int4 *out = rec + e * (RW / 4);
                out[0] = make_int4(w[0], w[1], w[2], w[3]);
                if constexpr (RW == 8) out[1] = make_int4(w[4], w[5], w[6], w[7]);
            }
#pragma unroll
            for (int m = 0; m < SPT_MAX_ORDER; ++m) {
                if (m >= d) continue;  // uniform
                // lanes holding the same digit are matched with eight ballots; the lowest of them
                // adds the group's count
                const uint32_t dg = valid ? ((uint32_t)w[m] & 255u) : 256u;
                uint64_t mk = __ballot(dg < 256u);
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                    const bool bit = (dg >> b) & 1u;
                    const uint64_t bb = __ballot(bit);
                    mk &= bit ? bb : ~bb;
                }
                if (dg < 256u && (__ffsll((unsigned long long)mk) - 1) == lane)
                    atomicAdd(&h[m][dg], (uint32_t)__popcll(mk));
            }
        }
    }
    if (bad_min != INT64_MAX) {
        raise_status(st, SPT_ERANGE);
        atomicMin((unsigned long long *)&st->bad_entry, (unsigned long long)bad_min);
    }
    __syncthreads();
    for (int m = 0; m < d; ++m)
        counts[(int64_t)m * 256 * ntiles + (int64_t)tid * ntiles + tile] = h[m][tid];
}

__global__ void k_status_init(SptStatusBlock *st) {
    st->code = 0;
    st->pad = 0;
    st->bad_entry = INT64_MAX;
}

// ------------------------------------------------------------------------------------------
// radix sort: keys are mode-n subscripts (non-negative int32), values are entry positions
// ------------------------------------------------------------------------------------------

// Reads the pass input key of element e: from the records on the first pass, else from keys.
template <bool FIRST>
__device__ __forceinline__ int32_t sort_key(const int32_t *keys, const int32_t *recw, int rw,
                                            int n, int64_t e) {
    if constexpr (FIRST) return recw[e * rw + n];
    else return keys[e];
}

template <bool FIRST>
__global__ __launch_bounds__(kBlock) void k_radix_hist(const int32_t *__restrict__ keys,
                                                        const int32_t *__restrict__ recw, int rw,
                                                        int n, int64_t P, int shift,
                                                        uint32_t *__restrict__ counts,
                                                        int64_t ntiles) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    // the next sub-tile's digits are loaded while the current one is counted
    uint32_t pdg[kSortItems];
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
        const int64_t e = (int64_t)blockIdx.x * kSortTile + it * kBlock + threadIdx.x;
        pdg[it] = (e < P) ? (((uint32_t)sort_key<FIRST>(keys, recw, rw, n, e) >> shift) & 255u) : 256u;
    }
    for (int sub = 0; sub < kSortSubs; ++sub) {
        const int64_t base = (int64_t)blockIdx.x * kSortTile + (int64_t)sub * kSortSub;
        uint32_t dgs[kSortItems];
#pragma unroll
        for (int it = 0; it < kSortItems; ++it) dgs[it] = pdg[it];
        if (sub + 1 < kSortSubs) {
#pragma unroll
            for (int it = 0; it < kSortItems; ++it) {
                const int64_t e = base + kSortSub + it * kBlock + threadIdx.x;
                pdg[it] = (e < P) ? (((uint32_t)sort_key<FIRST>(keys, recw, rw, n, e) >> shift) & 255u) : 256u;
            }
        }
#pragma unroll
        for (int it = 0; it < kSortItems; ++it) {
            // lanes holding the same digit are matched with eight ballots; only the lowest of them
            // adds the group's count, so a skewed digit costs one LDS atomic per wave, not 64
            const uint32_t dg = dgs[it];
            uint64_t m = __ballot(dg < 256u);
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const bool bit = (dg >> b) & 1u;
                const uint64_t bb = __ballot(bit);
                m &= bit ? bb : ~bb;
            }
            if (dg < 256u && (__ffsll((unsigned long long)m) - 1) == lane)
                atomicAdd(&h[dg], (uint32_t)__popcll(m));
        }
    }
    __syncthreads();
    counts[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// block-wide exclusive scan of one value per thread; returns the block total in *total
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *total) {
    __shared__ uint32_t wsum[kBlock / kWave];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kBlock / kWave; ++w) {
        if (w < wave) before += wsum[w];
        all += wsum[w];
    }
    __syncthreads();
    *total = all;
    return before + x - v;
}

__global__ __launch_bounds__(kBlock) void k_scan_reduce(const uint32_t *__restrict__ a, int64_t L,
                                                         uint32_t *__restrict__ part) {
    int64_t base = (int64_t)blockIdx.x * kScanSeg + threadIdx.x * 8;
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k)
        if (base + k < L) s += a[base + k];
    uint32_t tot;
    block_exclusive_scan(s, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kBlock) void k_scan_partials(uint32_t *part, int64_t nb) {
    uint32_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += kBlock) {
        int64_t b = b0 + threadIdx.x;
        uint32_t v = b < nb ? part[b] : 0;
        uint32_t tot;
        uint32_t ex = block_exclusive_scan(v, &tot);
        if (b < nb) part[b] = carry + ex;
        carry += tot;
    }
}

__global__ __launch_bounds__(kBlock) void k_scan_down(uint32_t *__restrict__ a, int64_t L,
                                                       const uint32_t *__restrict__ part) {
    int64_t base = (int64_t)blockIdx.x * kScanSeg + threadIdx.x * 8;
    uint32_t v[8];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        v[k] = (base + k < L) ? a[base + k] : 0;
        s += v[k];
    }
    uint32_t tot;
    uint32_t run = block_exclusive_scan(s, &tot) + part[blockIdx.x];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        if (base + k < L) a[base + k] = run;
        run += v[k];
    }
}

// Stable scatter of one workgroup's tile: its sub-tiles in order, and inside a sub-tile the
// element order (item, wave, lane).  gofs[d] is the next output position of digit d.  Each
// sub-tile is first ordered by digit in LDS, then written out with consecutive threads on
// consecutive positions of a digit's run, so the stores coalesce.
// Tile of scatter workgroup b of n.  Workgroups go to the eight XCDs in turn, so consecutive
// ones run on different XCDs; this mapping gives each XCD a contiguous range of tiles, whose
// digit runs land next to each other in the output and so share lines in that XCD's L2
// (three-mode permutation of 1e8 keys: 7.19 ms against 7.35).
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t n) {
    const int64_t x = b & 7, l = b >> 3, per = n >> 3, rem = n & 7;
    return x * per + (x < rem ? x : rem) + l;
}

template <bool FIRST>
__global__ __launch_bounds__(kBlock) void k_radix_scatter(
    const int32_t *__restrict__ keys, const int32_t *__restrict__ vals,
    const int32_t *__restrict__ recw, int rw, int n, int64_t P, int shift,
    const uint32_t *__restrict__ offsets, int64_t ntiles, int32_t *__restrict__ okeys,
    int32_t *__restrict__ ovals) {
    __shared__ uint16_t cnt[kSortItems][kBlock / kWave][256];
    __shared__ uint32_t gofs[256];
    __shared__ uint32_t tstart[256];
    __shared__ int32_t lkey[kSortSub];
    __shared__ int32_t lval[kSortSub];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);  // the grid is one workgroup per tile
    gofs[tid] = offsets[(int64_t)tid * ntiles + tile];
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    // the next sub-tile's keys and values are loaded while the current one is ranked (three-mode
    // permutation of 1e8 keys: 6.3 ms against 7.2 with each sub-tile's loads waited for in turn)
    int32_t pk[kSortItems], pv[kSortItems];
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
        const int64_t e = tile * kSortTile + it * kBlock + tid;
        pk[it] = (e < P) ? sort_key<FIRST>(keys, recw, rw, n, e) : 0;
        pv[it] = (e < P) ? (FIRST ? (int32_t)e : vals[e]) : 0;
    }
    for (int sub = 0; sub < kSortSubs; ++sub) {
        const int64_t base = tile * kSortTile + (int64_t)sub * kSortSub;
        if (base >= P) break;  // uniform
        int32_t ck[kSortItems], cv[kSortItems];
#pragma unroll
        for (int it = 0; it < kSortItems; ++it) {
            ck[it] = pk[it];
            cv[it] = pv[it];
        }
        if (sub + 1 < kSortSubs) {
#pragma unroll
            for (int it = 0; it < kSortItems; ++it) {
                const int64_t e = base + kSortSub + it * kBlock + tid;
                pk[it] = (e < P) ? sort_key<FIRST>(keys, recw, rw, n, e) : 0;
                pv[it] = (e < P) ? (FIRST ? (int32_t)e : vals[e]) : 0;
            }
        }
        {
            uint32_t *c32 = reinterpret_cast<uint32_t *>(&cnt[0][0][0]);
            for (int k = tid; k < kSortItems * (kBlock / kWave) * 128; k += kBlock) c32[k] = 0;
        }
        __syncthreads();
        int32_t k_[kSortItems], v_[kSortItems];
        uint32_t dg_[kSortItems];
        uint16_t rk_[kSortItems];
#pragma unroll
        for (int it = 0; it < kSortItems; ++it) {
            int64_t e = base + it * kBlock + tid;
            bool valid = e < P;
            int32_t key = valid ? ck[it] : 0;
            int32_t val = valid ? cv[it] : 0;
            uint32_t dg = ((uint32_t)key >> shift) & 255u;
            uint64_t m = __ballot(valid);
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                bool bit = (dg >> b) & 1u;
                uint64_t bb = __ballot(bit);
                m &= bit ? bb : ~bb;
            }
            rk_[it] = (uint16_t)__popcll(m & lt);
            if (valid && (__ffsll((unsigned long long)m) - 1) == lane)
                cnt[it][wave][dg] = (uint16_t)__popcll(m);
            k_[it] = key;
            v_[it] = val;
            dg_[it] = valid ? dg : 256u;
        }
        __syncthreads();
        uint32_t run = 0;  // per digit: exclusive prefix over (item, wave) in element order
        for (int it = 0; it < kSortItems; ++it)
            for (int w = 0; w < kBlock / kWave; ++w) {
                uint32_t c = cnt[it][w][tid];
                cnt[it][w][tid] = (uint16_t)run;
                run += c;
            }
        uint32_t all;
        tstart[tid] = block_exclusive_scan(run, &all);  // sub-tile start of digit tid
        __syncthreads();
#pragma unroll
        for (int it = 0; it < kSortItems; ++it) {
            uint32_t dg = dg_[it];
            if (dg < 256u) {
                const uint32_t lp = tstart[dg] + cnt[it][wave][dg] + rk_[it];
                lkey[lp] = k_[it];
                lval[lp] = v_[it];
            }
        }
        __syncthreads();
        for (uint32_t i = tid; i < all; i += kBlock) {
            const int32_t key = lkey[i];
            const uint32_t dg = ((uint32_t)key >> shift) & 255u;
            const uint32_t dst = gofs[dg] + (i - tstart[dg]);
            okeys[dst] = key;
            ovals[dst] = lval[i];
        }
        __syncthreads();
        gofs[tid] += run;  // this sub-tile's count of digit tid
    }
}

// Mode-sorted copy of the records: out[q] = rec[perm[q]] (coalesced writes, gathered reads).
template <int RQ>
__global__ __launch_bounds__(kBlock) void k_gather_records(const int4 *__restrict__ rec,
                                                           const int32_t *__restrict__ perm,
                                                           int64_t P, int4 *__restrict__ out) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < P; q += stride) {
        const int64_t p = perm[q];
        out[q * RQ] = rec[p * RQ];
        if constexpr (RQ == 2) out[q * RQ + 1] = rec[p * RQ + 1];
    }
}

__global__ void k_iota_perm(int32_t *perm, int32_t *skey, int64_t P) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < P) {
        perm[i] = (int32_t)i;
        skey[i] = 0;
    }
}

static int bit_width(int64_t x) {  // bits needed for values 0..x
    int b = 0;
    while (x > 0) {
        ++b;
        x >>= 1;
    }
    return b;
}

static int permute_mode(spt_tensor *X, int n, hipStream_t s) {
    const int64_t P = X->P;
    X->srec[n] = nullptr;
    X->sperm[n] = nullptr;
    if (P == 0) {
        X->permuted[n] = 1;
        return SPT_OK;
    }
    const int nbits = bit_width(X->dims[n] - 1);
    if (nbits == 0) {
        hipLaunchKernelGGL(k_iota_perm, dim3((unsigned)ceil_div(P, kBlock)), dim3(kBlock), 0, s,
                           X->perm[n], X->skey[n], P);
        SPT_LAUNCH_CHECK();
        X->permuted[n] = 1;
        return SPT_OK;
    }
    const int passes = (nbits + 7) / 8;
    const int64_t ntiles = ceil_div(P, kSortTile);
    const int64_t L = 256 * ntiles;
    const int64_t nseg = ceil_div(L, kScanSeg);
    const int32_t *recw = reinterpret_cast<const int32_t *>(X->rec);
    const int32_t *ik = nullptr, *iv = nullptr;
    for (int pass = 0; pass < passes; ++pass) {
        const bool to_final = ((passes - 1 - pass) % 2) == 0;
        int32_t *ok = to_final ? X->skey[n] : X->tmp_keys;
        int32_t *ov = to_final ? X->perm[n] : X->tmp_vals;
        const int shift = pass * 8;
        dim3 g((unsigned)ntiles), b(kBlock);
        if (pass == 0 && X->hist0 != nullptr)
            // counted while packing; the scan below works in place, so on a copy
            SPT_HIP(hipMemcpyAsync(X->hist, X->hist0 + (size_t)n * L, (size_t)L * 4,
                                   hipMemcpyDeviceToDevice, s));
        else if (pass == 0)
            hipLaunchKernelGGL(k_radix_hist<true>, g, b, 0, s, ik, recw, X->rec_words, n, P,
                               shift, X->hist, ntiles);
        else
            hipLaunchKernelGGL(k_radix_hist<false>, g, b, 0, s, ik, recw, X->rec_words, n, P,
                               shift, X->hist, ntiles);
        SPT_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nseg), b, 0, s, X->hist, L,
                           X->scan_part);
        hipLaunchKernelGGL(k_scan_partials, dim3(1), b, 0, s, X->scan_part, nseg);
        hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nseg), b, 0, s, X->hist, L, X->scan_part);
        SPT_LAUNCH_CHECK();
        if (pass == 0)
            hipLaunchKernelGGL(k_radix_scatter<true>, g, b, 0, s, ik, iv, recw, X->rec_words, n,
                               P, shift, X->hist, ntiles, ok, ov);
        else
            hipLaunchKernelGGL(k_radix_scatter<false>, g, b, 0, s, ik, iv, recw, X->rec_words,
                               n, P, shift, X->hist, ntiles, ok, ov);
        SPT_LAUNCH_CHECK();
        ik = ok;
        iv = ov;
    }
    X->permuted[n] = 1;
    return SPT_OK;
}

// workspace layout -----------------------------------------------------------------------------

struct WsLayout {
    size_t status, rec, perm, skey, tmp_keys, tmp_vals, hist, hist0, scan_part, red, total;
};

static bool layout(int d, const int64_t *dims, int64_t P, int vdtype, WsLayout *L) {
    if (d < 2 || d > SPT_MAX_ORDER || dims == nullptr || P < 0 || P > INT32_MAX) return false;
    if (vdtype != SPT_F64 && vdtype != SPT_F32) return false;
    for (int m = 0; m < d; ++m)
        if (dims[m] < 1 || dims[m] > INT32_MAX) return false;
    const int rw = rec_words_for(d, vdtype);
    const int64_t ntiles = ceil_div(P, kSortTile);
    const int64_t Lh = 256 * (ntiles > 0 ? ntiles : 1);
    size_t o = 0;
    L->status = o;
    o += align256(sizeof(SptStatusBlock));
    L->rec = o;
    o += align256((size_t)P * rw * 4);
    L->perm = o;
    o += (size_t)d * align256((size_t)P * 4);
    L->skey = o;
    o += (size_t)d * align256((size_t)P * 4);
    L->tmp_keys = o;
    o += align256((size_t)P * 4);
    L->tmp_vals = o;
    o += align256((size_t)P * 4);
    L->hist = o;
    o += align256((size_t)Lh * 4);
    L->hist0 = o;
    o += (size_t)d * align256((size_t)Lh * 4);
    L->scan_part = o;
    o += align256((size_t)(ceil_div(Lh, kScanSeg) + 1) * 4);
    L->red = o;
    o += align256((size_t)kRedSlots * 8);
    L->total = o;
    return true;
}

}  // namespace spt

using namespace spt;

extern "C" {

const char *spt_status_string(int status) {
    switch (status) {
        case SPT_OK: return "ok";
        case SPT_EINVAL: return "invalid argument";
        case SPT_ERANGE: return "subscript out of range";
        case SPT_EHIP: return "HIP runtime error";
        case SPT_ESINGULAR: return "Gram matrix product not positive definite";
        case SPT_EWORKSPACE: return "workspace too small or misaligned";
        case SPT_EUNSUPPORTED: return "unsupported order, rank or dtype combination";
        case SPT_ESTATE: return "call out of order";
        default: return "unknown status";
    }
}

int spt_version(void) { return 100; }

size_t spt_tensor_workspace_bytes(int d, const int64_t *dims, int64_t nnz, int vals_dtype) {
    WsLayout L;
    if (!layout(d, dims, nnz, vals_dtype, &L)) return 0;
    return L.total;
}

int spt_tensor_create_begin(spt_tensor **out, int d, const int64_t *dims, int64_t nnz,
                            int vals_dtype, void *ws, size_t ws_bytes, void *stream) {
    if (out == nullptr) return SPT_EINVAL;
    *out = nullptr;
    WsLayout L;
    if (d > SPT_MAX_ORDER && d >= 2) return SPT_EUNSUPPORTED;
    if (!layout(d, dims, nnz, vals_dtype, &L)) return SPT_EINVAL;
    if (ws == nullptr || ((uintptr_t)ws & 255u) != 0 || ws_bytes < L.total)
        return SPT_EWORKSPACE;
    spt_tensor *X = new (std::nothrow) spt_tensor;
    if (!X) return SPT_EINVAL;
    memset(X, 0, sizeof *X);
    X->d = d;
    for (int m = 0; m < d; ++m) X->dims[m] = dims[m];
    for (int m = d; m < SPT_MAX_ORDER; ++m) X->dims[m] = 1;
    X->P = nnz;
    X->vdtype = vals_dtype;
    X->rec_words = rec_words_for(d, vals_dtype);
    uint8_t *w = static_cast<uint8_t *>(ws);
    X->ws = w;
    X->ws_bytes = ws_bytes;
    X->status = reinterpret_cast<SptStatusBlock *>(w + L.status);
    X->rec = reinterpret_cast<int4 *>(w + L.rec);
    for (int m = 0; m < d; ++m) {
        X->perm[m] = reinterpret_cast<int32_t *>(w + L.perm + m * align256((size_t)nnz * 4));
        X->skey[m] = reinterpret_cast<int32_t *>(w + L.skey + m * align256((size_t)nnz * 4));
    }
    X->tmp_keys = reinterpret_cast<int32_t *>(w + L.tmp_keys);
    X->tmp_vals = reinterpret_cast<int32_t *>(w + L.tmp_vals);
    X->hist = reinterpret_cast<uint32_t *>(w + L.hist);
    X->hist0 = nullptr;  // set once every tile has been packed
    X->scan_part = reinterpret_cast<uint32_t *>(w + L.scan_part);
    X->red = reinterpret_cast<double *>(w + L.red);
    X->appended = 0;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_status_init, dim3(1), dim3(1), 0, s, X->status);
    if (hipGetLastError() != hipSuccess) {
        delete X;
        return SPT_EHIP;
    }
    *out = X;
    return SPT_OK;
}

int spt_tensor_append(spt_tensor *X, int64_t first, int64_t count, const int32_t *subs,
                      const void *vals, void *stream) {
    if (X == nullptr || first < 0 || count < 1 || first + count > X->P) return SPT_EINVAL;
    if (subs == nullptr || vals == nullptr) return SPT_EINVAL;
    if (first % kSortTile != 0 || (count % kSortTile != 0 && first + count != X->P))
        return SPT_EINVAL;
    if (first != X->appended) return SPT_ESTATE;  // chunks arrive in order, once each
    const int64_t ntiles = ceil_div(X->P, kSortTile);
    const int64_t tile0 = first / kSortTile;
    const int64_t nt = ceil_div(count, kSortTile);
    uint32_t *counts = reinterpret_cast<uint32_t *>(
        reinterpret_cast<uint8_t *>(X->hist) + align256((size_t)256 * ntiles * 4));
    hipStream_t s = static_cast<hipStream_t>(stream);
    dim3 g((unsigned)nt), b(kBlock);
    const int64_t *dd = X->dims;
    const int d = X->d;
    if (X->vdtype == SPT_F64) {
        if (X->rec_words == 4)
            hipLaunchKernelGGL((k_pack_tiles<double, 4>), g, b, 0, s, subs,
                               static_cast<const double *>(vals), d, X->P, first, tile0, ntiles,
                               X->rec, counts, X->status, dd[0], dd[1], dd[2], dd[3], dd[4]);
        else
            hipLaunchKernelGGL((k_pack_tiles<double, 8>), g, b, 0, s, subs,
                               static_cast<const double *>(vals), d, X->P, first, tile0, ntiles,
                               X->rec, counts, X->status, dd[0], dd[1], dd[2], dd[3], dd[4]);
    } else {
        if (X->rec_words == 4)
            hipLaunchKernelGGL((k_pack_tiles<float, 4>), g, b, 0, s, subs,
                               static_cast<const float *>(vals), d, X->P, first, tile0, ntiles,
                               X->rec, counts, X->status, dd[0], dd[1], dd[2], dd[3], dd[4]);
        else
            hipLaunchKernelGGL((k_pack_tiles<float, 8>), g, b, 0, s, subs,
                               static_cast<const float *>(vals), d, X->P, first, tile0, ntiles,
                               X->rec, counts, X->status, dd[0], dd[1], dd[2], dd[3], dd[4]);
    }
    SPT_LAUNCH_CHECK();
    X->appended = first + count;
    if (X->appended == X->P) X->hist0 = counts;
    return SPT_OK;
}

int spt_tensor_create(spt_tensor **out, int d, const int64_t *dims, int64_t nnz,
                      const int32_t *subs, const void *vals, int vals_dtype, void *ws,
                      size_t ws_bytes, void *stream) {
    if (out == nullptr) return SPT_EINVAL;
    *out = nullptr;
    if (nnz > 0 && (subs == nullptr || vals == nullptr)) return SPT_EINVAL;
    spt_tensor *X = nullptr;
    int rc = spt_tensor_create_begin(&X, d, dims, nnz, vals_dtype, ws, ws_bytes, stream);
    if (rc) return rc;
    if (nnz > 0) {
        rc = spt_tensor_append(X, 0, nnz, subs, vals, stream);
        if (rc) {
            delete X;
            return rc;
        }
    }
    *out = X;
    return SPT_OK;
}

int spt_tensor_status(const spt_tensor *X, void *stream) {
    if (X == nullptr) return SPT_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    SptStatusBlock h;
    if (hipMemcpyAsync(&h, X->status, sizeof h, hipMemcpyDeviceToHost, s) != hipSuccess)
        return SPT_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return SPT_EHIP;
    if (h.code != 0 && h.code != SPT_ERANGE) {
        // clear a transient status (a range error is a property of the data and stays)
        int32_t zero = 0;
        if (hipMemcpyAsync(&X->status->code, &zero, sizeof zero, hipMemcpyHostToDevice, s) !=
                hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return SPT_EHIP;
    }
    return h.code;
}

int spt_tensor_validate(const spt_tensor *X, int64_t *bad_entry, void *stream) {
    if (X == nullptr) return SPT_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    SptStatusBlock h;
    if (hipMemcpyAsync(&h, X->status, sizeof h, hipMemcpyDeviceToHost, s) != hipSuccess)
        return SPT_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return SPT_EHIP;
    if (bad_entry) *bad_entry = (h.bad_entry == INT64_MAX) ? -1 : h.bad_entry;
    return h.code;
}

int spt_tensor_permute(spt_tensor *X, int mode, void *stream) {
    if (X == nullptr || mode < -1 || mode >= X->d) return SPT_EINVAL;
    if (X->appended != X->P) return SPT_ESTATE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int n = 0; n < X->d; ++n) {
        if (mode != -1 && n != mode) continue;
        int rc = permute_mode(X, n, s);
        if (rc) return rc;
    }
    return SPT_OK;
}

// keys[i] = mode-n subscript of entry idx[i]
__global__ __launch_bounds__(kBlock) void k_gather_keys(const int32_t *__restrict__ recw, int rw,
                                                        int n, const int32_t *__restrict__ idx,
                                                        int64_t P, int32_t *__restrict__ keys) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < P; i += stride)
        keys[i] = recw[(int64_t)idx[i] * rw + n];
}

// The other mode with the most rows (lowest index among equals): the one whose factor rows a
// mode-n traversal is least likely to find in cache.
static int second_mode(const spt_tensor *X, int n) {
    int m2 = -1;
    for (int m = 0; m < X->d; ++m)
        if (m != n && (m2 < 0 || X->dims[m] > X->dims[m2])) m2 = m;
    return m2;
}

static size_t copy_bytes_one(const spt_tensor *X, int order) {
    const size_t recs = align256((size_t)X->P * X->rec_words * 4);
    return order == SPT_COPY_BY_SECOND_MODE ? recs + align256((size_t)X->P * 4) : recs;
}

size_t spt_tensor_sorted_copy_bytes(const spt_tensor *X, int mode, int order) {
    if (X == nullptr || mode < -1 || mode >= X->d) return 0;
    if (order != SPT_COPY_STORAGE_ORDER && order != SPT_COPY_BY_SECOND_MODE) return 0;
    const size_t one = copy_bytes_one(X, order);
    return mode == -1 ? one * X->d : one;
}

// Order of the entries by (mode-n subscript, mode-m subscript, storage position): perm_m, which
// is stable in mode m, stably re-sorted by the mode-n subscript with the LSD passes of
// permute_mode.  scratch holds three arrays of P int32 (gathered keys and one ping-pong pair);
// the other pair is tmp_keys / q, so the last pass leaves the order in q.
static int order_by_two_modes(spt_tensor *X, int n, int m, int32_t *scratch, int32_t *q,
                              hipStream_t s) {
    const int64_t P = X->P;
    const int64_t words = (P + 3) & ~(int64_t)3;
    int32_t *k0 = scratch, *k1 = scratch + words, *v1 = scratch + 2 * words;
    const int nbits = bit_width(X->dims[n] - 1);
    if (nbits == 0) {
        if (hipMemcpyAsync(q, X->perm[m], (size_t)P * 4, hipMemcpyDeviceToDevice, s) !=
            hipSuccess)
            return SPT_EHIP;
        return SPT_OK;
    }
    const int32_t *recw = reinterpret_cast<const int32_t *>(X->rec);
    int64_t gblocks = ceil_div(P, kBlock);
    if (gblocks > 65536) gblocks = 65536;
    hipLaunchKernelGGL(k_gather_keys, dim3((unsigned)gblocks), dim3(kBlock), 0, s, recw,
                       X->rec_words, n, X->perm[m], P, k0);
    SPT_LAUNCH_CHECK();
    const int passes = (nbits + 7) / 8;
    const int64_t ntiles = ceil_div(P, kSortTile);
    const int64_t L = 256 * ntiles;
    const int64_t nseg = ceil_div(L, kScanSeg);
    const int32_t *ik = k0, *iv = X->perm[m];
    for (int pass = 0; pass < passes; ++pass) {
        const bool to_final = ((passes - 1 - pass) % 2) == 0;
        int32_t *ok = to_final ? X->tmp_keys : k1;
        int32_t *ov = to_final ? q : v1;
        const int shift = pass * 8;
        dim3 g((unsigned)ntiles), b(kBlock);
        hipLaunchKernelGGL(k_radix_hist<false>, g, b, 0, s, ik, recw, X->rec_words, n, P, shift,
                           X->hist, ntiles);
        SPT_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nseg), b, 0, s, X->hist, L,
                           X->scan_part);
        hipLaunchKernelGGL(k_scan_partials, dim3(1), b, 0, s, X->scan_part, nseg);
        hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nseg), b, 0, s, X->hist, L, X->scan_part);
        SPT_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_radix_scatter<false>, g, b, 0, s, ik, iv, recw, X->rec_words, n, P,
                           shift, X->hist, ntiles, ok, ov);
        SPT_LAUNCH_CHECK();
        ik = ok;
        iv = ov;
    }
    return SPT_OK;
}

int spt_tensor_sort_copy(spt_tensor *X, int mode, int order, void *ws, size_t ws_bytes,
                         void *stream) {
    if (X == nullptr || mode < -1 || mode >= X->d) return SPT_EINVAL;
    if (order != SPT_COPY_STORAGE_ORDER && order != SPT_COPY_BY_SECOND_MODE) return SPT_EINVAL;
    const size_t need = spt_tensor_sorted_copy_bytes(X, mode, order);
    if (need > 0 && (ws == nullptr || ((uintptr_t)ws & 255u) || ws_bytes < need))
        return SPT_EWORKSPACE;
    for (int n = 0; n < X->d; ++n) {
        if (mode != -1 && n != mode) continue;
        if (!X->permuted[n]) return SPT_ESTATE;
        if (order == SPT_COPY_BY_SECOND_MODE && !X->permuted[second_mode(X, n)])
            return SPT_ESTATE;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    uint8_t *w = static_cast<uint8_t *>(ws);
    const size_t recs = align256((size_t)X->P * X->rec_words * 4);
    for (int n = 0; n < X->d; ++n) {
        if (mode != -1 && n != mode) continue;
        int4 *dst = reinterpret_cast<int4 *>(w);
        const int32_t *q = X->perm[n];
        if (order == SPT_COPY_BY_SECOND_MODE) {
            int32_t *qd = reinterpret_cast<int32_t *>(w + recs);
            if (X->P > 0) {
                // the record area is free until the records are gathered into it
                int rc = order_by_two_modes(X, n, second_mode(X, n), reinterpret_cast<int32_t *>(w),
                                            qd, s);
                if (rc) return rc;
            }
            q = qd;
        }
        w += copy_bytes_one(X, order);
        if (X->P > 0) {
            int64_t blocks = ceil_div(X->P, kBlock);
            if (blocks > 65536) blocks = 65536;
            if (X->rec_words == 4)
                hipLaunchKernelGGL(k_gather_records<1>, dim3((unsigned)blocks), dim3(kBlock), 0, s,
                                   X->rec, q, X->P, dst);
            else
                hipLaunchKernelGGL(k_gather_records<2>, dim3((unsigned)blocks), dim3(kBlock), 0, s,
                                   X->rec, q, X->P, dst);
            SPT_LAUNCH_CHECK();
        }
        // an empty tensor's copy holds nothing (and its workspace may be null): the records'
        // address, never read, marks the copy as present
        X->srec[n] = (X->P > 0) ? dst : X->rec;
        X->sperm[n] = (X->P > 0) ? q : X->perm[n];
    }
    return SPT_OK;
}

int spt_tensor_drop_sorted_copy(spt_tensor *X, int mode) {
    if (X == nullptr || mode < -1 || mode >= X->d) return SPT_EINVAL;
    for (int n = 0; n < X->d; ++n)
        if (mode == -1 || n == mode) {
            X->srec[n] = nullptr;
            X->sperm[n] = nullptr;
        }
    return SPT_OK;
}

int spt_tensor_perm(const spt_tensor *X, int mode, const int32_t **perm, const int32_t **skey) {
    if (X == nullptr || mode < 0 || mode >= X->d) return SPT_EINVAL;
    if (!X->permuted[mode]) return SPT_ESTATE;
    if (perm) *perm = X->perm[mode];
    if (skey) *skey = X->skey[mode];
    return SPT_OK;
}

int spt_tensor_info(const spt_tensor *X, int *d, int64_t *dims, int64_t *nnz, int *vals_dtype) {
    if (X == nullptr) return SPT_EINVAL;
    if (d) *d = X->d;
    if (dims)
        for (int m = 0; m < X->d; ++m) dims[m] = X->dims[m];
    if (nnz) *nnz = X->P;
    if (vals_dtype) *vals_dtype = X->vdtype;
    return SPT_OK;
}

int spt_tensor_destroy(spt_tensor *X) {
    delete X;
    return SPT_OK;
}

}  // extern "C"
