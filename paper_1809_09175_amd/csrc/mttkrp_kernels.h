// MTTKRP kernels (eq. (mttkrp), Sec. 3) for gfx950, included by the per-dtype translation units.
//
// Work mapping shared by both kernels (the paper's league/team/vector hierarchy, Sec. 4.1,
// re-cast for 64-wide wavefronts):
//   - a wavefront owns a contiguous chunk of entries (storage order or mode-n sorted order);
//   - the wave is split into NG = 64/G lane groups; a group handles one entry at a time and its
//     G lanes hold CPL consecutive rank columns each (the register-resident row slice that the
//     paper's compile-time polymorphic arrays provide, Sec. 5);
//   - 64 entry records are fetched per batch with one 16/32-byte load per lane and staged in
//     LDS, from where each group reads its entry with one broadcast LDS load;
//   - U entries are gathered ahead (all factor-row loads issued before any is consumed) so
//     several row gathers are in flight per lane.
//
// k_mttkrp_perm walks the mode-n sorted order (Sec. 6).  Each group owns a contiguous slice of
// the wave's chunk and keeps a running row sum while the mode-n subscript is unchanged; a row
// that starts and ends inside the slice is written with a plain store.  The first and last
// rows of each slice meet in LDS, where the wave combines them (a segmented reduction across
// its groups); only the chunk's first and last rows, which neighbouring waves may share, are
// added atomically.  No LDS table and no barrier beyond the wavefront.
//
// k_mttkrp_atomic walks storage order in tiles; each tile's entries are sorted by output row in
// LDS and summed per row like the permuted kernel's chunks, so every distinct row of a tile
// receives one global atomic per column (see the kernel's own description below).
#pragma once

#include "spt_internal.h"

namespace spt {

template <int D, class VT>
struct RecShape {
    static constexpr int RW = (D * 4 + (int)sizeof(VT) <= 16) ? 4 : 8;  // 32-bit words
    static constexpr int RQ = RW / 4;                                     // 16-byte quads
};

template <class VT, int RW>
__device__ __forceinline__ VT rec_value(const int *w) {
    if constexpr (sizeof(VT) == 8)
        return __hiloint2double(w[RW - 1], w[RW - 2]);
    else
        return __int_as_float(w[RW - 1]);
}

template <class VT, int RW>
__device__ __forceinline__ void rec_set_value(int *w, VT v) {
    if constexpr (sizeof(VT) == 8) {
        w[RW - 2] = __double2loint(v);
        w[RW - 1] = __double2hiint(v);
    } else {
        w[RW - 1] = __float_as_int(v);
    }
}

// Mode-n subscript of a record staged in LDS.  Read with its own LDS load at a run-time word
// offset: selecting it from the record's registers by the run-time mode makes the compiler
// spill the record to scratch memory to index it.
template <int RW>
__device__ __forceinline__ int lds_sub(const int4 *q, int n) {
    return reinterpret_cast<const int *>(q)[n];
}

// CPL consecutive factor entries, widened to the accumulation type
template <class FT, int CPL, class AT>
__device__ __forceinline__ void load_cols(const FT *__restrict__ p, AT *out) {
    if constexpr (sizeof(FT) == 2) {  // BF16 bit patterns
        if constexpr (CPL == 1) {
            out[0] = bf16_bits_to_f32(*reinterpret_cast<const uint16_t *>(p));
        } else if constexpr (CPL == 2) {
            uint32_t v = *reinterpret_cast<const uint32_t *>(p);
            out[0] = bf16_bits_to_f32(v & 0xffffu);
            out[1] = bf16_bits_to_f32(v >> 16);
        } else if constexpr (CPL == 4) {
            uint2 v = *reinterpret_cast<const uint2 *>(p);
            out[0] = bf16_bits_to_f32(v.x & 0xffffu);
            out[1] = bf16_bits_to_f32(v.x >> 16);
            out[2] = bf16_bits_to_f32(v.y & 0xffffu);
            out[3] = bf16_bits_to_f32(v.y >> 16);
        } else {
            uint4 v = *reinterpret_cast<const uint4 *>(p);
            const uint32_t q[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                out[2 * h] = bf16_bits_to_f32(q[h] & 0xffffu);
                out[2 * h + 1] = bf16_bits_to_f32(q[h] >> 16);
            }
        }
    } else if constexpr (sizeof(FT) == 4) {
        if constexpr (CPL == 1) {
            out[0] = *p;
        } else if constexpr (CPL == 2) {
            float2 v = *reinterpret_cast<const float2 *>(p);
            out[0] = v.x;
            out[1] = v.y;
        } else {
#pragma unroll
            for (int h = 0; h < CPL; h += 4) {
                float4 v = *reinterpret_cast<const float4 *>(p + h);
                out[h] = v.x;
                out[h + 1] = v.y;
                out[h + 2] = v.z;
                out[h + 3] = v.w;
            }
        }
    } else {
        if constexpr (CPL == 1) {
            out[0] = *p;
        } else {
#pragma unroll
            for (int h = 0; h < CPL; h += 2) {
                double2 v = *reinterpret_cast<const double2 *>(p + h);
                out[h] = v.x;
                out[h + 1] = v.y;
            }
        }
    }
}

template <class AT, int CPL>
__device__ __forceinline__ void store_cols(AT *__restrict__ p, const AT *v) {
    if constexpr (sizeof(AT) == 4 && CPL == 2) {
        *reinterpret_cast<float2 *>(p) = make_float2(v[0], v[1]);
    } else if constexpr (sizeof(AT) == 4 && CPL >= 4) {
#pragma unroll
        for (int h = 0; h < CPL; h += 4)
            *reinterpret_cast<float4 *>(p + h) = make_float4(v[h], v[h + 1], v[h + 2], v[h + 3]);
    } else {
#pragma unroll
        for (int c = 0; c < CPL; ++c) p[c] = v[c];
    }
}

// A record is read once per traversal: a non-temporal load keeps the records, streamed from a
// sorted copy or gathered through the permutation, from displacing factor rows in L2 and the
// Infinity Cache (measured on the 1e8-entry power-law tensor, all-mode MTTKRP: sorted copies
// 3.76-3.79 ms instead of 3.84 at R = 32 and 6.45-6.64 instead of 7.05 at R = 64; gathered
// records 8.05 instead of 8.33 and 11.3 instead of 12.0).  Non-temporal output stores measured
// no different and are not used.
__device__ __forceinline__ int4 load_stream(const int4 *p) {
    typedef int v4i __attribute__((ext_vector_type(4)));
    const v4i v = __builtin_nontemporal_load(reinterpret_cast<const v4i *>(p));
    return make_int4(v.x, v.y, v.z, v.w);
}

template <class AT, int CPL>
__device__ __forceinline__ void atomic_cols(AT *__restrict__ p, const AT *v) {
#pragma unroll
    for (int c = 0; c < CPL; ++c) atomic_add_f(p + c, v[c]);
}

// The factor matrices of the modes other than n, in increasing mode order (other mode j is
// mode j below n, mode j + 1 from n on), chosen once per wavefront: the per-entry gathers then
// carry no branch on the run-time mode, so the loads of several entries can be in flight at
// once instead of each waiting behind a branch.
template <int D>
struct OtherModes {
    const char *base[D - 1];
    int up[D - 1];  // all ones when other mode j is mode j + 1, else zero
};

template <int D, class FT>
__device__ __forceinline__ OtherModes<D> other_modes(const FactorSet<FT> &A, int n) {
    OtherModes<D> o;
#pragma unroll
    for (int j = 0; j < D - 1; ++j) {
        const bool up = j >= n;
        o.base[j] = reinterpret_cast<const char *>(up ? A.p[j + 1] : A.p[j]);
        o.up[j] = up ? -1 : 0;
    }
    return o;
}

// Product row of one entry: t[c] = x * lambda_j * prod_{m != n} A^(m)(l_m, j), for this lane's
// columns j = col0 .. col0+CPL-1 (multiply order as in Sec. 4.1: x times the weight first,
// then each other mode in increasing order).  Factor rows are addressed with 32-bit byte
// offsets from the (wave-uniform) matrix base, so each gather needs one offset register and
// the hardware's scalar-base addressing; every factor matrix must be smaller than 4 GiB.
// Lanes past column R pass colbytes = 0: they read the row's first columns and their products
// are never stored, which keeps the gathers free of lane-divergent branches.
template <int D, int RW, int CPL, class FT, class VT, class AT>
__device__ __forceinline__ void entry_product(const int *w, const OtherModes<D> &om,
                                              uint32_t rowbytes, uint32_t colbytes,
                                              const AT *lam, AT *t) {
    AT f[D - 1][CPL];
#pragma unroll
    for (int j = 0; j < D - 1; ++j) {
        const int sub = (w[j] & ~om.up[j]) | (w[j + 1] & om.up[j]);
        const uint32_t off = (uint32_t)sub * rowbytes + colbytes;
        load_cols<FT, CPL, AT>(reinterpret_cast<const FT *>(om.base[j] + off), f[j]);
    }
    const AT x = (AT)rec_value<VT, RW>(w);
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        AT v = x * lam[c];
#pragma unroll
        for (int j = 0; j < D - 1; ++j) v *= f[j][c];
        t[c] = v;
    }
}

// The same product without the entry value and the weights: t[c] = prod_{m != n} A^(m)(l_m, j),
// and x = the entry value, for a caller that accumulates x * t with one multiply-add per column
// and applies lambda once per output row.  With BF16 factors this form takes the gathers' widening
// plus two instructions per column and entry instead of four: 7-8% on the 1e8-entry power-law
// tensor at R = 32 and 64 (with FP32 factors it measured no faster).
template <int D, int RW, int CPL, class FT, class VT, class AT>
__device__ __forceinline__ void entry_product_nx(const int *w, const OtherModes<D> &om,
                                                 uint32_t rowbytes, uint32_t colbytes, AT *t,
                                                 AT &x) {
    AT f[D - 1][CPL];
#pragma unroll
    for (int j = 0; j < D - 1; ++j) {
        const int sub = (w[j] & ~om.up[j]) | (w[j + 1] & om.up[j]);
        const uint32_t off = (uint32_t)sub * rowbytes + colbytes;
        load_cols<FT, CPL, AT>(reinterpret_cast<const FT *>(om.base[j] + off), f[j]);
    }
    x = (AT)rec_value<VT, RW>(w);
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        AT v = f[0][c];
#pragma unroll
        for (int j = 1; j < D - 1; ++j) v *= f[j][c];
        t[c] = v;
    }
}

// Generalized CP elementwise losses f(x, m) (FP64) and their derivatives df/dm:
// 0 Poisson with log link, 1 Bernoulli with logit link, 2 Gaussian, 3 Gamma (the model is the
// positive mean; m + 1e-10 guards m = 0).
constexpr double kGammaEps = 1e-10;

__device__ __forceinline__ double gcp_loss_term(int loss, double x, double m) {
    if (loss == 0) return exp(m) - x * m;
    if (loss == 1) return (m > 0.0 ? m : 0.0) + log1p(exp(-fabs(m))) - x * m;  // log(1 + e^m)
    if (loss == 3) return x / (m + kGammaEps) + log(m + kGammaEps);
    return (x - m) * (x - m);
}

template <class T>
__device__ __forceinline__ T gcp_dloss(int loss, T x, T m) {
    if (loss == 0) return exp(m) - x;                       // Poisson, log link
    if (loss == 1) return (T)1 / ((T)1 + exp(-m)) - x;      // Bernoulli, logit link
    if (loss == 3) {                                        // Gamma
        const T r = (T)1 / (m + (T)kGammaEps);
        return r - x * r * r;
    }
    return (T)2 * (m - x);                                  // Gaussian
}

// One entry of the fused generalized-CP pass over mode n: the model value
// m = sum_j prod_m A^(m)(l_m, j) (product in mode order, this lane's columns summed, then a
// butterfly over the G lanes of the group), y = df(x, m), and the gradient row contribution
// t = y * prod_{m != n} A^(m)(l_m, j).  lterm receives f(x, m).  All lanes of the group must
// take part (the butterfly); lanes past column R add nothing to m.  The mode-n row is kept in
// an[] across calls and loaded only when the key differs from ankey (the caller starts ankey at
// -1): along the sorted order a lane group meets each mode-n row in one run, so the row is
// fetched once per run instead of once per entry.
template <int D, int RW, int G, int CPL, class FT, class AT>
__device__ __forceinline__ void entry_gcp(const int *w, int key, const OtherModes<D> &om,
                                          const char *anb, int n, uint32_t rowbytes,
                                          uint32_t colbytes, bool colok, int loss, AT *t,
                                          double &lterm, AT *an, int &ankey) {
    AT f[D - 1][CPL];
#pragma unroll
    for (int j = 0; j < D - 1; ++j) {
        const int sub = (w[j] & ~om.up[j]) | (w[j + 1] & om.up[j]);
        load_cols<FT, CPL, AT>(reinterpret_cast<const FT *>(om.base[j] + (uint32_t)sub * rowbytes + colbytes),
                               f[j]);
    }
    if (key != ankey) {
        load_cols<FT, CPL, AT>(reinterpret_cast<const FT *>(anb + (uint32_t)key * rowbytes + colbytes), an);
        ankey = key;
    }
    const AT x = rec_value<AT, RW>(w);
    AT q = 0;
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        AT p = 1;
#pragma unroll
        for (int j = 0; j < D - 1; ++j) {
            p *= (j == n) ? an[c] : (AT)1;
            p *= f[j][c];
        }
        p *= (n == D - 1) ? an[c] : (AT)1;
        q += colok ? p : (AT)0;
    }
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) q += __shfl_xor(q, o, G);
    const AT y = gcp_dloss<AT>(loss, x, q);
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        AT v = y;
#pragma unroll
        for (int j = 0; j < D - 1; ++j) v *= f[j][c];
        t[c] = v;
    }
    lterm = gcp_loss_term(loss, (double)x, (double)q);
}

template <int RQ>
__device__ __forceinline__ void lds_record(const int4 *q, int *w) {
    int4 a = q[0];
    w[0] = a.x; w[1] = a.y; w[2] = a.z; w[3] = a.w;
    if constexpr (RQ == 2) {
        int4 b = q[1];
        w[4] = b.x; w[5] = b.y; w[6] = b.z; w[7] = b.w;
    }
}

// entries gathered ahead per lane group: enough loads in flight to cover the gather latency
// while the registers still allow 6-8 waves per SIMD
// Entries a lane group gathers ahead (its loads in flight at once), per kernel, lane layout and
// factor element size.  Measured on MI355X (1e8-entry Zipf tensor, R = 16/32/64, U in
// {1, 2, 4, 8, 16}); with U = 1 the compiler still overlaps consecutive entries, which is why
// some wide layouts do best there.  Unmeasured layouts: 32 / CPL entries for 4-lane groups,
// 16 / CPL for wider ones.  Never more than G (the entries a group stages per batch).
enum { KERNEL_PERM = 0, KERNEL_ATOMIC = 1, KERNEL_MODEL = 2 };

__host__ __device__ constexpr int unroll_for(int kernel, int G, int CPL, int fbytes) {
    int u = (G <= 4 ? 32 : 16) / CPL;
    if (kernel == KERNEL_PERM && fbytes == 4) {
        if (G == 8 && CPL == 8) u = 1;
        if (G == 16 && CPL == 4) u = 1;
        if (G == 8 && CPL == 4) u = 8;
        if (G == 16 && CPL == 2) u = 8;
        if (G == 32 && CPL == 2) u = 8;
    } else if (kernel == KERNEL_PERM && fbytes == 2) {
        if (G >= 8 && (CPL == 8 || (CPL == 4 && G <= 16))) u = 1;
        if (G == 16 && CPL == 2) u = 8;
        if (G == 32 && CPL == 2) u = 8;
    } else if (kernel == KERNEL_ATOMIC && CPL == 1) {
        u = (G <= 32) ? 1 : 4;
    } else if (kernel == KERNEL_MODEL) {
        u = 1;  // fit 2.8 vs 3.6 ms at R = 32 (unroll 4); model values alike
    }
    if (u < 1) u = 1;
    return u < G ? u : G;
}

template <int KERNEL, int G, int CPL, class FT>
struct UnrollFor {
    static constexpr int value = unroll_for(KERNEL, G, CPL, (int)sizeof(FT));
};

// Staged records of one lane group in LDS: its G records plus one 16-byte pad.  The lanes of a
// group read the same record at a time while the groups read records G records apart; without
// the pad those addresses are a multiple of 128 bytes apart for G >= 8, so every group hits the
// same LDS banks (an 8-way conflict at 8 x 4, counted as 1.25e8 conflict cycles per launch on
// the 1e8-entry power-law tensor).  With it, group g starts 4g banks further on.  The kernels
// measured no faster for it: the conflicts overlapped the wait for the factor-row gathers.
__host__ __device__ constexpr int staged_group_stride(int G, int RQ) { return G * RQ + 1; }

// Bytes of one wavefront's PermShared (the batched kernel sizes its dynamic LDS with it).
constexpr size_t perm_shared_bytes(int G, int CPL, int RQ, int at_bytes) {
    const int NG = kWave / G;
    const size_t b = (size_t)NG * staged_group_stride(G, RQ) * 16 +
                     (size_t)2 * NG * G * CPL * at_bytes + (size_t)2 * NG * 4;
    return (b + 15) / 16 * 16;
}

// LDS of one wavefront in the permuted kernel: the staged records of the current batch and the
// boundary partial rows (first and last row of every lane group's slice).
template <int D, int G, int CPL, class VT, class AT>
struct PermShared {
    static constexpr int RQ = RecShape<D, VT>::RQ, NG = kWave / G;
    int4 rec[NG * staged_group_stride(G, RQ)];
    AT part[2 * NG][G * CPL];
    int pkey[2 * NG];
};

// One wavefront processes sorted positions [c0, min(c0 + chunk, P)) of mode n (c0 < P).
// With GCP, the entries' values are replaced by the generalized-CP loss derivative computed on
// the fly (entry_gcp; lambda and vovr unused), and when loss_part is given each wavefront also
// writes the sum of its entries' loss terms to loss_part[c0 / chunk].
template <int D, int G, int CPL, class FT, class VT, class AT, int UMAX = 64, bool GCP = false>
__device__ __forceinline__ void perm_wave_chunk(PermShared<D, G, CPL, VT, AT> &sm,
                                                const int4 *__restrict__ rec,
                                                const int32_t *__restrict__ perm,
                                                const int4 *__restrict__ srec, int64_t P,
                                                int n, int R, const FactorSet<FT> &A,
                                                const double *__restrict__ lambda,
                                                const VT *__restrict__ vovr, AT *__restrict__ V,
                                                int chunk, int64_t c0,
                                                int *__restrict__ slot_keys = nullptr,
                                                AT *__restrict__ slot_vals = nullptr,
                                                int loss_kind = 0,
                                                double *__restrict__ loss_part = nullptr) {
    constexpr int RW = RecShape<D, VT>::RW, RQ = RecShape<D, VT>::RQ;
    constexpr int NG = kWave / G;
    constexpr int U0 = UnrollFor<KERNEL_PERM, G, CPL, FT>::value;
    constexpr int U = U0 < UMAX ? U0 : UMAX;
    // BF16 factors: entry value and weights applied by multiply-add (entry_product_nx)
    constexpr bool XFMA = !GCP && sizeof(FT) == 2;
    const int lane = threadIdx.x & 63;
    const int g = lane / G, gl = lane % G;
    const int col0 = gl * CPL;
    const bool colok = col0 < R;
    const uint32_t rowbytes = (uint32_t)R * sizeof(FT);
    const uint32_t colbytes = colok ? (uint32_t)col0 * sizeof(FT) : 0u;
    const OtherModes<D> om = other_modes<D>(A, n);
    const char *anb = reinterpret_cast<const char *>(A.p[n]);
    double lacc = 0.0;
    AT an[CPL];
    int ankey = -1;
    (void)anb;
    (void)an;
    (void)ankey;
    const int64_t c1 = (c0 + chunk < P) ? c0 + chunk : P;
    const int S = chunk / NG;  // slice per group
    const int64_t gb = c0 + (int64_t)g * S;
    const int64_t ge = (gb + S < c1) ? gb + S : c1;
    const int glen = ge > gb ? (int)(ge - gb) : 0;
    const int wlen = (int)((c1 - c0) < S ? (c1 - c0) : S);
    const int nb = (wlen + G - 1) / G;
    const int32_t *gperm = perm + gb;

    AT lam[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c)
        lam[c] = (lambda != nullptr && colok) ? (AT)lambda[col0 + c] : (AT)1;
    if (gl == 0) {
        sm.pkey[2 * g] = -1;
        sm.pkey[2 * g + 1] = -1;
    }

    // software pipeline: the records of batch b+1 (and, when they are gathered through the
    // permutation, the permutation entries of batch b+2) are in flight while batch b is
    // processed.  With a mode-sorted copy of the records (srec) the records stream in order.
    const int4 *gsrec = (srec != nullptr) ? srec + gb * RQ : nullptr;
    int4 rc0 = make_int4(0, 0, 0, 0), rc1 = rc0;
    VT vo = 0;
    int pn = -1;
    if (gl < glen) {
        if (gsrec != nullptr) {
            rc0 = load_stream(gsrec + gl * RQ);
            if constexpr (RQ == 2) rc1 = load_stream(gsrec + gl * RQ + 1);
            if (vovr != nullptr) vo = vovr[gperm[gl]];
        } else {
            const int p = gperm[gl];
            rc0 = load_stream(rec + (int64_t)p * RQ);
            if constexpr (RQ == 2) rc1 = load_stream(rec + (int64_t)p * RQ + 1);
            if (vovr != nullptr) vo = vovr[p];
        }
    }
    if (gsrec == nullptr && G + gl < glen) pn = gperm[G + gl];

    int key = -1, first_key = -1;
    AT acc[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) acc[c] = 0;

    constexpr int GS = staged_group_stride(G, RQ);
    const int slot = g * GS + gl * RQ;  // this lane's staging slot
    for (int b = 0; b < nb; ++b) {
        if (b * G + gl < glen) {
            sm.rec[slot] = rc0;
            if constexpr (RQ == 2) sm.rec[slot + 1] = rc1;
            if (vovr != nullptr)
                rec_set_value<VT, RW>(reinterpret_cast<int *>(&sm.rec[slot]), vo);
        }
        wave_sync();
        if (gsrec != nullptr) {
            const int nx = (b + 1) * G + gl;
            if (nx < glen) {
                rc0 = load_stream(gsrec + nx * RQ);
                if constexpr (RQ == 2) rc1 = load_stream(gsrec + nx * RQ + 1);
                if (vovr != nullptr) vo = vovr[gperm[nx]];
            }
        } else {
            if (pn >= 0) {
                rc0 = load_stream(rec + (int64_t)pn * RQ);
                if constexpr (RQ == 2) rc1 = load_stream(rec + (int64_t)pn * RQ + 1);
                if (vovr != nullptr) vo = vovr[pn];
            }
            pn = ((b + 2) * G + gl < glen) ? gperm[(b + 2) * G + gl] : -1;
        }

        const int cnt = glen - b * G < G ? glen - b * G : G;
        const int4 *sr = &sm.rec[g * GS];
        for (int s0 = 0; s0 < cnt; s0 += U) {
            AT t[U][CPL];
            AT xv[U];
            (void)xv;
            int kk[U];
            if (s0 + U <= cnt) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    int w[RW];
                    lds_record<RQ>(sr + (s0 + u) * RQ, w);
                    kk[u] = lds_sub<RW>(sr + (s0 + u) * RQ, n);
                    if constexpr (GCP) {
                        double lt;
                        entry_gcp<D, RW, G, CPL, FT, AT>(w, kk[u], om, anb, n, rowbytes, colbytes,
                                                         colok, loss_kind, t[u], lt, an, ankey);
                        lacc += (gl == 0) ? lt : 0.0;
                    } else if constexpr (XFMA) {
                        entry_product_nx<D, RW, CPL, FT, VT, AT>(w, om, rowbytes, colbytes, t[u], xv[u]);
                    } else {
                        entry_product<D, RW, CPL, FT, VT, AT>(w, om, rowbytes, colbytes, lam, t[u]);
                    }
                }
            } else {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    kk[u] = -1;
                    if (s0 + u < cnt) {
                        int w[RW];
                        lds_record<RQ>(sr + (s0 + u) * RQ, w);
                        kk[u] = lds_sub<RW>(sr + (s0 + u) * RQ, n);
                        if constexpr (GCP) {
                            double lt;
                            entry_gcp<D, RW, G, CPL, FT, AT>(w, kk[u], om, anb, n, rowbytes,
                                                             colbytes, colok, loss_kind, t[u], lt, an, ankey);
                            lacc += (gl == 0) ? lt : 0.0;
                        } else if constexpr (XFMA) {
                            entry_product_nx<D, RW, CPL, FT, VT, AT>(w, om, rowbytes, colbytes, t[u], xv[u]);
                        } else {
                            entry_product<D, RW, CPL, FT, VT, AT>(w, om, rowbytes, colbytes, lam, t[u]);
                        }
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (kk[u] >= 0) {
                    if (kk[u] != key) {
                        if (key >= 0) {
                            if (XFMA && lambda != nullptr) {
#pragma unroll
                                for (int c = 0; c < CPL; ++c) acc[c] *= lam[c];
                            }
                            if (key == first_key) {
#pragma unroll
                                for (int c = 0; c < CPL; ++c) sm.part[2 * g][col0 + c] = acc[c];
                                if (gl == 0) sm.pkey[2 * g] = key;
                            } else if (colok) {
                                store_cols<AT, CPL>(V + (int64_t)key * R + col0, acc);
                            }
                        } else {
                            first_key = kk[u];
                        }
                        key = kk[u];
#pragma unroll
                        for (int c = 0; c < CPL; ++c) acc[c] = 0;
                    }
                    if constexpr (XFMA) {
#pragma unroll
                        for (int c = 0; c < CPL; ++c) acc[c] = fma(xv[u], t[u][c], acc[c]);
                    } else {
#pragma unroll
                        for (int c = 0; c < CPL; ++c) acc[c] += t[u][c];
                    }
                }
            }
        }
        wave_sync();
    }
    if (key >= 0) {
        if (XFMA && lambda != nullptr) {
#pragma unroll
            for (int c = 0; c < CPL; ++c) acc[c] *= lam[c];
        }
#pragma unroll
        for (int c = 0; c < CPL; ++c) sm.part[2 * g + 1][col0 + c] = acc[c];
        if (gl == 0) sm.pkey[2 * g + 1] = key;
    }
    wave_sync();
    if (g == 0) {
        // Rows shared with neighbouring chunks are the chunk's first and last rows.  They are
        // added atomically, or, in the deterministic mode, parked in two scratch slots per chunk
        // (slot 2c: first row, slot 2c+1: last row or key -1) for k_det_fixup to sum in chunk
        // order, so no atomic is issued at all.
        const int64_t cid = c0 / chunk;
        int ck = -1;
        bool first_seg = true;
        AT cacc[CPL];
#pragma unroll
        for (int c = 0; c < CPL; ++c) cacc[c] = 0;
        for (int e = 0; e < 2 * NG; ++e) {
            const int ke = sm.pkey[e];
            if (ke < 0) continue;
            if (ke != ck) {
                if (ck >= 0) {
                    if (first_seg) {
                        if (slot_keys != nullptr) {
                            if (gl == 0) slot_keys[2 * cid] = ck;
                            if (colok) store_cols<AT, CPL>(slot_vals + 2 * cid * R + col0, cacc);
                        } else if (colok) {
                            atomic_cols<AT, CPL>(V + (int64_t)ck * R + col0, cacc);
                        }
                    } else if (colok) {
                        store_cols<AT, CPL>(V + (int64_t)ck * R + col0, cacc);
                    }
                    first_seg = false;
                }
                ck = ke;
#pragma unroll
                for (int c = 0; c < CPL; ++c) cacc[c] = 0;
            }
#pragma unroll
            for (int c = 0; c < CPL; ++c) cacc[c] += sm.part[e][col0 + c];
        }
        if (ck >= 0) {
            if (slot_keys != nullptr) {
                const int64_t slot = first_seg ? 2 * cid : 2 * cid + 1;
                if (gl == 0) {
                    slot_keys[slot] = ck;
                    if (first_seg) slot_keys[2 * cid + 1] = -1;
                }
                if (colok) store_cols<AT, CPL>(slot_vals + slot * R + col0, cacc);
            } else if (colok) {
                atomic_cols<AT, CPL>(V + (int64_t)ck * R + col0, cacc);
            }
        }
    }
    if constexpr (GCP) {
        if (loss_part != nullptr) {
            // lane sums in a fixed butterfly, one partial per wave chunk
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) lacc += __shfl_xor(lacc, o, 64);
            if (lane == 0) loss_part[c0 / chunk] = lacc;
        }
    }
}

// Deterministic mode, second pass: one wavefront per slot; the first slot of every run of equal
// keys sums the run in slot (= sorted) order and stores the row.  Slots with key -1 are skipped.
template <class AT>
__global__ __launch_bounds__(kBlock) void k_det_fixup(const int *__restrict__ keys,
                                                      const AT *__restrict__ vals,
                                                      int64_t nslots, int R,
                                                      AT *__restrict__ V) {
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * (kBlock / kWave) + (threadIdx.x >> 6);
    if (i >= nslots) return;
    const int k = keys[i];
    if (k < 0) return;
    if (i > 0) {
        int prev = keys[i - 1];
        if (prev < 0 && i > 1) prev = keys[i - 2];
        if (prev == k) return;  // not the first slot of its run
    }
    for (int col = lane; col < R; col += kWave) {
        AT s = 0;
        for (int64_t j = i; j < nslots; ++j) {
            const int kj = keys[j];
            if (kj < 0) continue;
            if (kj != k) break;
            s += vals[j * R + col];
        }
        V[(int64_t)k * R + col] = s;
    }
}

template <int D, int G, int CPL, class FT, class VT, class AT>
__global__ __launch_bounds__(kBlock) void k_mttkrp_perm(
    const int4 *__restrict__ rec, const int32_t *__restrict__ perm,
    const int4 *__restrict__ srec, int64_t P, int n, int R,
    FactorSet<FT> A, const double *__restrict__ lambda, const VT *__restrict__ vovr,
    AT *__restrict__ V, int chunk, int *__restrict__ slot_keys, AT *__restrict__ slot_vals) {
    __shared__ PermShared<D, G, CPL, VT, AT> sm[kBlock / kWave];
    const int wave = threadIdx.x >> 6;
    const int64_t c0 = ((int64_t)blockIdx.x * (kBlock / kWave) + wave) * chunk;
    if (c0 >= P) return;  // whole wavefront leaves together
    perm_wave_chunk<D, G, CPL, FT, VT, AT>(sm[wave], rec, perm, srec, P, n, R, A, lambda, vovr, V,
                                           chunk, c0, slot_keys, slot_vals);
}

// ------------------------------------------------------------------------------------------
// Atomic MTTKRP over storage order (the paper's atomic kernels, Fig. mttkrp_alg and
// Fig. mttkrp_array), with the partial rows combined inside the workgroup before they reach V.
//
// A workgroup takes a tile of T consecutive entries in storage order (T = 1024, fewer where the
// staging would not fit 64 KiB of LDS):
//   1. the tile's records are read with coalesced loads and staged in LDS;
//   2. the tile's mode-n subscripts are sorted in LDS (a bitonic network over (subscript, tile
//      position) pairs: T / 256 pairs per thread, the compare-exchanges between a thread's own
//      pairs in registers, the others through LDS with a wavefront barrier, or a workgroup
//      barrier for the strides that span wavefronts), so the entries of each output row are
//      adjacent;
//   3. each wavefront walks a quarter of the sorted tile as the permuted kernel walks its chunk:
//      lane groups keep a running row sum while the subscript is unchanged, the first and last
//      rows of every group meet in LDS, then the first and last rows of every wavefront;
//   4. every distinct row of the tile is added to V with one global atomic per column.
// So no row receives more than one atomic per tile: a hot row's FP32 sum in V collects
// P / T pre-summed terms instead of one per entry (with per-entry atomics, rows of a
// million entries of the 1e8-entry power-law tensor drifted beyond the FP32 tolerance).
// ------------------------------------------------------------------------------------------

// Entries sorted together: the largest of 1024, 512, 256 whose staging (records, keys,
// positions) and partial rows fit 64 KiB of LDS.  Measured on the 1e8-entry power-law tensor
// (all modes, R = 16 / 32 / 64): 1024-entry tiles 12.9 / 27.3 / 52.3 ms, 2048 (two workgroups
// per CU for lack of LDS) 20.5 / 31.7 / 52.1 ms, 512 17.9 / 34.3 / 68.8 ms.
constexpr int atomic_tile_for(int RQ, int G, int CPL, int at_bytes) {
    const int fixed = (512 * CPL + 8 * G * CPL) * at_bytes + 8 * (kWave / G) * 4 + 64;
    int t = 1024;
    while (t > 256 && t * (16 * RQ + 6) + fixed > 64 * 1024) t >>= 1;
    return t;
}

template <int D, int G, int CPL, class VT, class AT>
struct AtomicTileShared {
    static constexpr int RQ = RecShape<D, VT>::RQ, NG = kWave / G, NW = kBlock / kWave;
    static constexpr int T = atomic_tile_for(RQ, G, CPL, (int)sizeof(AT));
    static constexpr int E = T / kBlock;      // sorted positions per thread
    static constexpr int WS = T / NW;         // sorted positions per wavefront
    int4 rec[T * RQ];                // the tile's records, in storage order
    int key[T];                      // mode-n subscripts, sorted in place
    uint16_t pos[T];                 // tile position of each sorted subscript
    AT part[NW][2 * NG][G * CPL];    // first / last row of every lane group
    int pkey[NW][2 * NG];
    AT wpart[2 * NW][G * CPL];       // first / last row of every wavefront
    int wkey[2 * NW];
};

template <int D, int G, int CPL, class VT, class AT>
constexpr size_t atomic_tile_smem_bytes() {
    return (sizeof(AtomicTileShared<D, G, CPL, VT, AT>) + 15) / 16 * 16;
}

// compare-exchange for a bitonic stage: the pair at sorted position p keeps the smaller key when
// it is the lower position of an ascending block (or the upper one of a descending block)
__device__ __forceinline__ void bitonic_take(int &k, int &q, int ko, int qo, bool take_min) {
    const bool swap = take_min ? (ko < k) : (ko > k);
    k = swap ? ko : k;
    q = swap ? qo : q;
}

// Sorts sm.key[0..T) (with sm.pos) ascending.  Thread t holds positions E t .. E t + E - 1.
template <class SM>
__device__ __forceinline__ void tile_sort(SM &sm) {
    constexpr int E = SM::E, T = SM::T;
    const int base = threadIdx.x * E;
    int k[E], q[E];
#pragma unroll
    for (int i = 0; i < E; ++i) {
        k[i] = sm.key[base + i];
        q[i] = base + i;
    }
    for (int size = 2; size <= T; size <<= 1) {
        for (int stride = size >> 1; stride >= E; stride >>= 1) {
            // partners live in other threads: publish, then read the partner's pair
#pragma unroll
            for (int i = 0; i < E; ++i) {
                sm.key[base + i] = k[i];
                sm.pos[base + i] = (uint16_t)q[i];
            }
            const bool block_wide = stride >= SM::WS;
            if (block_wide) __syncthreads(); else wave_sync();
            int ko[E], qo[E];
#pragma unroll
            for (int i = 0; i < E; ++i) {
                const int p = base + i, o = p ^ stride;
                ko[i] = sm.key[o];
                qo[i] = sm.pos[o];
            }
            // the next stage overwrites these slots: every reader must be done first (within a
            // wavefront the reads above complete before any later write is issued)
            if (block_wide) __syncthreads();
#pragma unroll
            for (int i = 0; i < E; ++i) {
                const int p = base + i;
                const bool asc = (p & size) == 0, lower = (p & stride) == 0;
                bitonic_take(k[i], q[i], ko[i], qo[i], asc == lower);
            }
        }
        // strides below E: pairs inside this thread's eight positions
#pragma unroll
        for (int stride = E / 2; stride > 0; stride >>= 1) {
            if (stride >= size) continue;
#pragma unroll
            for (int i = 0; i < E; ++i) {
                if (i & stride) continue;
                const int j = i + stride;
                const bool asc = ((base + i) & size) == 0;
                const bool sw = asc ? (k[j] < k[i]) : (k[j] > k[i]);
                const int tk = k[i], tq = q[i];
                k[i] = sw ? k[j] : k[i];
                q[i] = sw ? q[j] : q[i];
                k[j] = sw ? tk : k[j];
                q[j] = sw ? tq : q[j];
            }
        }
    }
#pragma unroll
    for (int i = 0; i < E; ++i) {
        sm.key[base + i] = k[i];
        sm.pos[base + i] = (uint16_t)q[i];
    }
    __syncthreads();
}

// Combines the partial rows parts[0..cnt) (keys ks, -1 = none) of one lane group's columns in
// sorted order: runs of equal keys are summed.  Runs in between the first and the last are added
// to V with one atomic per column; the first run goes to (first_out, *first_key) and the last
// run, when it differs from the first, to (last_out, *last_key) -- or, with FINAL, to V as well.
// Called by the G lanes of one group.
template <bool FINAL, int CPL, class AT, class PA>
__device__ __forceinline__ void combine_runs(const PA &parts, const int *ks, int cnt, int col0,
                                             bool colok, int gl, AT *__restrict__ V, int R,
                                             AT *first_out, int *first_key, AT *last_out,
                                             int *last_key) {
    int ck = -1;
    bool first_run = true;
    AT acc[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) acc[c] = 0;
    for (int e = 0; e < cnt; ++e) {
        const int ke = ks[e];
        if (ke < 0) continue;
        if (ke != ck) {
            if (ck >= 0) {
                if (first_run && !FINAL) {
#pragma unroll
                    for (int c = 0; c < CPL; ++c) first_out[col0 + c] = acc[c];
                    if (gl == 0) *first_key = ck;
                } else if (colok) {
                    atomic_cols<AT, CPL>(V + (int64_t)ck * R + col0, acc);
                }
                first_run = false;
            }
            ck = ke;
#pragma unroll
            for (int c = 0; c < CPL; ++c) acc[c] = 0;
        }
#pragma unroll
        for (int c = 0; c < CPL; ++c) acc[c] += parts[e][col0 + c];
    }
    if constexpr (FINAL) {
        if (ck >= 0 && colok) atomic_cols<AT, CPL>(V + (int64_t)ck * R + col0, acc);
    } else {
        if (gl == 0) {
            *last_key = -1;
            if (first_run) *first_key = ck;
        }
        if (ck >= 0) {
            AT *dst = first_run ? first_out : last_out;
#pragma unroll
            for (int c = 0; c < CPL; ++c) dst[col0 + c] = acc[c];
            if (!first_run && gl == 0) *last_key = ck;
        }
    }
}

// One workgroup processes the storage positions [r0, r1) tile by tile.  Every thread of the
// workgroup must call it.
template <int D, int G, int CPL, class FT, class VT, class AT, int UMAX = 64>
__device__ __forceinline__ void atomic_tile_range(AtomicTileShared<D, G, CPL, VT, AT> &sm,
                                                  const int4 *__restrict__ rec, int n, int R,
                                                  const FactorSet<FT> &A,
                                                  const double *__restrict__ lambda,
                                                  const VT *__restrict__ vovr,
                                                  AT *__restrict__ V, int64_t r0, int64_t r1) {
    using SM = AtomicTileShared<D, G, CPL, VT, AT>;
    constexpr int RW = RecShape<D, VT>::RW, RQ = RecShape<D, VT>::RQ;
    constexpr int NG = SM::NG, NW = SM::NW, T = SM::T;
    constexpr int S = SM::WS / NG;  // sorted positions per lane group
    constexpr int U0 = UnrollFor<KERNEL_ATOMIC, G, CPL, FT>::value;
    constexpr int U = U0 < UMAX ? U0 : UMAX;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane / G, gl = lane % G;
    const int col0 = gl * CPL;
    const bool colok = col0 < R;
    const uint32_t rowbytes = (uint32_t)R * sizeof(FT);
    const uint32_t colbytes = colok ? (uint32_t)col0 * sizeof(FT) : 0u;
    const OtherModes<D> om = other_modes<D>(A, n);
    AT lam[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c)
        lam[c] = (lambda != nullptr && colok) ? (AT)lambda[col0 + c] : (AT)1;

    for (int64_t t0 = r0; t0 < r1; t0 += T) {
        const int valid = (int)((r1 - t0) < T ? (r1 - t0) : T);
        // 1. stage the tile (coalesced), subscripts to sort; past the end: sentinel keys that
        // sort last and are never processed
#pragma unroll
        for (int r = 0; r < SM::E; ++r) {
            const int e = tid + r * kBlock;
            int k = 0x7fffffff;
            if (e < valid) {
                const int4 *src = rec + (t0 + e) * RQ;
                sm.rec[e * RQ] = load_stream(src);
                if constexpr (RQ == 2) sm.rec[e * RQ + 1] = load_stream(src + 1);
                if (vovr != nullptr)
                    rec_set_value<VT, RW>(reinterpret_cast<int *>(&sm.rec[e * RQ]), vovr[t0 + e]);
                k = lds_sub<RW>(&sm.rec[e * RQ], n);
            }
            sm.key[e] = k;
        }
        __syncthreads();
        // 2. sort the subscripts
        tile_sort(sm);
        // 3. segmented sums over this wavefront's quarter of the sorted tile
        const int gb = wave * SM::WS + g * S;
        const int ge = (gb + S < valid) ? gb + S : valid;
        int key = -1, first_key = -1;
        AT acc[CPL];
#pragma unroll
        for (int c = 0; c < CPL; ++c) acc[c] = 0;
        if (gl == 0) {
            sm.pkey[wave][2 * g] = -1;
            sm.pkey[wave][2 * g + 1] = -1;
        }
        for (int s0 = gb; s0 < ge; s0 += U) {
            AT t[U][CPL];
            int kk[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                kk[u] = -1;
                if (s0 + u < ge) {
                    const int q = sm.pos[s0 + u];
                    int w[RW];
                    lds_record<RQ>(&sm.rec[q * RQ], w);
                    kk[u] = sm.key[s0 + u];
                    entry_product<D, RW, CPL, FT, VT, AT>(w, om, rowbytes, colbytes, lam, t[u]);
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (kk[u] < 0) continue;
                if (kk[u] != key) {
                    if (key >= 0) {
                        if (key == first_key) {
#pragma unroll
                            for (int c = 0; c < CPL; ++c) sm.part[wave][2 * g][col0 + c] = acc[c];
                            if (gl == 0) sm.pkey[wave][2 * g] = key;
                        } else if (colok) {
                            atomic_cols<AT, CPL>(V + (int64_t)key * R + col0, acc);
                        }
                    } else {
                        first_key = kk[u];
                    }
                    key = kk[u];
#pragma unroll
                    for (int c = 0; c < CPL; ++c) acc[c] = 0;
                }
#pragma unroll
                for (int c = 0; c < CPL; ++c) acc[c] += t[u][c];
            }
        }
        if (key >= 0) {
            // the last row (also the first, when the slice holds one row: its first slot stays
            // empty)
#pragma unroll
            for (int c = 0; c < CPL; ++c) sm.part[wave][2 * g + 1][col0 + c] = acc[c];
            if (gl == 0) sm.pkey[wave][2 * g + 1] = key;
        }
        wave_sync();
        // the groups' first and last rows, in sorted order: inner runs go to V, the wavefront's
        // first and last rows to the workgroup
        if (g == 0)
            combine_runs<false, CPL, AT>(sm.part[wave], sm.pkey[wave], 2 * NG, col0, colok, gl, V,
                                         R, sm.wpart[2 * wave], &sm.wkey[2 * wave],
                                         sm.wpart[2 * wave + 1], &sm.wkey[2 * wave + 1]);
        __syncthreads();
        // 4. the wavefronts' first and last rows: one atomic per distinct row
        if (wave == 0 && g == 0)
            combine_runs<true, CPL, AT>(sm.wpart, sm.wkey, 2 * NW, col0, colok, gl, V, R, nullptr,
                                        nullptr, nullptr, nullptr);
        __syncthreads();
    }
}

template <int D, int G, int CPL, class FT, class VT, class AT>
__global__ __launch_bounds__(kBlock) void k_mttkrp_atomic(
    const int4 *__restrict__ rec, int64_t P, int n, int R, FactorSet<FT> A,
    const double *__restrict__ lambda, const VT *__restrict__ vovr, AT *__restrict__ V,
    int64_t per_block) {
    extern __shared__ int4 smem4[];
    using SM = AtomicTileShared<D, G, CPL, VT, AT>;
    const int64_t r0 = (int64_t)blockIdx.x * per_block;
    const int64_t r1 = (r0 + per_block < P) ? r0 + per_block : P;
    atomic_tile_range<D, G, CPL, FT, VT, AT>(*reinterpret_cast<SM *>(smem4), rec, n, R, A,
                                             lambda, vovr, V, r0, r1);
}

// Privatised output for short modes (Sec. 8 proposes private result copies reduced afterwards,
// a hybrid of the atomic and the reduction strategies): one LDS copy of the whole V per
// workgroup, each product row added there with LDS atomics, and one flush of the non-zero
// entries per workgroup.  The workgroup processes storage positions [bc0, bc0 + 4 chunk), one
// chunk per wavefront.  Every thread of the workgroup must call it.
template <int D, int G, int CPL, class FT, class VT, class AT>
__device__ __forceinline__ void privatized_block_unit(int4 *smem4, const int4 *__restrict__ rec,
                                                      int64_t P, int n, int R,
                                                      const FactorSet<FT> &A,
                                                      const double *__restrict__ lambda,
                                                      const VT *__restrict__ vovr,
                                                      AT *__restrict__ V, int chunk, int In,
                                                      int64_t bc0) {
    constexpr int RW = RecShape<D, VT>::RW, RQ = RecShape<D, VT>::RQ;
    constexpr int RP = G * CPL;
    constexpr int U = UnrollFor<KERNEL_ATOMIC, G, CPL, FT>::value;
    constexpr int GS = staged_group_stride(G, RQ);
    int4 *s_rec = smem4 + (threadIdx.x >> 6) * ((kWave / G) * GS);
    AT *pvals = reinterpret_cast<AT *>(smem4 + (kBlock / kWave) * (kWave / G) * GS);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane / G, gl = lane % G;
    const int col0 = gl * CPL;
    const bool colok = col0 < R;
    const uint32_t rowbytes = (uint32_t)R * sizeof(FT);
    const uint32_t colbytes = colok ? (uint32_t)col0 * sizeof(FT) : 0u;
    const OtherModes<D> om = other_modes<D>(A, n);
    for (int i = tid; i < In * RP; i += kBlock) pvals[i] = 0;
    __syncthreads();

    AT lam[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c)
        lam[c] = (lambda != nullptr && colok) ? (AT)lambda[col0 + c] : (AT)1;

    const int64_t c0 = bc0 + (int64_t)wave * chunk;
    const int64_t c1 = (c0 + chunk < P) ? c0 + chunk : P;
    const int len = c1 > c0 ? (int)(c1 - c0) : 0;
    const int nb = (len + kWave - 1) / kWave;
    for (int b = 0; b < nb; ++b) {
        const int off = b * kWave + lane;
        if (off < len) {
            const int4 *r = rec + (c0 + off) * RQ;
            s_rec[g * GS + gl * RQ] = r[0];
            if constexpr (RQ == 2) s_rec[g * GS + gl * RQ + 1] = r[1];
            if (vovr != nullptr)
                rec_set_value<VT, RW>(reinterpret_cast<int *>(&s_rec[g * GS + gl * RQ]),
                                      vovr[c0 + off]);
        }
        wave_sync();
        int cnt = len - b * kWave - g * G;
        cnt = cnt < G ? cnt : G;
        for (int s0 = 0; s0 < cnt; s0 += U) {
            AT t[U][CPL];
            int kk[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int s = s0 + u;
                kk[u] = -1;
                if (s < cnt) {
                    int w[RW];
                    lds_record<RQ>(&s_rec[g * GS + s * RQ], w);
                    kk[u] = lds_sub<RW>(&s_rec[g * GS + s * RQ], n);
                    entry_product<D, RW, CPL, FT, VT, AT>(w, om, rowbytes, colbytes, lam, t[u]);
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (kk[u] < 0 || !colok) continue;
#pragma unroll
                for (int c = 0; c < CPL; ++c) atomicAdd(&pvals[kk[u] * RP + col0 + c], t[u][c]);
            }
        }
        wave_sync();
    }
    __syncthreads();
    // skip untouched entries: adding zero changes nothing
    for (int i = tid; i < In * RP; i += kBlock) {
        const int row = i / RP, col = i - row * RP;
        if (col < R && pvals[i] != (AT)0) atomic_add_f(V + (int64_t)row * R + col, pvals[i]);
    }
}

template <int D, int G, int CPL, class FT, class VT, class AT>
__global__ __launch_bounds__(kBlock) void k_mttkrp_privatized(
    const int4 *__restrict__ rec, int64_t P, int n, int R, FactorSet<FT> A,
    const double *__restrict__ lambda, const VT *__restrict__ vovr, AT *__restrict__ V,
    int chunk, int In) {
    extern __shared__ int4 smem4[];
    privatized_block_unit<D, G, CPL, FT, VT, AT>(smem4, rec, P, n, R, A, lambda, vovr, V, chunk, In,
                                                 (int64_t)blockIdx.x * (kBlock / kWave) * chunk);
}

// ------------------------------------------------------------------------------------------
// launch dispatch over (order, lane config) for one dtype triple
// ------------------------------------------------------------------------------------------

// spt_tune.flags bit set by the library (never by callers) when nnz_per_wave took the default
constexpr int kTuneChunkDefaulted = 1 << 30;

struct MttkrpArgs {
    const int4 *rec;
    const int32_t *perm;
    const int4 *srec;
    int64_t P;
    int n, R;
    const double *lambda;
    const void *vovr;
    void *V;
    int chunk;
    int privatized;   // atomic algorithm into a per-workgroup LDS copy of the whole output
    int algo;
    int *slot_keys;   // deterministic mode: 2 slots per wave chunk (null: boundary atomics)
    void *slot_vals;
    int In;           // output rows (privatised mode)
    int auto_chunk;   // chunk is the default and may be matched to the resident capacity
    int cus;          // compute units of the device
    int *query_chunk; // non-null: store the chunk the launch would use, launch nothing
    hipStream_t stream;
};

// Default wave chunk of the permuted kernel over sorted record copies, for layouts of 4 or more
// columns per lane (gathering through the permutation prefers the short default): the fewest
// rounds k of the wavefronts the whole GPU holds at once (cap) whose chunk ceil(P / (k cap)),
// rounded up to 64 entries, stays within 32768, so the wave count lands just under a whole
// number of rounds instead of leaving a partial last round.  Measured on MI355X (1e8-entry
// power-law tensor, R = 32): 32768-entry chunks 3.39 ms, 4096 3.73, 24576 (1.3 rounds) 4.55.
// Chunks below 8192 keep the default.
inline int capacity_chunk(int64_t P, int64_t cap, int dflt) {
    if (cap <= 0) return dflt;
    for (int64_t k = 1; k <= 1024; ++k) {
        int64_t c = ceil_div(P, k * cap);
        c = ceil_div(c, 64) * 64;
        if (c <= 32768) return c >= 8192 ? (int)c : dflt;
    }
    return dflt;
}

template <class AT>
inline size_t privatized_smem_bytes(int RQ, int G, int In, int RP) {
    return (size_t)(kBlock / kWave) * (kWave / G) * staged_group_stride(G, RQ) * 16 +
           (size_t)In * RP * sizeof(AT);
}

template <int D, int G, int CPL, class FT, class VT, class AT>
int launch_cfg(const MttkrpArgs &a, const FactorSet<FT> &A) {
    const VT *vovr = static_cast<const VT *>(a.vovr);
    AT *V = static_cast<AT *>(a.V);
    const int64_t per_block = (int64_t)a.chunk * (kBlock / kWave);
    const unsigned grid = (unsigned)ceil_div(a.P, per_block);
    if (grid == 0) return SPT_OK;
    if (a.algo == SPT_ALGO_PERMUTED || a.algo == SPT_ALGO_PERMUTED_COPY) {
        int chunk = a.chunk;
        if (a.auto_chunk && a.slot_keys == nullptr && a.srec != nullptr && CPL >= 4 &&
            (sizeof(FT) == 2 || (sizeof(FT) == 4 && a.R <= 64))) {
            // resident wavefronts of this instantiation on the whole device (queried once);
            // FP64 factors, and FP32 ones above R = 64, keep the default chunk (8192-entry
            // chunks ran 4% faster than the matched 24-32k ones at R = 32 in FP64, 4096-entry
            // chunks 3.5% faster at R = 128 in FP32)
            static const int per_cu = [] {
                int nb = 0;
                if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                        &nb, k_mttkrp_perm<D, G, CPL, FT, VT, AT>, kBlock, 0) != hipSuccess)
                    nb = 0;
                return nb * (kBlock / kWave);
            }();
            chunk = capacity_chunk(a.P, (int64_t)per_cu * a.cus, chunk);
        }
        if (a.query_chunk != nullptr) {
            *a.query_chunk = chunk;
            return SPT_OK;
        }
        const unsigned pgrid = (unsigned)ceil_div(a.P, (int64_t)chunk * (kBlock / kWave));
        hipLaunchKernelGGL((k_mttkrp_perm<D, G, CPL, FT, VT, AT>), dim3(pgrid), dim3(kBlock), 0,
                           a.stream, a.rec, a.perm, a.srec, a.P, a.n, a.R, A, a.lambda, vovr, V,
                           chunk, a.slot_keys, static_cast<AT *>(a.slot_vals));
        if (a.slot_keys != nullptr) {
            const int64_t nslots = 2 * ceil_div(a.P, a.chunk);
            hipLaunchKernelGGL((k_det_fixup<AT>), dim3((unsigned)ceil_div(nslots, kBlock / kWave)),
                               dim3(kBlock), 0, a.stream, a.slot_keys,
                               static_cast<const AT *>(a.slot_vals), nslots, a.R, V);
        }
    } else if (a.privatized) {
        if (a.query_chunk != nullptr) {
            *a.query_chunk = a.chunk;
            return SPT_OK;
        }
        const size_t smem = privatized_smem_bytes<AT>(RecShape<D, VT>::RQ, G, a.In, G * CPL);
        hipLaunchKernelGGL((k_mttkrp_privatized<D, G, CPL, FT, VT, AT>), dim3(grid), dim3(kBlock),
                           smem, a.stream, a.rec, a.P, a.n, a.R, A, a.lambda, vovr, V, a.chunk,
                           a.In);
    } else {
        if (a.query_chunk != nullptr) {
            *a.query_chunk = a.chunk;
            return SPT_OK;
        }
        // a workgroup takes four wave chunks of entries, rounded up to whole sorted tiles
        constexpr int T = AtomicTileShared<D, G, CPL, VT, AT>::T;
        const int64_t per_block = ceil_div((int64_t)a.chunk * (kBlock / kWave), T) * T;
        const unsigned agrid = (unsigned)ceil_div(a.P, per_block);
        const size_t smem = atomic_tile_smem_bytes<D, G, CPL, VT, AT>();
        hipLaunchKernelGGL((k_mttkrp_atomic<D, G, CPL, FT, VT, AT>), dim3(agrid), dim3(kBlock),
                           smem, a.stream, a.rec, a.P, a.n, a.R, A, a.lambda, vovr, V, per_block);
    }
    return hipGetLastError() == hipSuccess ? SPT_OK : SPT_EHIP;
}

template <int D, class FT, class VT, class AT>
int launch_d(const MttkrpArgs &a, const FactorSet<FT> &A, int G, int CPL) {
    switch (G * 16 + CPL) {
        case 4 * 16 + 4: return launch_cfg<D, 4, 4, FT, VT, AT>(a, A);
        case 4 * 16 + 8: return launch_cfg<D, 4, 8, FT, VT, AT>(a, A);
        case 8 * 16 + 1: return launch_cfg<D, 8, 1, FT, VT, AT>(a, A);
        case 8 * 16 + 2: return launch_cfg<D, 8, 2, FT, VT, AT>(a, A);
        case 8 * 16 + 4: return launch_cfg<D, 8, 4, FT, VT, AT>(a, A);
        case 8 * 16 + 8: return launch_cfg<D, 8, 8, FT, VT, AT>(a, A);
        case 16 * 16 + 1: return launch_cfg<D, 16, 1, FT, VT, AT>(a, A);
        case 16 * 16 + 2: return launch_cfg<D, 16, 2, FT, VT, AT>(a, A);
        case 16 * 16 + 4: return launch_cfg<D, 16, 4, FT, VT, AT>(a, A);
        case 16 * 16 + 8: return launch_cfg<D, 16, 8, FT, VT, AT>(a, A);
        case 32 * 16 + 1: return launch_cfg<D, 32, 1, FT, VT, AT>(a, A);
        case 32 * 16 + 2: return launch_cfg<D, 32, 2, FT, VT, AT>(a, A);
        case 32 * 16 + 4: return launch_cfg<D, 32, 4, FT, VT, AT>(a, A);
        case 32 * 16 + 8: return launch_cfg<D, 32, 8, FT, VT, AT>(a, A);
        case 64 * 16 + 1: return launch_cfg<D, 64, 1, FT, VT, AT>(a, A);
        case 64 * 16 + 2: return launch_cfg<D, 64, 2, FT, VT, AT>(a, A);
        case 64 * 16 + 4: return launch_cfg<D, 64, 4, FT, VT, AT>(a, A);
        default: return SPT_EUNSUPPORTED;
    }
}

template <class FT, class VT, class AT>
int launch_typed(const MttkrpArgs &a, int d, const void *const *factors, int G, int CPL) {
    FactorSet<FT> A{};
    for (int m = 0; m < d; ++m) A.p[m] = static_cast<const FT *>(factors[m]);
    switch (d) {
        case 2: return launch_d<2, FT, VT, AT>(a, A, G, CPL);
        case 3: return launch_d<3, FT, VT, AT>(a, A, G, CPL);
        case 4: return launch_d<4, FT, VT, AT>(a, A, G, CPL);
        case 5: return launch_d<5, FT, VT, AT>(a, A, G, CPL);
        default: return SPT_EUNSUPPORTED;
    }
}

int launch_mttkrp_f64(const MttkrpArgs &a, int d, const void *const *factors, int G, int CPL);
int launch_mttkrp_f32(const MttkrpArgs &a, int d, const void *const *factors, int G, int CPL);
int launch_mttkrp_bf16(const MttkrpArgs &a, int d, const void *const *factors, int G, int CPL);

}  // namespace spt
