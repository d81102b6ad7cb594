// CP-ALS on the GPU (Sec. 3 defers the algorithm to Kolda & Bader; this is the textbook update):
// Gram matrices, their Hadamard product, an R x R Cholesky factorisation, row-parallel
// triangular solves, column normalisation, and the fit computed from the stored entries (or,
// after a mode update, from that mode's MTTKRP).  All of it in FP64; factors are stored in
// FP64, FP32 or BF16.
#include <algorithm>
#include <mutex>

#include "mttkrp_kernels.h"

namespace spt {

constexpr int kCpSmallR = 64;       // register / LDS-resident kernels up to this rank
constexpr int kCpMaxR = 256;        // largest rank of the CP-ALS and model calls
// workgroups of one Gram call above kCpSmallR (row ranges x 128 x 128 output blocks of the upper
// triangle): about one round at three per CU; 100 MB of partials at R = 128, 134 MB at 256
constexpr int kBigGramWgs = 768;
constexpr int kCholB = 16;          // block size of the large-rank Cholesky factor and inverse
constexpr int kCholMaxRp = 256;     // kCpMaxR rounded up to kCholB
constexpr int kGramRows = 64;       // rows staged per tile in the Gram kernel
constexpr int kMaxPartBlocks = 1024;
constexpr int kModelMaxBlocks = 2048;  // workgroups of the model pass (fit, GCP forward)

struct CpWs {
    size_t V, Y, L, Lx, Xinv, Ginv, gpart, cpart, misc, total;
};

// partial Grams one Gram call writes (each R x R doubles)
static int gram_parts(int R) {
    if (R <= kCpSmallR) return kMaxPartBlocks;
    const int nbk = (R + 127) / 128;  // output blocks of 128 columns (kGemmTile)
    const int blocks = nbk * (nbk + 1) / 2;
    return (kBigGramWgs + blocks - 1) / blocks;
}

static CpWs cp_layout(int64_t Imax, int R) {
    CpWs w;
    size_t o = 0;
    w.V = o;
    o += align256((size_t)Imax * R * 8);
    w.Y = o;
    o += align256((size_t)Imax * R * 8);
    w.L = o;
    o += align256((size_t)R * R * 8);
    // above kCpSmallR: W (Gamma padded to a multiple of 16, factored in place), X = L^-1, and
    // Gamma^-1
    const size_t rp = (size_t)(R + kCholB - 1) / kCholB * kCholB;
    const size_t big = R > kCpSmallR ? align256(rp * rp * 8) : 0;
    w.Lx = o;
    w.Xinv = o + big;
    w.Ginv = w.Xinv + big;
    o = w.Ginv + big;
    w.gpart = o;  // Gram / column partials (R x R per block), or fit partials (2 per block)
    o += align256((size_t)std::max<size_t>((size_t)gram_parts(R) * R * R,
                                           std::max<size_t>((size_t)kMaxPartBlocks * R,
                                                            2 * kModelMaxBlocks)) * 8);
    w.cpart = o;  // Y^T Y
    o += align256((size_t)R * R * 8);
    w.misc = o;
    o += align256(64 * 8);
    w.total = o;
    return w;
}

template <class FT>
__device__ __forceinline__ double load_f64(const FT *p) {
    if constexpr (sizeof(FT) == 2) return (double)bf16_bits_to_f32(*reinterpret_cast<const uint16_t *>(p));
    else return (double)*p;
}

template <class FT>
__device__ __forceinline__ void store_from_f64(FT *p, double v) {
    if constexpr (sizeof(FT) == 2) *reinterpret_cast<uint16_t *>(p) = f64_to_bf16_rne(v);
    else *p = (FT)v;
}

// deterministic block sum of one double per thread (result valid in every thread)
__device__ double block_sum_f64(double v) {
    __shared__ double red[kBlock / kWave];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kBlock / kWave; ++w) s += red[w];
    return s;
}

// ------------------------------------------------------------------------------------------
// Gram matrices  G = A^T A  (FP64).  Optionally normalises and stores the factor first.
// ------------------------------------------------------------------------------------------

// Tile of rows -> per-block partial Gram.  With NORMALIZE, the tile comes from the FP64 solve
// output Y: a = y / lambda (columns with lambda > 0), stored to A in FT, and the Gram uses the
// stored (rounded) values.  Thread (ta, tb) of a 16 x 16 arrangement accumulates the B x B block
// of G at rows ta*B.., columns tb*B.. (B = ceil(R / 16)): 2B LDS reads feed B*B FMAs, and every
// entry still sums its rows in increasing order.
template <class FT, bool NORMALIZE, int B>
__global__ __launch_bounds__(kBlock) void k_gram_partial(const FT *__restrict__ Ain,
                                                         const double *__restrict__ Y,
                                                         const double *__restrict__ lambda,
                                                         FT *__restrict__ Aout, int64_t I, int R,
                                                         double *__restrict__ gpart) {
    __shared__ double tile[kGramRows][kCpSmallR + 1];
    const int tid = threadIdx.x;
    const int a0 = (tid >> 4) * B, b0 = (tid & 15) * B;
    double acc[B][B];
#pragma unroll
    for (int x = 0; x < B; ++x)
#pragma unroll
        for (int y = 0; y < B; ++y) acc[x][y] = 0.0;
    for (int64_t r0 = (int64_t)blockIdx.x * kGramRows; r0 < I; r0 += (int64_t)gridDim.x * kGramRows) {
        const int nrows = (I - r0 < kGramRows) ? (int)(I - r0) : kGramRows;
        for (int e = tid; e < kGramRows * R; e += kBlock) {
            const int rr = e / R, c = e - rr * R;
            double v = 0.0;
            if (rr < nrows) {
                const int64_t idx = (r0 + rr) * R + c;
                if constexpr (NORMALIZE) {
                    double y = Y[idx];
                    const double l = lambda[c];
                    if (l > 0.0) y = y / l;
                    store_from_f64<FT>(Aout + idx, y);
                    v = load_f64<FT>(Aout + idx);
                } else {
                    v = load_f64<FT>(Ain + idx);
                }
            }
            tile[rr][c] = v;
        }
        __syncthreads();
        if (a0 < R && b0 < R) {
            for (int rr = 0; rr < nrows; ++rr) {
                double va[B], vb[B];
#pragma unroll
                for (int x = 0; x < B; ++x) {
                    va[x] = tile[rr][a0 + x];  // blocks past column R are never stored
                    vb[x] = tile[rr][b0 + x];
                }
#pragma unroll
                for (int x = 0; x < B; ++x)
#pragma unroll
                    for (int y = 0; y < B; ++y) acc[x][y] += va[x] * vb[y];
            }
        }
        __syncthreads();
    }
    const int RR = R * R;
#pragma unroll
    for (int x = 0; x < B; ++x)
#pragma unroll
        for (int y = 0; y < B; ++y)
            if (a0 + x < R && b0 + y < R)
                gpart[(int64_t)blockIdx.x * RR + (a0 + x) * R + (b0 + y)] = acc[x][y];
}

// out[i] = sum over the partials b = 0..nblk-1, one wavefront per entry: lane l adds partials
// l, l + 64, ... in order, then the 64 lane sums combine in a fixed butterfly.  The order is
// fixed for a given nblk, so the result is reproducible run to run.
__global__ __launch_bounds__(kBlock) void k_sum_parts(const double *__restrict__ part, int nblk,
                                                      int len, double *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * (kBlock / kWave) + (threadIdx.x >> 6);
    if (i >= len) return;  // whole wavefront
    double s = 0.0;
    for (int b = lane; b < nblk; b += kWave) s += part[(int64_t)b * len + i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) out[i] = s;
}

// ------------------------------------------------------------------------------------------
// Hadamard product of the other modes' Grams (the whole workgroup) and its Cholesky factor (the
// first wavefront alone).  Lane r owns row r of L in registers; row c of L, which lane c wrote
// to LDS as it computed it, is read into registers with independent LDS broadcasts at the start
// of column step c, so each step is one dependent chain of register arithmetic; the steps
// synchronise with wave barriers.  Same column-by-column order and operation order as the
// textbook algorithm, and no FMA contraction, so the factor follows the plain definition's
// rounding.  Lanes from R on compute on unused rows and store nothing.
template <int RMAX>
__global__ __launch_bounds__(kBlock) void k_hadamard_chol(const double *__restrict__ grams, int d,
                                                          int n, int R, double *__restrict__ L,
                                                          SptStatusBlock *st) {
#pragma clang fp contract(off)
    __shared__ double S[kCpSmallR][kCpSmallR];
    __shared__ double Lc[kCpSmallR][kCpSmallR];
    __shared__ double lcc_s;
    __shared__ int bad;
    const int tid = threadIdx.x;
    if (tid == 0) bad = 0;
    for (int e = tid; e < kCpSmallR * kCpSmallR; e += kBlock) Lc[e / kCpSmallR][e % kCpSmallR] = 0.0;
    for (int ab = tid; ab < R * R; ab += kBlock) {
        double g = 1.0;
        for (int m = 0; m < d; ++m)
            if (m != n) g *= grams[(int64_t)m * R * R + ab];
        S[ab / R][ab % R] = g;
    }
    __syncthreads();
    if (tid >= kWave) return;
    const int r = tid;
    double maxdiag = 0.0;
    for (int k = 0; k < R; ++k) maxdiag = S[k][k] > maxdiag ? S[k][k] : maxdiag;
    const double tol = (double)R * 2.220446049250313e-16 * maxdiag;
    // Column step c: every lane forms s = S[r][c] - sum_k L[r][k] L[c][k] over the 8-column chunks
    // that start before c; the terms from column c on are 0 * 0 (neither row has them yet) and
    // leave s unchanged, so the sums equal the textbook ones term for term.  Lane c's s is the
    // pivot.
    double row[RMAX];
#pragma unroll
    for (int k = 0; k < RMAX; ++k) row[k] = 0.0;
    for (int c = 0; c < R; ++c) {
        // row c of L so far (LDS broadcasts) and s = S[r][c] - sum_k L[r][k] L[c][k], in chunks
        // of 8 columns; chunks that start at or after c hold only 0 * 0 terms and are skipped
        // (c is uniform, so whole chunks are branched over and the sums stay the same)
        double lrow[RMAX];
        double sacc = S[r][c];
#pragma unroll
        for (int kb = 0; kb < RMAX; kb += 8) {
            if (kb < c) {
#pragma unroll
                for (int k = kb; k < kb + 8; ++k) lrow[k] = Lc[c][k];
#pragma unroll
                for (int k = kb; k < kb + 8; ++k) sacc -= row[k] * lrow[k];
            }
        }
        if (r == c) {
            double piv = sacc;
            if (!(piv > tol)) {
                bad = 1;
                piv = 1.0;  // keep the factor finite; the status word reports the failure
            }
            lcc_s = sqrt(piv);
            Lc[c][c] = lcc_s;
        }
        wave_sync();
        const double lcc = lcc_s;
        double v = 0.0;
        if (r == c) v = lcc;
        if (r > c && r < R) {
            v = sacc / lcc;
            Lc[r][c] = v;
        }
#pragma unroll
        for (int k = 0; k < RMAX; ++k)
            if (k == c) row[k] = v;
        wave_sync();
    }
    for (int ab = tid; ab < R * R; ab += kWave) L[ab] = Lc[ab / R][ab % R];
    if (tid == 0 && bad) raise_status(st, SPT_ESINGULAR);
}

// ------------------------------------------------------------------------------------------
// Row solves: row k of the unnormalised factor solves  a Gamma = v  with Gamma = L L^T
// (forward substitution with L, then back substitution with L^T), in the textbook order, except
// that each step multiplies by the reciprocal of the diagonal entry (formed once per workgroup)
// instead of dividing by it: the FP64 division sits on every step's dependency chain, and the
// quotient changes by at most about one ulp (measured: R = 32 solve 76 us instead of 86).  One
// thread solves NR rows at once (NR = 2 up to R = 32) so that every L entry read from LDS feeds
// NR rows; L and its transpose sit in LDS zero-padded to RMAX columns and are read two entries
// per load (padded terms subtract 0 * 0 and leave the sums unchanged).  With VEC (R a multiple of
// 4) rows of V and Y move with 16-byte accesses.  The column 2-norms come afterwards from the
// column sums of squares of Y.
template <int RMAX, int NR, bool VEC, class VT>
__global__ __launch_bounds__(kBlock) void k_solve_rows(const VT *__restrict__ V, int64_t I, int R,
                                                       const double *__restrict__ Lg,
                                                       double *__restrict__ Y) {
#pragma clang fp contract(off)
    __shared__ double2 L2[RMAX][RMAX / 2];   // L[c][q] at L2[c][q/2], lower triangle
    __shared__ double2 LT2[RMAX][RMAX / 2];  // L[q][c] at LT2[c][q/2]
    __shared__ double dg[RMAX];              // 1 / L[c][c]
    const int tid = threadIdx.x;
    double *Lf = reinterpret_cast<double *>(&L2[0][0]);
    double *LTf = reinterpret_cast<double *>(&LT2[0][0]);
    for (int e = tid; e < RMAX * RMAX; e += kBlock) {
        const int r = e / RMAX, c = e - r * RMAX;
        const double v = (r < R && c < R) ? Lg[r * R + c] : 0.0;
        Lf[r * RMAX + c] = v;
        LTf[c * RMAX + r] = v;
        if (r == c) dg[r] = (r < R) ? 1.0 / v : 0.0;  // reciprocal diagonal
    }
    __syncthreads();
    // one pass per thread (the grid covers every row), so no L value is worth keeping in
    // registers across iterations
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    const int64_t k0 = (int64_t)blockIdx.x * kBlock + tid;
    {
        double a[NR][RMAX];
#pragma unroll
        for (int h = 0; h < NR; ++h) {
            const int64_t k = k0 + h * stride;
            if constexpr (VEC) {
                // 16-byte loads: a row is read with R/4 (FP32) or R/2 (FP64) instructions
                constexpr int W = 16 / (int)sizeof(VT);
#pragma unroll
                for (int c = 0; c < RMAX; c += W) {
                    if (c < R && k < I) {
                        if constexpr (W == 4) {
                            const float4 v = *reinterpret_cast<const float4 *>(V + k * R + c);
                            a[h][c] = v.x; a[h][c + 1] = v.y; a[h][c + 2] = v.z; a[h][c + 3] = v.w;
                        } else {
                            const double2 v = *reinterpret_cast<const double2 *>(V + k * R + c);
                            a[h][c] = v.x; a[h][c + 1] = v.y;
                        }
                    } else {
#pragma unroll
                        for (int w = 0; w < W; ++w) a[h][c + w] = 0.0;
                    }
                }
            } else {
#pragma unroll
                for (int c = 0; c < RMAX; ++c) a[h][c] = (c < R && k < I) ? (double)V[k * R + c] : 0.0;
            }
        }
        // forward: a_c = (v_c - sum_{q<c} L[c][q] a_q) / L[c][c]
#pragma unroll
        for (int c = 0; c < RMAX; ++c) {
            if (c < R) {
                double sv[NR];
#pragma unroll
                for (int h = 0; h < NR; ++h) sv[h] = a[h][c];
#pragma unroll
                for (int q = 0; q + 1 < c; q += 2) {
                    const double2 l = L2[c][q / 2];
#pragma unroll
                    for (int h = 0; h < NR; ++h) {
                        sv[h] -= l.x * a[h][q];
                        sv[h] -= l.y * a[h][q + 1];
                    }
                }
                if (c & 1) {
                    const double l = Lf[c * RMAX + c - 1];
#pragma unroll
                    for (int h = 0; h < NR; ++h) sv[h] -= l * a[h][c - 1];
                }
                const double d = dg[c];
#pragma unroll
                for (int h = 0; h < NR; ++h) a[h][c] = sv[h] * d;
            }
        }
        // backward: a_c = (a_c - sum_{q>c} L[q][c] a_q) / L[c][c], q ascending
#pragma unroll
        for (int c = RMAX - 1; c >= 0; --c) {
            if (c < R) {
                double sv[NR];
#pragma unroll
                for (int h = 0; h < NR; ++h) sv[h] = a[h][c];
                int q = c + 1;
                if (q & 1) {
                    if (q < RMAX) {
                        const double l = LTf[c * RMAX + q];
#pragma unroll
                        for (int h = 0; h < NR; ++h) sv[h] -= l * a[h][q];
                    }
                    ++q;
                }
#pragma unroll
                for (; q + 1 < RMAX + 1 && q < RMAX; q += 2) {
                    const double2 l = LT2[c][q / 2];
#pragma unroll
                    for (int h = 0; h < NR; ++h) {
                        sv[h] -= l.x * a[h][q];
                        sv[h] -= l.y * a[h][q + 1];
                    }
                }
                const double d = dg[c];
#pragma unroll
                for (int h = 0; h < NR; ++h) a[h][c] = sv[h] * d;
            }
        }
#pragma unroll
        for (int h = 0; h < NR; ++h) {
            const int64_t k = k0 + h * stride;
            if (k < I) {
                if constexpr (VEC) {
#pragma unroll
                    for (int c = 0; c < RMAX; c += 2)
                        if (c < R) *reinterpret_cast<double2 *>(Y + k * R + c) = make_double2(a[h][c], a[h][c + 1]);
                } else {
#pragma unroll
                    for (int c = 0; c < RMAX; ++c)
                        if (c < R) Y[k * R + c] = a[h][c];
                }
            }
        }
    }
}

// Column sums of squares of Y (I x R, FP64) as per-block partials in a fixed order: thread
// (q, c) = (tid / R, tid % R) sums column c over rows q, q + Q, ... of the block's 64-row tiles
// (Q = 256 / R rows per pass, consecutive threads read consecutive addresses), then the block
// adds its Q partial sums per column in order q = 0..Q-1.
__global__ __launch_bounds__(kBlock) void k_colsq_partial(const double *__restrict__ Y, int64_t I,
                                                          int R, double *__restrict__ part) {
    __shared__ double red[kBlock];
    const int tid = threadIdx.x;
    const int Q = kBlock / R;
    const int q = tid / R, c = tid - q * R;
    double acc = 0.0;
    if (q < Q) {
        for (int64_t r0 = (int64_t)blockIdx.x * kGramRows; r0 < I;
             r0 += (int64_t)gridDim.x * kGramRows) {
            const int64_t r1 = (r0 + kGramRows < I) ? r0 + kGramRows : I;
            for (int64_t r = r0 + q; r < r1; r += Q) {
                const double y = Y[r * R + c];
                acc += y * y;
            }
        }
    }
    red[tid] = acc;
    __syncthreads();
    if (tid < R) {
        double t = 0.0;
        for (int k = 0; k < Q; ++k) t += red[k * R + tid];
        part[(int64_t)blockIdx.x * R + tid] = t;
    }
}

// lambda_j = sqrt(sum_k Y(k, j)^2)
__global__ void k_norms(const double *__restrict__ sq, int R, double *__restrict__ lambda) {
    for (int c = threadIdx.x; c < R; c += blockDim.x) lambda[c] = sqrt(sq[c]);
}

// ------------------------------------------------------------------------------------------
// Ranks above kCpSmallR (up to 256): Gamma, its Cholesky factor and its inverse in global memory
// (L2-resident, R x R doubles each) with one workgroup, then the row solves as one FP64 GEMM
// V Gamma^-1, then normalisation and the Gram of the stored factor in 64 x 64 output blocks.
// ------------------------------------------------------------------------------------------

// Blocked Cholesky factor and inverse of Gamma in one workgroup, for 64 < R <= 256.  Gamma is
// padded to Rp = 16 nb columns with the identity; W (Rp x Rp, global, L2-resident) holds the
// Hadamard product of the other Grams and is factored in place, 16 x 16 blocks at a time:
//   a. the diagonal block by one wavefront (lane r holds row r; row c of the factor broadcast
//      through LDS before column step c; pivots <= R eps max diag(Gamma) raise SPT_ESINGULAR),
//   b. the panel below it by forward substitution (a thread per row, the diagonal block in LDS),
//   c. the trailing lower triangle minus the panel times its transpose (4 x 4 tiles per
//      thread, the panel in LDS).
// Then X = L^-1 (into Xg, Rp x Rp): the diagonal blocks' inverses (a thread per column), then
// block diagonals of increasing distance d, X_ik = -X_ii sum_{k <= j < i} L_ij X_jk (the pairs
// at one distance are independent).  Gamma^-1 = X^T X follows in k_xtx.

__global__ __launch_bounds__(kBlock) void k_chol_inverse_big(const double *__restrict__ grams,
                                                             int d, int n, int R, int Rp,
                                                             double *__restrict__ W,
                                                             double *__restrict__ Xg,
                                                             SptStatusBlock *st) {
#pragma clang fp contract(off)
    constexpr int B = kCholB;
    __shared__ double Lkk[B][B + 1];
    __shared__ double buf[(kCholMaxRp - B) * (B + 1)];  // the panel, later the T blocks
    __shared__ double maxdiag_s;
    __shared__ int bad;
    const int tid = threadIdx.x, lane = tid & 63;
    const int nb = Rp / B;
    for (int ab = tid; ab < Rp * Rp; ab += kBlock) {
        const int a = ab / Rp, b = ab - a * Rp;
        double g;
        if (a < R && b < R) {
            g = 1.0;
            for (int m = 0; m < d; ++m)
                if (m != n) g *= grams[(int64_t)m * R * R + a * R + b];
        } else {
            g = (a == b) ? 1.0 : 0.0;  // identity padding
        }
        W[ab] = g;
        Xg[ab] = 0.0;
    }
    __syncthreads();
    if (tid == 0) {
        double md = 0.0;
        for (int k = 0; k < R; ++k) md = W[k * Rp + k] > md ? W[k * Rp + k] : md;
        maxdiag_s = md;
        bad = 0;
    }
    __syncthreads();
    const double tol = (double)R * 2.220446049250313e-16 * maxdiag_s;
    for (int k = 0; k < nb; ++k) {
        const int k0 = k * B;
        // a. diagonal block, one wavefront: lane r < B owns row r
        if (tid < kWave) {
            const int r = lane;
            double row[B];
#pragma unroll
            for (int q = 0; q < B; ++q) row[q] = 0.0;
            for (int c = 0; c < B; ++c) {
                double sacc = (r < B) ? W[(k0 + r) * Rp + k0 + c] : 0.0;
#pragma unroll
                for (int q = 0; q < B; ++q)
                    if (q < c) sacc -= row[q] * Lkk[c][q];
                if (r == c) {
                    double piv = sacc;
                    if (k0 + c < R && !(piv > tol)) {
                        bad = 1;
                        piv = 1.0;  // keep the factor finite; the status word reports it
                    }
                    Lkk[c][c] = sqrt(piv);
                }
                wave_sync();
                const double lcc = Lkk[c][c];
                double v = 0.0;
                if (r == c) v = lcc;
                if (r > c && r < B) {
                    v = sacc / lcc;
                    Lkk[r][c] = v;
                }
#pragma unroll
                for (int q = 0; q < B; ++q)
                    if (q == c) row[q] = v;
                wave_sync();
            }
            if (r < B)
                for (int q = 0; q < B; ++q) W[(k0 + r) * Rp + k0 + q] = (q <= r) ? row[q] : 0.0;
        }
        __syncthreads();
        // b. panel: rows below the diagonal block solve z L_kk^T = w
        const int m = Rp - k0 - B;  // rows (and columns) of the trailing matrix
        if (tid < m) {
            const int i = k0 + B + tid;
            double z[B];
#pragma unroll
            for (int c = 0; c < B; ++c) z[c] = W[i * Rp + k0 + c];
#pragma unroll
            for (int c = 0; c < B; ++c) {
                double v = z[c];
#pragma unroll
                for (int q = 0; q < B; ++q)
                    if (q < c) v -= z[q] * Lkk[c][q];
                z[c] = v / Lkk[c][c];
            }
#pragma unroll
            for (int c = 0; c < B; ++c) {
                W[i * Rp + k0 + c] = z[c];
                buf[tid * (B + 1) + c] = z[c];
            }
        }
        __syncthreads();
        // c. trailing lower triangle: W_ij -= sum_q P_iq P_jq, 4 x 4 tiles per thread
        const int mt = (m + 3) / 4;
        for (int t = tid; t < mt * mt; t += kBlock) {
            const int ti = t / mt, tj = t - ti * mt;
            if (tj > ti) continue;
            double acc[4][4];
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y) acc[x][y] = 0.0;
#pragma unroll
            for (int q = 0; q < B; ++q) {
                double a[4], b[4];
#pragma unroll
                for (int x = 0; x < 4; ++x) {
                    const int ii = ti * 4 + x, jj = tj * 4 + x;
                    a[x] = ii < m ? buf[ii * (B + 1) + q] : 0.0;
                    b[x] = jj < m ? buf[jj * (B + 1) + q] : 0.0;
                }
#pragma unroll
                for (int x = 0; x < 4; ++x)
#pragma unroll
                    for (int y = 0; y < 4; ++y) acc[x][y] += a[x] * b[y];
            }
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y) {
                    const int ii = ti * 4 + x, jj = tj * 4 + y;
                    if (ii < m && jj < m && jj <= ii)
                        W[(k0 + B + ii) * Rp + k0 + B + jj] -= acc[x][y];
                }
        }
        __syncthreads();
    }
    // X = L^-1.  Diagonal blocks first: thread t inverts column t % B of block t / B.
    {
        const int k = tid / B, c = tid % B;
        if (k < nb) {
            const int k0 = k * B;
            double x[B];
#pragma unroll
            for (int i = 0; i < B; ++i) {
                double v = (i == c) ? 1.0 : 0.0;
#pragma unroll
                for (int q = 0; q < B; ++q)
                    if (q >= c && q < i) v -= W[(k0 + i) * Rp + k0 + q] * x[q];
                x[i] = (i < c) ? 0.0 : v / W[(k0 + i) * Rp + k0 + i];
            }
#pragma unroll
            for (int i = 0; i < B; ++i) Xg[(k0 + i) * Rp + k0 + c] = x[i];
        }
    }
    __syncthreads();
    // then the blocks at distance dist below the diagonal, all pairs of one distance at once
    for (int dist = 1; dist < nb; ++dist) {
        const int npairs = nb - dist;
        // T_ik = sum_{j = k .. i-1} L_ij X_jk into buf (pair p = k)
        for (int e = tid; e < npairs * B * B; e += kBlock) {
            const int k = e / (B * B), rc = e - k * B * B, r = rc / B, c = rc - r * B;
            const int i = k + dist;
            double v = 0.0;
            for (int j = k; j < i; ++j)
                for (int q = 0; q < B; ++q)
                    v += W[(i * B + r) * Rp + j * B + q] * Xg[(j * B + q) * Rp + k * B + c];
            buf[e] = v;
        }
        __syncthreads();
        // X_ik = -X_ii T_ik (X_ii lower triangular)
        for (int e = tid; e < npairs * B * B; e += kBlock) {
            const int k = e / (B * B), rc = e - k * B * B, r = rc / B, c = rc - r * B;
            const int i = k + dist;
            double v = 0.0;
            for (int q = 0; q <= r; ++q)
                v += Xg[(i * B + r) * Rp + i * B + q] * buf[k * B * B + q * B + c];
            Xg[(i * B + r) * Rp + k * B + c] = -v;
        }
        __syncthreads();
    }
    if (tid == 0 && bad) raise_status(st, SPT_ESINGULAR);
}

// Gamma^-1 = X^T X for the lower triangular X = L^-1 (Rp x Rp; rows past R are zero in the
// first R columns): 64 x 64 output tiles, the sum over rows in steps of 16 through LDS.
constexpr int kXtxTile = 64, kXtxK = 16;

__global__ __launch_bounds__(kBlock) void k_xtx(const double *__restrict__ Xg, int Rp, int R,
                                                double *__restrict__ Ginv) {
    __shared__ double As[kXtxK][kXtxTile + 1];
    __shared__ double Bs[kXtxK][kXtxTile + 1];
    const int tid = threadIdx.x, tr = tid / 16, tc = tid % 16;
    const int a0 = blockIdx.x * kXtxTile, b0 = blockIdx.y * kXtxTile;
    double acc[4][4];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = 0.0;
    const int t0 = (a0 > b0 ? a0 : b0) / kXtxK * kXtxK;  // X[t][a] = 0 below t < a
    for (int t = t0; t < Rp; t += kXtxK) {
        for (int e = tid; e < kXtxK * kXtxTile; e += kBlock) {
            const int tt = e / kXtxTile, cc = e - tt * kXtxTile;
            As[tt][cc] = (a0 + cc < Rp) ? Xg[(t + tt) * Rp + a0 + cc] : 0.0;
            Bs[tt][cc] = (b0 + cc < Rp) ? Xg[(t + tt) * Rp + b0 + cc] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int tt = 0; tt < kXtxK; ++tt) {
            double a[4], b[4];
#pragma unroll
            for (int x = 0; x < 4; ++x) a[x] = As[tt][tr * 4 + x];
#pragma unroll
            for (int y = 0; y < 4; ++y) b[y] = Bs[tt][tc * 4 + y];
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y) acc[x][y] += a[x] * b[y];
        }
        __syncthreads();
    }
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) {
            const int a = a0 + tr * 4 + x, b = b0 + tc * 4 + y;
            if (a < R && b < R) Ginv[a * R + b] = acc[x][y];
        }
}

// Y = V Gamma^-1 (I x R times R x R, FP64 products and sums): 128 x 128 output tiles, the
// reduction dimension in steps of 16 staged through LDS (transposed, so a thread's eight rows
// and eight columns are contiguous), 8 x 8 outputs per thread (64 FMAs per 16 LDS values).
constexpr int kGemmTile = 128, kGemmK = 16, kGemmSub = 8;

template <class VT>
__global__ __launch_bounds__(kBlock) void k_solve_gemm(const VT *__restrict__ V, int64_t I,
                                                       int R, const double *__restrict__ Ginv,
                                                       double *__restrict__ Y) {
    __shared__ double As[kGemmK][kGemmTile];  // As[k][row]
    __shared__ double Bs[kGemmK][kGemmTile];  // Bs[k][col]
    const int tid = threadIdx.x, tr = tid / 16, tc = tid % 16;
    const int64_t r0 = (int64_t)blockIdx.x * kGemmTile;
    const int c0 = blockIdx.y * kGemmTile;
    double acc[kGemmSub][kGemmSub];
#pragma unroll
    for (int x = 0; x < kGemmSub; ++x)
#pragma unroll
        for (int y = 0; y < kGemmSub; ++y) acc[x][y] = 0.0;
    for (int k0 = 0; k0 < R; k0 += kGemmK) {
        for (int e = tid; e < kGemmTile * kGemmK; e += kBlock) {
            const int rr = e / kGemmK, kk = e - rr * kGemmK;  // consecutive k along a row of V
            const int64_t row = r0 + rr;
            const int k = k0 + kk;
            As[kk][rr] = (row < I && k < R) ? (double)V[row * R + k] : 0.0;
        }
        for (int e = tid; e < kGemmK * kGemmTile; e += kBlock) {
            const int kk = e / kGemmTile, cc = e - kk * kGemmTile;
            const int k = k0 + kk, c = c0 + cc;
            Bs[kk][cc] = (k < R && c < R) ? Ginv[k * R + c] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kGemmK; ++kk) {
            double a[kGemmSub], b[kGemmSub];
#pragma unroll
            for (int x = 0; x < kGemmSub; ++x) a[x] = As[kk][tr * kGemmSub + x];
#pragma unroll
            for (int y = 0; y < kGemmSub; ++y) b[y] = Bs[kk][tc * kGemmSub + y];
#pragma unroll
            for (int x = 0; x < kGemmSub; ++x)
#pragma unroll
                for (int y = 0; y < kGemmSub; ++y) acc[x][y] += a[x] * b[y];
        }
        __syncthreads();
    }
#pragma unroll
    for (int x = 0; x < kGemmSub; ++x) {
        const int64_t row = r0 + tr * kGemmSub + x;
        if (row >= I) continue;
#pragma unroll
        for (int y = 0; y < kGemmSub; ++y) {
            const int c = c0 + tc * kGemmSub + y;
            if (c < R) Y[row * R + c] = acc[x][y];
        }
    }
}

// A = Y / lambda column by column (columns with lambda = 0 unscaled), stored in FT
template <class FT>
__global__ __launch_bounds__(kBlock) void k_normalize_store(const double *__restrict__ Y,
                                                            const double *__restrict__ lambda,
                                                            int64_t len, int R,
                                                            FT *__restrict__ A) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < len; i += stride) {
        double y = Y[i];
        const double l = lambda[i % R];
        if (l > 0.0) y = y / l;
        store_from_f64<FT>(A + i, y);
    }
}

// Partial Gram A^T A for one 128 x 128 output block (bi, bj) with bi <= bj (blockIdx.y indexes
// the upper block triangle row by row) over a range of rows (blockIdx.x of gridDim.x): rows
// staged 16 at a time in LDS, 8 x 8 outputs per thread, each entry summing its rows in
// increasing order.  An off-diagonal block is written to both (a, b) and (b, a).
constexpr int kBigGramRows = 16;

template <class FT>
__global__ __launch_bounds__(kBlock) void k_gram_big_partial(const FT *__restrict__ A, int64_t I,
                                                             int R, double *__restrict__ gpart) {
    __shared__ double Ta[kBigGramRows][kGemmTile];
    __shared__ double Tb[kBigGramRows][kGemmTile];
    const int tid = threadIdx.x, ta = tid / 16, tb = tid % 16;
    const int nbk = (R + kGemmTile - 1) / kGemmTile;
    int bi = 0, rem = blockIdx.y;
    while (rem >= nbk - bi) {  // blockIdx.y -> (bi, bj), bj >= bi
        rem -= nbk - bi;
        ++bi;
    }
    const int bj = bi + rem;
    const int ca = bi * kGemmTile, cb = bj * kGemmTile;
    const int64_t per = ceil_div(ceil_div(I, (int64_t)gridDim.x), (int64_t)kBigGramRows) * kBigGramRows;
    const int64_t rbeg = (int64_t)blockIdx.x * per;
    const int64_t rend = (rbeg + per < I) ? rbeg + per : I;
    double acc[kGemmSub][kGemmSub];
#pragma unroll
    for (int x = 0; x < kGemmSub; ++x)
#pragma unroll
        for (int y = 0; y < kGemmSub; ++y) acc[x][y] = 0.0;
    for (int64_t r0 = rbeg; r0 < rend; r0 += kBigGramRows) {
        for (int e = tid; e < kBigGramRows * kGemmTile; e += kBlock) {
            const int rr = e / kGemmTile, cc = e - rr * kGemmTile;
            const int64_t row = r0 + rr;
            const bool ok = row < rend;
            Ta[rr][cc] = (ok && ca + cc < R) ? load_f64<FT>(A + row * R + ca + cc) : 0.0;
            Tb[rr][cc] = (ok && cb + cc < R) ? load_f64<FT>(A + row * R + cb + cc) : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int rr = 0; rr < kBigGramRows; ++rr) {
            double a[kGemmSub], b[kGemmSub];
#pragma unroll
            for (int x = 0; x < kGemmSub; ++x) a[x] = Ta[rr][ta * kGemmSub + x];
#pragma unroll
            for (int y = 0; y < kGemmSub; ++y) b[y] = Tb[rr][tb * kGemmSub + y];
#pragma unroll
            for (int x = 0; x < kGemmSub; ++x)
#pragma unroll
                for (int y = 0; y < kGemmSub; ++y) acc[x][y] += a[x] * b[y];
        }
        __syncthreads();
    }
    double *out = gpart + (int64_t)blockIdx.x * R * R;
#pragma unroll
    for (int x = 0; x < kGemmSub; ++x)
#pragma unroll
        for (int y = 0; y < kGemmSub; ++y) {
            const int a = ca + ta * kGemmSub + x, b = cb + tb * kGemmSub + y;
            if (a < R && b < R) {
                out[a * R + b] = acc[x][y];
                if (bi != bj) out[b * R + a] = acc[x][y];
            }
        }
}

// ------------------------------------------------------------------------------------------
// Fit / model values / GCP forward: one pass over the stored entries in storage order.
// Lane groups of G lanes evaluate one entry: each lane forms lambda_j prod_m A^(m)(l_m, j) for
// its column, the group sums over columns.
// ------------------------------------------------------------------------------------------
enum { KIND_FIT = 0, KIND_VALUES = 1, KIND_GCP = 2 };


// One entry of the model pass: x = its value, t = this lane's share of the model value,
// sum_{j in lane} lambda_j prod_m A^(m)(l_m, j) (zero on lanes past column R, which still gather
// the row's first columns so that the loads carry no lane-divergent branch).
template <int D, int RW, int RQ, int CPL, class FT, class VT, class CT>
__device__ __forceinline__ void model_entry(const int4 *q, const FactorSet<FT> &A, uint32_t rowbytes,
                                            uint32_t colbytes, bool colok, const CT *lam, CT &t,
                                            VT &x) {
    int wv[RW];
    lds_record<RQ>(q, wv);
    x = rec_value<VT, RW>(wv);
    CT f[D][CPL];
#pragma unroll
    for (int m = 0; m < D; ++m) {
        const uint32_t off = (uint32_t)wv[m] * rowbytes + colbytes;
        load_cols<FT, CPL, CT>(reinterpret_cast<const FT *>(reinterpret_cast<const char *>(A.p[m]) + off),
                               f[m]);
    }
    CT sum = 0;
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        CT p = lam[c];
#pragma unroll
        for (int m = 0; m < D; ++m) p *= f[m][c];
        sum += p;
    }
    t = colok ? sum : (CT)0;
}

template <int D, int G, int CPL, class FT, class VT, class CT, int KIND>
__global__ __launch_bounds__(kBlock) void k_model(const int4 *__restrict__ rec, int64_t P, int R,
                                                  FactorSet<FT> A, const double *__restrict__ lambda,
                                                  const CT *__restrict__ w, void *__restrict__ mout,
                                                  double *__restrict__ part, int chunk, int loss) {
    constexpr int RW = RecShape<D, VT>::RW, RQ = RecShape<D, VT>::RQ;
    constexpr int U = UnrollFor<KERNEL_MODEL, G, CPL, FT>::value;
    constexpr int GS = staged_group_stride(G, RQ);
    __shared__ int4 s_rec[kBlock / kWave][(kWave / G) * GS];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane / G, gl = lane % G;
    const int col0 = gl * CPL;
    const bool colok = col0 < R;
    const uint32_t rowbytes = (uint32_t)R * sizeof(FT);
    // lanes past column R read the row's first columns and contribute zero, so the gathers
    // need no lane-divergent branch
    const uint32_t colbytes = colok ? (uint32_t)col0 * sizeof(FT) : 0u;
    CT lam[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c)
        lam[c] = (lambda != nullptr && colok) ? (CT)lambda[col0 + c] : (CT)1;
    double s0acc = 0.0, s1acc = 0.0;
    const int64_t nchunks = ceil_div(P, chunk);
    for (int64_t ch = (int64_t)blockIdx.x * (kBlock / kWave) + wave; ch < nchunks;
         ch += (int64_t)gridDim.x * (kBlock / kWave)) {
        const int64_t c0 = ch * chunk;
        const int len = (int)((c0 + chunk < P) ? chunk : P - c0);
        for (int b = 0; b < len; b += kWave) {
            if (b + lane < len) {
                const int4 *r = rec + (c0 + b + lane) * RQ;
                // streamed once: non-temporal, as in the permuted MTTKRP (fit 1.83 ms instead
                // of 1.89 on 1e8 entries at R = 32)
                s_rec[wave][g * GS + gl * RQ] = load_stream(r);
                if constexpr (RQ == 2) s_rec[wave][g * GS + gl * RQ + 1] = load_stream(r + 1);
            }
            wave_sync();
            int cnt = len - b - g * G;
            cnt = cnt < G ? cnt : G;
            for (int u0 = 0; u0 < cnt; u0 += U) {
                CT t[U];
                VT x[U];
                if (u0 + U <= cnt) {  // whole unroll: straight-line code, all gathers in flight
#pragma unroll
                    for (int u = 0; u < U; ++u)
                        model_entry<D, RW, RQ, CPL, FT, VT, CT>(&s_rec[wave][g * GS + (u0 + u) * RQ], A,
                                                                rowbytes, colbytes, colok, lam, t[u], x[u]);
                } else {
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        t[u] = 0;
                        x[u] = 0;
                        if (u0 + u < cnt)
                            model_entry<D, RW, RQ, CPL, FT, VT, CT>(&s_rec[wave][g * GS + (u0 + u) * RQ], A,
                                                                    rowbytes, colbytes, colok, lam, t[u],
                                                                    x[u]);
                    }
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    CT m = t[u];
#pragma unroll
                    for (int o = G / 2; o > 0; o >>= 1) m += __shfl_xor(m, o, G);
                    if (u0 + u < cnt && gl == 0) {
                        const int64_t i = c0 + b + g * G + u0 + u;
                        if constexpr (KIND == KIND_FIT) {
                            const double xv = (double)x[u];
                            s0acc += xv * xv;
                            s1acc += xv * (double)m;
                        } else if constexpr (KIND == KIND_VALUES) {
                            static_cast<CT *>(mout)[i] = m;
                        } else {
                            static_cast<CT *>(mout)[i] = m;
                            const double wi = (w != nullptr) ? (double)w[i] : 1.0;
                            s0acc += wi * gcp_loss_term(loss, (double)x[u], (double)m);
                        }
                    }
                }
            }
            wave_sync();
        }
    }
    if constexpr (KIND != KIND_VALUES) {
        const double a0 = block_sum_f64(s0acc);
        const double a1 = block_sum_f64(s1acc);
        if (tid == 0) {
            part[2 * blockIdx.x] = a0;
            part[2 * blockIdx.x + 1] = a1;
        }
    }
}

// fit = 1 - sqrt(max(0, xx - 2 xm + mm)) / sqrt(xx),  mm = lambda^T (Hadamard of all G) lambda
__global__ __launch_bounds__(kBlock) void k_fit_final(const double *__restrict__ part, int nblk,
                                                      const double *__restrict__ lambda,
                                                      const double *__restrict__ grams, int d,
                                                      int R, double *__restrict__ out) {
    double xx = 0.0, xm = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kBlock) {
        xx += part[2 * b];
        xm += part[2 * b + 1];
    }
    double mm = 0.0;
    for (int ab = threadIdx.x; ab < R * R; ab += kBlock) {
        const int a = ab / R, b = ab - a * R;
        double g = 1.0;
        for (int m = 0; m < d; ++m) g *= grams[(int64_t)m * R * R + ab];
        const double la = lambda ? lambda[a] : 1.0, lb = lambda ? lambda[b] : 1.0;
        mm += la * g * lb;
    }
    xx = block_sum_f64(xx);
    xm = block_sum_f64(xm);
    mm = block_sum_f64(mm);
    if (threadIdx.x == 0) {
        double r2 = xx - 2.0 * xm + mm;
        if (r2 < 0.0) r2 = 0.0;
        out[0] = 1.0 - sqrt(r2) / sqrt(xx);
        out[1] = xx;
        out[2] = xm;
        out[3] = mm;
    }
}

// ||X||^2 = sum of the squared stored values (FP64): block b's share at part[2b], the slot of
// the pair layout k_fit_final reads.
template <int RW, class VT>
__global__ __launch_bounds__(kBlock) void k_values_sumsq(const int4 *__restrict__ rec, int64_t P,
                                                         double *__restrict__ part) {
    double s = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < P; i += stride) {
        int w[RW];
#pragma unroll
        for (int k = 0; k < RW; ++k) w[k] = reinterpret_cast<const int *>(rec)[i * RW + k];
        const double x = (double)rec_value<VT, RW>(w);
        s += x * x;
    }
    s = block_sum_f64(s);
    if (threadIdx.x == 0) part[2 * blockIdx.x] = s;
}

// <X, M> from the mode-n MTTKRP V (computed from the other, normalised factors with unit
// weights): sum over r, j of lambda_j A^(n)(r, j) V(r, j), FP64.  Block b's share goes to
// part[2b + 1]; with have_xx block 0 also stores xx at part[0] and the others 0 at part[2b].
template <class FT, class AT>
__global__ __launch_bounds__(kBlock) void k_inner_av(const FT *__restrict__ A,
                                                     const AT *__restrict__ V,
                                                     const double *__restrict__ lambda,
                                                     int64_t len, int R, int have_xx, double xx,
                                                     double *__restrict__ part) {
    double s = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < len; i += stride)
        s += lambda[i % R] * load_f64(A + i) * (double)V[i];
    s = block_sum_f64(s);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x + 1] = s;
        if (have_xx) part[2 * blockIdx.x] = (blockIdx.x == 0) ? xx : 0.0;
    }
}

__global__ __launch_bounds__(kBlock) void k_loss_final(const double *__restrict__ part, int nblk,
                                                       double *__restrict__ loss) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kBlock) s += part[2 * b];
    s = block_sum_f64(s);
    if (threadIdx.x == 0) *loss = s;
}

// ------------------------------------------------------------------------------------------
// host side
// ------------------------------------------------------------------------------------------

// lane layout of the model-value pass: 8 lanes per entry with up to 8 columns each (wide
// loads, a 3-step group reduction), else one column per lane
static void model_layout(int R, int *G, int *CPL) {
    // four lanes per entry at R = 16 and 32 (4 x 4, 4 x 8 columns; fewer butterfly steps per entry:
    // fit at R = 32 on the 1e8-entry power-law tensor 1.73 ms against 2.39 ms with 8 x 4),
    // else the fewest columns per lane that cover R with 8 lanes
    if (R == 16 || R == 32) {
        *G = 4;
        *CPL = R / 4;
        return;
    }
    const int opts[] = {1, 2, 4, 8};
    for (int c : opts)
        if (R % c == 0 && R / c <= 8) {
            *G = 8;
            *CPL = c;
            return;
        }
    if (R <= 64) {
        int g = 16;
        while (g < R) g <<= 1;
        *G = g;
        *CPL = 1;
        return;
    }
    // above 64 columns: 32 or 64 lanes with several columns each (CPL must divide R)
    const int wide[][2] = {{32, 4}, {64, 2}, {32, 8}, {64, 4}};
    for (const auto &w : wide)
        if (R % w[1] == 0 && w[0] * w[1] >= R) {
            *G = w[0];
            *CPL = w[1];
            return;
        }
    *G = 0;  // no compiled layout: the caller reports SPT_EUNSUPPORTED
    *CPL = 0;
}

constexpr int kModelChunk = 2048;  // entries per wavefront chunk of the model pass

// workgroups of the model pass over P entries (each writes one pair of partial sums)
static int model_blocks(int64_t P) {
    int64_t nblk = ceil_div(ceil_div(P, kModelChunk), kBlock / kWave);
    if (nblk > kModelMaxBlocks) nblk = kModelMaxBlocks;
    return (int)(nblk < 1 ? 1 : nblk);
}

template <int D, class FT, class VT, class CT, int KIND>
static int launch_model_d(const spt_tensor *X, int R, const FactorSet<FT> &A,
                          const double *lambda, const CT *w, void *mout, double *part,
                          int *nblk_out, hipStream_t s, int loss) {
    const int chunk = kModelChunk;
    const int64_t nblk = model_blocks(X->P);
    *nblk_out = (int)nblk;
    int G = 8, CPL = 1;
    model_layout(R, &G, &CPL);
#define SPT_MODEL_CFG(GG, CC)                                                                  \
    case GG * 16 + CC:                                                                         \
        hipLaunchKernelGGL((k_model<D, GG, CC, FT, VT, CT, KIND>), dim3((unsigned)nblk),        \
                           dim3(kBlock), 0, s, X->rec, X->P, R, A, lambda, w, mout, part, chunk,  \
                           loss);                                                              \
        break;
    switch (G * 16 + CPL) {
        SPT_MODEL_CFG(4, 4)
        SPT_MODEL_CFG(4, 8)
        SPT_MODEL_CFG(8, 1)
        SPT_MODEL_CFG(8, 2)
        SPT_MODEL_CFG(8, 4)
        SPT_MODEL_CFG(8, 8)
        SPT_MODEL_CFG(16, 1)
        SPT_MODEL_CFG(32, 1)
        SPT_MODEL_CFG(64, 1)
        SPT_MODEL_CFG(32, 4)
        SPT_MODEL_CFG(32, 8)
        SPT_MODEL_CFG(64, 2)
        SPT_MODEL_CFG(64, 4)
        default: return SPT_EUNSUPPORTED;
    }
#undef SPT_MODEL_CFG
    return hipGetLastError() == hipSuccess ? SPT_OK : SPT_EHIP;
}

template <class FT, class VT, class CT, int KIND>
int launch_model(const spt_tensor *X, int R, const void *const *factors, const double *lambda,
                 const CT *w, void *mout, double *part, int *nblk, hipStream_t s, int loss = 0) {
    FactorSet<FT> A{};
    for (int m = 0; m < X->d; ++m) A.p[m] = static_cast<const FT *>(factors[m]);
    switch (X->d) {
        case 2: return launch_model_d<2, FT, VT, CT, KIND>(X, R, A, lambda, w, mout, part, nblk, s, loss);
        case 3: return launch_model_d<3, FT, VT, CT, KIND>(X, R, A, lambda, w, mout, part, nblk, s, loss);
        case 4: return launch_model_d<4, FT, VT, CT, KIND>(X, R, A, lambda, w, mout, part, nblk, s, loss);
        case 5: return launch_model_d<5, FT, VT, CT, KIND>(X, R, A, lambda, w, mout, part, nblk, s, loss);
        default: return SPT_EUNSUPPORTED;
    }
}

static int64_t max_dim(const spt_tensor *X) {
    int64_t m = 1;
    for (int i = 0; i < X->d; ++i) m = X->dims[i] > m ? X->dims[i] : m;
    return m;
}

// partial Grams per call: up to four workgroups per CU, each covering many 64-row tiles; the
// partials are then summed per entry by one wavefront in a fixed order
constexpr int kGramBlocks = 1024;
static int gram_blocks(int64_t I) {
    int64_t b = ceil_div(I, kGramRows);
    if (b > kGramBlocks) b = kGramBlocks;
    return (int)(b < 1 ? 1 : b);
}

template <class FT, bool NORM>
static int launch_gram(const FT *Ain, const double *Y, const double *lambda, FT *Aout, int64_t I,
                       int R, double *gpart, double *G, hipStream_t s) {
    const int nb = gram_blocks(I);
    if (R <= 16)
        hipLaunchKernelGGL((k_gram_partial<FT, NORM, 1>), dim3(nb), dim3(kBlock), 0, s, Ain, Y,
                           lambda, Aout, I, R, gpart);
    else if (R <= 32)
        hipLaunchKernelGGL((k_gram_partial<FT, NORM, 2>), dim3(nb), dim3(kBlock), 0, s, Ain, Y,
                           lambda, Aout, I, R, gpart);
    else
        hipLaunchKernelGGL((k_gram_partial<FT, NORM, 4>), dim3(nb), dim3(kBlock), 0, s, Ain, Y,
                           lambda, Aout, I, R, gpart);
    hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)ceil_div(R * R, kBlock / kWave)), dim3(kBlock), 0,
                       s, gpart, nb, R * R, G);
    return hipGetLastError() == hipSuccess ? SPT_OK : SPT_EHIP;
}

template <class FT>
static int launch_gram_big(const FT *A, const double *Y, const double *lambda, FT *Aout,
                           int64_t I, int R, double *gpart, double *G, hipStream_t s) {
    if (Y != nullptr) {  // normalise and store first, then the Gram of the stored values
        const int64_t len = I * (int64_t)R;
        int64_t nb = ceil_div(len, kBlock);
        if (nb > 65536) nb = 65536;
        hipLaunchKernelGGL((k_normalize_store<FT>), dim3((unsigned)nb), dim3(kBlock), 0, s, Y,
                           lambda, len, R, Aout);
        A = Aout;
    }
    const int nbk = (R + kGemmTile - 1) / kGemmTile;
    const int parts = (int)std::min<int64_t>(gram_parts(R),
                                             std::max<int64_t>(1, ceil_div(I, kBigGramRows)));
    hipLaunchKernelGGL((k_gram_big_partial<FT>),
                       dim3((unsigned)parts, (unsigned)(nbk * (nbk + 1) / 2)), dim3(kBlock), 0, s,
                       A, I, R, gpart);
    hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)ceil_div(R * R, kBlock / kWave)), dim3(kBlock), 0,
                       s, gpart, parts, R * R, G);
    return hipGetLastError() == hipSuccess ? SPT_OK : SPT_EHIP;
}

static int gram_any(int fdtype, const void *Ain, const double *Y, const double *lambda,
                    void *Aout, int64_t I, int R, double *gpart, double *G, bool norm,
                    hipStream_t s) {
    if (R > kCpSmallR) {
        switch (fdtype) {
            case SPT_F64:
                return launch_gram_big<double>((const double *)Ain, norm ? Y : nullptr, lambda,
                                               (double *)Aout, I, R, gpart, G, s);
            case SPT_F32:
                return launch_gram_big<float>((const float *)Ain, norm ? Y : nullptr, lambda,
                                              (float *)Aout, I, R, gpart, G, s);
            case SPT_BF16:
                return launch_gram_big<uint16_t>((const uint16_t *)Ain, norm ? Y : nullptr, lambda,
                                                 (uint16_t *)Aout, I, R, gpart, G, s);
            default: return SPT_EINVAL;
        }
    }
    switch (fdtype) {
        case SPT_F64:
            return norm ? launch_gram<double, true>(nullptr, Y, lambda, (double *)Aout, I, R, gpart, G, s)
                        : launch_gram<double, false>((const double *)Ain, nullptr, nullptr, nullptr, I, R, gpart, G, s);
        case SPT_F32:
            return norm ? launch_gram<float, true>(nullptr, Y, lambda, (float *)Aout, I, R, gpart, G, s)
                        : launch_gram<float, false>((const float *)Ain, nullptr, nullptr, nullptr, I, R, gpart, G, s);
        case SPT_BF16:
            return norm ? launch_gram<uint16_t, true>(nullptr, Y, lambda, (uint16_t *)Aout, I, R, gpart, G, s)
                        : launch_gram<uint16_t, false>((const uint16_t *)Ain, nullptr, nullptr, nullptr, I, R, gpart, G, s);
        default: return SPT_EINVAL;
    }
}

template <class VT, bool VEC>
static void launch_solve_v(const VT *V, int64_t I, int R, const double *L, double *Y, hipStream_t s) {
    int64_t nb = ceil_div(I, (int64_t)kBlock * (R <= 32 ? 2 : 1));  // every row in one pass
    if (nb < 1) nb = 1;
    if (R <= 16)
        hipLaunchKernelGGL((k_solve_rows<16, 2, VEC, VT>), dim3((unsigned)nb), dim3(kBlock), 0, s, V, I, R, L, Y);
    else if (R <= 32)
        hipLaunchKernelGGL((k_solve_rows<32, 2, VEC, VT>), dim3((unsigned)nb), dim3(kBlock), 0, s, V, I, R, L, Y);
    else
        hipLaunchKernelGGL((k_solve_rows<64, 1, VEC, VT>), dim3((unsigned)nb), dim3(kBlock), 0, s, V, I, R, L, Y);
}

template <class VT>
static int launch_solve(const VT *V, int64_t I, int R, const double *L, double *Y, hipStream_t s) {
    if (R % 4 == 0)
        launch_solve_v<VT, true>(V, I, R, L, Y, s);
    else
        launch_solve_v<VT, false>(V, I, R, L, Y, s);
    return hipGetLastError() == hipSuccess ? SPT_OK : SPT_EHIP;
}

// Fit from the stored entries: the model pass writes one (sum x^2, sum x m) pair per workgroup
// into part, k_fit_final reduces them with ||M||^2 into out[0..3], which is copied to the host.
static int fit_from_entries(const spt_tensor *X, int R, const void *const *factors, int fdtype,
                            const double *lambda, const double *grams, double *part, double *out,
                            double *fit, double *parts, hipStream_t s) {
    if ((fdtype == SPT_F64) != (X->vdtype == SPT_F64)) return SPT_EUNSUPPORTED;
    int nblk = 0, rc;
    switch (fdtype) {
        case SPT_F64:
            rc = launch_model<double, double, double, KIND_FIT>(X, R, factors, lambda, nullptr, nullptr, part, &nblk, s);
            break;
        case SPT_F32:
            rc = launch_model<float, float, double, KIND_FIT>(X, R, factors, lambda, nullptr, nullptr, part, &nblk, s);
            break;
        case SPT_BF16:
            rc = launch_model<uint16_t, float, double, KIND_FIT>(X, R, factors, lambda, nullptr, nullptr, part, &nblk, s);
            break;
        default: return SPT_EINVAL;
    }
    if (rc) return rc;
    hipLaunchKernelGGL(k_fit_final, dim3(1), dim3(kBlock), 0, s, part, nblk, lambda, grams, X->d,
                       R, out);
    SPT_LAUNCH_CHECK();
    double h[4];
    SPT_HIP(hipMemcpyAsync(h, out, sizeof h, hipMemcpyDeviceToHost, s));
    SPT_HIP(hipStreamSynchronize(s));
    *fit = h[0];
    if (parts) {
        parts[0] = h[1];
        parts[1] = h[2];
        parts[2] = h[3];
    }
    return spt_tensor_status(X, s);
}

// Scratch of spt_cp_fit_noalloc, for callers that cannot allocate device memory: the model
// pass's partial pairs (at most kModelMaxBlocks of them) and the four result words.  One copy
// per GPU, held until the process ends; every call on a GPU uses it, so calls that overlap on
// one GPU race.  Host code never passes the symbol itself to a kernel or a copy: it uses the
// device address that hipGetSymbolAddress returns for the current device.
constexpr size_t kFitScratchDoubles = 2 * (size_t)kModelMaxBlocks + 4;
static __device__ __align__(256) double scratch[kFitScratchDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[kMaxDevices];

// Address of this GPU's scratch, looked up once per device with that device current.
static int fit_scratch_ptr(double **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return SPT_EHIP;
    if (dev < 0 || dev >= kMaxDevices) return SPT_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr)
            return SPT_EHIP;
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[dev];
    return SPT_OK;
}

}  // namespace spt

using namespace spt;

extern "C" {

size_t spt_cp_workspace_bytes(const spt_tensor *X, int R) {
    if (X == nullptr || R < 1 || R > kCpMaxR) return 0;
    return cp_layout(max_dim(X), R).total;
}

int spt_cp_gram(int64_t I, int R, const void *A, int fdtype, double *G, void *ws,
                size_t ws_bytes, void *stream) {
    if (I < 1 || R < 1 || R > kCpMaxR || A == nullptr || G == nullptr || ws == nullptr)
        return SPT_EINVAL;
    if (ws_bytes < (size_t)gram_parts(R) * R * R * 8 || ((uintptr_t)ws & 255u))
        return SPT_EWORKSPACE;
    return gram_any(fdtype, A, nullptr, nullptr, nullptr, I, R, static_cast<double *>(ws), G,
                    false, static_cast<hipStream_t>(stream));
}

int spt_cp_als_mode(spt_tensor *X, int mode, int R, void *const *factors, int fdtype,
                    double *lambda, double *grams, void *ws, size_t ws_bytes,
                    const spt_tune *tune, void *stream) {
    if (X == nullptr || mode < 0 || mode >= X->d || R < 1 || lambda == nullptr ||
        grams == nullptr || factors == nullptr)
        return SPT_EINVAL;
    if (R > kCpMaxR) return SPT_EUNSUPPORTED;
    for (int m = 0; m < X->d; ++m)
        if (factors[m] == nullptr) return SPT_EINVAL;
    const CpWs L = cp_layout(max_dim(X), R);
    if (ws == nullptr || ((uintptr_t)ws & 255u) || ws_bytes < L.total) return SPT_EWORKSPACE;
    uint8_t *w = static_cast<uint8_t *>(ws);
    void *V = w + L.V;
    double *Y = reinterpret_cast<double *>(w + L.Y);
    double *Lf = reinterpret_cast<double *>(w + L.L);
    double *gpart = reinterpret_cast<double *>(w + L.gpart);
    double *GY = reinterpret_cast<double *>(w + L.cpart);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t I = X->dims[mode];

    int rc = check_mttkrp_args(X, mode, R, (const void *const *)factors, fdtype, V);
    if (rc) return rc;
    spt_tune t;
    rc = resolve_tune(X, mode, R, fdtype, tune, &t);
    if (rc) return rc;
    if (t.algo == SPT_ALGO_PERMUTED && !X->permuted[mode]) return SPT_ESTATE;
    if (t.algo == SPT_ALGO_PERMUTED_COPY && X->srec[mode] == nullptr) return SPT_ESTATE;
    // V = MTTKRP with the other (normalised) factors and unit weights
    rc = launch_mttkrp(X, mode, R, (const void *const *)factors, fdtype, nullptr, nullptr, V, t, s);
    if (rc) return rc;
    if (R > kCpSmallR) {
        // Gamma, L and Gamma^-1 in one workgroup; the row solves as one GEMM V Gamma^-1
        double *Wf = reinterpret_cast<double *>(w + L.Lx);
        double *Xi = reinterpret_cast<double *>(w + L.Xinv);
        double *Gi = reinterpret_cast<double *>(w + L.Ginv);
        const int Rp = (R + kCholB - 1) / kCholB * kCholB;
        hipLaunchKernelGGL(k_chol_inverse_big, dim3(1), dim3(kBlock), 0, s, grams, X->d, mode, R,
                           Rp, Wf, Xi, X->status);
        const unsigned nt = (unsigned)ceil_div(R, kXtxTile);
        hipLaunchKernelGGL(k_xtx, dim3(nt, nt), dim3(kBlock), 0, s, Xi, Rp, R, Gi);
        const dim3 g((unsigned)ceil_div(I, (int64_t)kGemmTile), (unsigned)ceil_div(R, kGemmTile));
        if (fdtype == SPT_F64)
            hipLaunchKernelGGL((k_solve_gemm<double>), g, dim3(kBlock), 0, s,
                               static_cast<const double *>(V), I, R, Gi, Y);
        else
            hipLaunchKernelGGL((k_solve_gemm<float>), g, dim3(kBlock), 0, s,
                               static_cast<const float *>(V), I, R, Gi, Y);
        SPT_LAUNCH_CHECK();
    } else {
        if (R <= 16)
            hipLaunchKernelGGL(k_hadamard_chol<16>, dim3(1), dim3(kBlock), 0, s, grams, X->d, mode,
                               R, Lf, X->status);
        else if (R <= 32)
            hipLaunchKernelGGL(k_hadamard_chol<32>, dim3(1), dim3(kBlock), 0, s, grams, X->d, mode,
                               R, Lf, X->status);
        else
            hipLaunchKernelGGL(k_hadamard_chol<64>, dim3(1), dim3(kBlock), 0, s, grams, X->d, mode,
                               R, Lf, X->status);
        SPT_LAUNCH_CHECK();
        rc = (fdtype == SPT_F64) ? launch_solve<double>((const double *)V, I, R, Lf, Y, s)
                                 : launch_solve<float>((const float *)V, I, R, Lf, Y, s);
        if (rc) return rc;
    }
    // column 2-norms of the FP64 solution
    {
        int64_t nb = ceil_div(I, (int64_t)kGramRows);
        if (nb > kMaxPartBlocks) nb = kMaxPartBlocks;
        hipLaunchKernelGGL(k_colsq_partial, dim3((unsigned)nb), dim3(kBlock), 0, s, Y, I, R, gpart);
        hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)ceil_div(R, kBlock / kWave)), dim3(kBlock), 0, s,
                           gpart, (int)nb, R, GY);
        hipLaunchKernelGGL(k_norms, dim3(1), dim3(64), 0, s, GY, R, lambda);
        SPT_LAUNCH_CHECK();
    }
    return gram_any(fdtype, nullptr, Y, lambda, factors[mode], I, R, gpart,
                    grams + (size_t)mode * R * R, true, s);
}

int spt_cp_als_sweep(spt_tensor *X, int R, void *const *factors, int fdtype, double *lambda,
                     double *grams, void *ws, size_t ws_bytes, const spt_tune *tune,
                     void *stream) {
    if (X == nullptr) return SPT_EINVAL;
    for (int n = 0; n < X->d; ++n) {
        int rc = spt_cp_als_mode(X, n, R, factors, fdtype, lambda, grams, ws, ws_bytes, tune, stream);
        if (rc) return rc;
    }
    return SPT_OK;
}

int spt_cp_solution(const spt_tensor *X, int R, const void *ws, size_t ws_bytes,
                    const double **Y) {
    if (X == nullptr || R < 1 || R > kCpMaxR || Y == nullptr) return SPT_EINVAL;
    const CpWs L = cp_layout(max_dim(X), R);
    if (ws == nullptr || ((uintptr_t)ws & 255u) || ws_bytes < L.total) return SPT_EWORKSPACE;
    *Y = reinterpret_cast<const double *>(static_cast<const uint8_t *>(ws) + L.Y);
    return SPT_OK;
}

int spt_cp_fit(const spt_tensor *X, int R, const void *const *factors, int fdtype,
               const double *lambda, const double *grams, void *ws, size_t ws_bytes,
               double *fit, double *parts, void *stream) {
    if (X == nullptr || R < 1 || R > kCpMaxR || grams == nullptr || fit == nullptr)
        return SPT_EINVAL;
    int rc = check_factors(X, -1, factors);
    if (rc == SPT_OK) rc = check_factor_extent(X, -1, R, fdtype);
    if (rc) return rc;
    const CpWs L = cp_layout(max_dim(X), R);
    if (ws == nullptr || ((uintptr_t)ws & 255u) || ws_bytes < L.total) return SPT_EWORKSPACE;
    uint8_t *w = static_cast<uint8_t *>(ws);
    return fit_from_entries(X, R, factors, fdtype, lambda, grams,
                            reinterpret_cast<double *>(w + L.gpart),
                            reinterpret_cast<double *>(w + L.misc), fit, parts,
                            static_cast<hipStream_t>(stream));
}

int spt_cp_fit_noalloc(const spt_tensor *X, int R, const void *const *factors, int fdtype,
                       const double *lambda, const double *grams, double *fit, double *parts,
                       void *stream) {
    if (X == nullptr || R < 1 || R > kCpMaxR || grams == nullptr || fit == nullptr)
        return SPT_EINVAL;
    int rc = check_factors(X, -1, factors);
    if (rc == SPT_OK) rc = check_factor_extent(X, -1, R, fdtype);
    if (rc) return rc;
    // partial pairs of the model pass, then the four result words
    if ((size_t)2 * model_blocks(X->P) + 4 > kFitScratchDoubles) return SPT_EWORKSPACE;
    double *sp = nullptr;
    rc = fit_scratch_ptr(&sp);
    if (rc) return rc;
    return fit_from_entries(X, R, factors, fdtype, lambda, grams, sp,
                            sp + kFitScratchDoubles - 4, fit, parts,
                            static_cast<hipStream_t>(stream));
}

int spt_cp_fit_after_mode(spt_tensor *X, int mode, int R, const void *const *factors,
                          int fdtype, const double *lambda, const double *grams, void *ws,
                          size_t ws_bytes, double *fit, double *parts, void *stream) {
    if (X == nullptr || mode < 0 || mode >= X->d || R < 1 || R > kCpMaxR || lambda == nullptr ||
        grams == nullptr || fit == nullptr)
        return SPT_EINVAL;
    if (fdtype != SPT_F64 && fdtype != SPT_F32 && fdtype != SPT_BF16) return SPT_EINVAL;
    int rc = check_factors(X, -1, factors);
    if (rc == SPT_OK) rc = check_factor_extent(X, -1, R, fdtype);
    if (rc) return rc;
    const CpWs L = cp_layout(max_dim(X), R);
    if (ws == nullptr || ((uintptr_t)ws & 255u) || ws_bytes < L.total) return SPT_EWORKSPACE;
    uint8_t *w = static_cast<uint8_t *>(ws);
    const void *V = w + L.V;  // left there by the mode update
    double *part = reinterpret_cast<double *>(w + L.gpart);
    double *out = reinterpret_cast<double *>(w + L.misc);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t len = X->dims[mode] * (int64_t)R;
    const int nblk = (int)std::min<int64_t>(kMaxPartBlocks, std::max<int64_t>(1, ceil_div(len, kBlock)));
    const bool have_xx = X->xx_valid != 0;
    if (!have_xx) {
        if (X->rec_words == 4) {
            if (X->vdtype == SPT_F64)
                hipLaunchKernelGGL((k_values_sumsq<4, double>), dim3(nblk), dim3(kBlock), 0, s, X->rec, X->P, part);
            else
                hipLaunchKernelGGL((k_values_sumsq<4, float>), dim3(nblk), dim3(kBlock), 0, s, X->rec, X->P, part);
        } else {
            if (X->vdtype == SPT_F64)
                hipLaunchKernelGGL((k_values_sumsq<8, double>), dim3(nblk), dim3(kBlock), 0, s, X->rec, X->P, part);
            else
                hipLaunchKernelGGL((k_values_sumsq<8, float>), dim3(nblk), dim3(kBlock), 0, s, X->rec, X->P, part);
        }
        SPT_LAUNCH_CHECK();
    }
    const double xx = have_xx ? X->xx : 0.0;
    if (fdtype == SPT_F64)
        hipLaunchKernelGGL((k_inner_av<double, double>), dim3(nblk), dim3(kBlock), 0, s,
                           static_cast<const double *>(factors[mode]), static_cast<const double *>(V),
                           lambda, len, R, (int)have_xx, xx, part);
    else if (fdtype == SPT_F32)
        hipLaunchKernelGGL((k_inner_av<float, float>), dim3(nblk), dim3(kBlock), 0, s,
                           static_cast<const float *>(factors[mode]), static_cast<const float *>(V),
                           lambda, len, R, (int)have_xx, xx, part);
    else
        hipLaunchKernelGGL((k_inner_av<uint16_t, float>), dim3(nblk), dim3(kBlock), 0, s,
                           static_cast<const uint16_t *>(factors[mode]), static_cast<const float *>(V),
                           lambda, len, R, (int)have_xx, xx, part);
    SPT_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_fit_final, dim3(1), dim3(kBlock), 0, s, part, nblk, lambda, grams, X->d,
                       R, out);
    SPT_LAUNCH_CHECK();
    double h[4];
    SPT_HIP(hipMemcpyAsync(h, out, sizeof h, hipMemcpyDeviceToHost, s));
    SPT_HIP(hipStreamSynchronize(s));
    if (!have_xx) {
        X->xx = h[1];
        X->xx_valid = 1;
    }
    *fit = h[0];
    if (parts) {
        parts[0] = h[1];
        parts[1] = h[2];
        parts[2] = h[3];
    }
    return spt_tensor_status(X, stream);
}

int spt_model_values(const spt_tensor *X, int R, const void *const *factors, int fdtype,
                     const double *lambda, void *out, void *stream) {
    if (X == nullptr || R < 1 || R > kCpMaxR || out == nullptr) return SPT_EINVAL;
    int rc = check_factors(X, -1, factors);
    if (rc == SPT_OK) rc = check_factor_extent(X, -1, R, fdtype);
    if (rc) return rc;
    if ((fdtype == SPT_F64) != (X->vdtype == SPT_F64)) return SPT_EUNSUPPORTED;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int nblk = 0;
    switch (fdtype) {
        case SPT_F64:
            return launch_model<double, double, double, KIND_VALUES>(X, R, factors, lambda, nullptr, out, nullptr, &nblk, s);
        case SPT_F32:
            return launch_model<float, float, float, KIND_VALUES>(X, R, factors, lambda, nullptr, out, nullptr, &nblk, s);
        case SPT_BF16:
            return launch_model<uint16_t, float, float, KIND_VALUES>(X, R, factors, lambda, nullptr, out, nullptr, &nblk, s);
        default: return SPT_EINVAL;
    }
}

}  // extern "C"

// GCP forward reuses k_model; defined here so the loss reduction kernel stays local.
namespace spt {
int gcp_forward_impl(const spt_tensor *X, int R, const void *const *factors, int fdtype,
                     int loss_kind, const void *w, void *m, double *loss, double *part,
                     hipStream_t s) {
    int nblk = 0;
    int rc;
    if (fdtype == SPT_F64)
        rc = launch_model<double, double, double, KIND_GCP>(X, R, factors, nullptr,
                                                           static_cast<const double *>(w), m, part,
                                                           &nblk, s, loss_kind);
    else
        rc = launch_model<float, float, float, KIND_GCP>(X, R, factors, nullptr,
                                                        static_cast<const float *>(w), m, part,
                                                        &nblk, s, loss_kind);
    if (rc) return rc;
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(kBlock), 0, s, part, nblk, loss);
    return hipGetLastError() == hipSuccess ? SPT_OK : SPT_EHIP;
}
}  // namespace spt
