/*
 * oracle.c -- plain, single-threaded FP64 CPU reference for the sparse COO MTTKRP / CP-ALS path
 * of Phipps & Kolda, "Software for Sparse Tensor Decomposition on Emerging Computing
 * Architectures" (arXiv 1809.09175).
 *
 * TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT PATH.  Only the test suite, the smoke check and
 * the benchmark's CPU-baseline leg may load or call it.  It shares no code with the HIP library.
 *
 * Every routine is the plain definition written out, with no blocking, fusion or reordering:
 *   - MTTKRP: eq. (mttkrp), Section 3.  The per-term multiply order follows the paper's
 *     description of the kernel (Section 4.1): start from x_i * lambda_j, then multiply by each
 *     other mode's factor entry in increasing mode order.
 *   - permutation: Section 6 sorts the entries by their mode-n coordinate with a stable sort;
 *     here a counting sort (stable by construction).
 *   - CP model and fit: eq. (CP), Section 3.
 *   - CP-ALS: Section 3 defers the algorithm to Kolda & Bader; this is the textbook update.
 *   - GCP Poisson loss: named as future work in Section 8 (generalized CP of Hong, Kolda and
 *     Duersch); loss exp(m) - x m, derivative exp(m) - x.
 * Parity status of every function is listed in the module's Python wrapper header.
 */
#include "oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

static int check_tensor(int d, const int64_t *dims, int64_t P, const int32_t *subs)
{
    if (d < 1 || dims == NULL || P < 0 || (P > 0 && subs == NULL)) return ORACLE_EINVAL;
    for (int m = 0; m < d; ++m)
        if (dims[m] < 1) return ORACLE_EINVAL;
    for (int64_t i = 0; i < P; ++i)
        for (int m = 0; m < d; ++m) {
            int32_t l = subs[i * d + m];
            if (l < 0 || (int64_t)l >= dims[m]) return ORACLE_ERANGE;
        }
    return ORACLE_OK;
}

int oracle_mttkrp(int d, const int64_t *dims, int64_t P, const int32_t *subs, const double *vals,
                  int n, int R, const double *const *A, const double *lambda, double *V)
{
    int rc = check_tensor(d, dims, P, subs);
    if (rc) return rc;
    if (n < 0 || n >= d || R < 1 || V == NULL || A == NULL || (P > 0 && vals == NULL))
        return ORACLE_EINVAL;
    memset(V, 0, sizeof(double) * (size_t)dims[n] * (size_t)R);
    for (int64_t i = 0; i < P; ++i) {
        const int32_t *l = subs + i * d;
        double *vrow = V + (int64_t)l[n] * R;
        for (int j = 0; j < R; ++j) {
            double t = vals[i] * (lambda ? lambda[j] : 1.0);
            for (int m = 0; m < d; ++m)
                if (m != n) t *= A[m][(int64_t)l[m] * R + j];
            vrow[j] += t;
        }
    }
    return ORACLE_OK;
}

int oracle_perm(int d, const int64_t *dims, int64_t P, const int32_t *subs, int n,
                int32_t *perm, int32_t *skey)
{
    int rc = check_tensor(d, dims, P, subs);
    if (rc) return rc;
    if (n < 0 || n >= d || P > INT32_MAX) return ORACLE_EINVAL;
    int64_t I = dims[n];
    int64_t *start = (int64_t *)calloc((size_t)I + 1, sizeof(int64_t));
    if (!start) return ORACLE_EINVAL;
    /* count entries per key, then the first output slot of each key */
    for (int64_t i = 0; i < P; ++i) start[subs[i * d + n] + 1] += 1;
    for (int64_t k = 0; k < I; ++k) start[k + 1] += start[k];
    /* place entries in storage order: equal keys keep their relative order */
    for (int64_t i = 0; i < P; ++i) {
        int32_t k = subs[i * d + n];
        int64_t q = start[k]++;
        if (perm) perm[q] = (int32_t)i;
        if (skey) skey[q] = k;
    }
    free(start);
    return ORACLE_OK;
}

int oracle_model_values(int d, const int64_t *dims, int64_t P, const int32_t *subs, int R,
                        const double *const *A, const double *lambda, double *m)
{
    int rc = check_tensor(d, dims, P, subs);
    if (rc) return rc;
    if (R < 1 || A == NULL || (P > 0 && m == NULL)) return ORACLE_EINVAL;
    for (int64_t i = 0; i < P; ++i) {
        const int32_t *l = subs + i * d;
        double s = 0.0;
        for (int j = 0; j < R; ++j) {
            double t = lambda ? lambda[j] : 1.0;
            for (int q = 0; q < d; ++q) t *= A[q][(int64_t)l[q] * R + j];
            s += t;
        }
        m[i] = s;
    }
    return ORACLE_OK;
}

int oracle_gram(int64_t I, int R, const double *A, double *G)
{
    if (I < 0 || R < 1 || (I > 0 && A == NULL) || G == NULL) return ORACLE_EINVAL;
    for (int a = 0; a < R; ++a)
        for (int b = 0; b < R; ++b) {
            double s = 0.0;
            for (int64_t k = 0; k < I; ++k) s += A[k * R + a] * A[k * R + b];
            G[a * R + b] = s;
        }
    return ORACLE_OK;
}

/* Lower Cholesky factor of the symmetric matrix S (R x R): S = L L^T.  A pivot that is not
 * larger than R * DBL_EPSILON * max_k S(k,k) makes the matrix singular for this purpose. */
static int cholesky_lower(int R, const double *S, double *L)
{
    double maxdiag = 0.0;
    for (int k = 0; k < R; ++k)
        if (S[k * R + k] > maxdiag) maxdiag = S[k * R + k];
    double tol = (double)R * DBL_EPSILON * maxdiag;
    memset(L, 0, sizeof(double) * (size_t)R * (size_t)R);
    for (int c = 0; c < R; ++c) {
        double piv = S[c * R + c];
        for (int k = 0; k < c; ++k) piv -= L[c * R + k] * L[c * R + k];
        if (!(piv > tol)) return ORACLE_ESINGULAR;
        double lcc = sqrt(piv);
        L[c * R + c] = lcc;
        for (int r = c + 1; r < R; ++r) {
            double s = S[r * R + c];
            for (int k = 0; k < c; ++k) s -= L[r * R + k] * L[c * R + k];
            L[r * R + c] = s / lcc;
        }
    }
    return ORACLE_OK;
}

int oracle_cp_als_mode(int d, const int64_t *dims, int64_t P, const int32_t *subs,
                       const double *vals, int n, int R, double *const *A, double *lambda,
                       double *G)
{
    if (n < 0 || n >= d || R < 1 || A == NULL || lambda == NULL || G == NULL)
        return ORACLE_EINVAL;
    int64_t I = dims[n];
    double *V = (double *)malloc(sizeof(double) * (size_t)I * (size_t)R);
    double *Gam = (double *)malloc(sizeof(double) * (size_t)R * (size_t)R);
    double *L = (double *)malloc(sizeof(double) * (size_t)R * (size_t)R);
    double *y = (double *)malloc(sizeof(double) * (size_t)R);
    int rc = ORACLE_EINVAL;
    if (!V || !Gam || !L || !y) goto done;

    rc = oracle_mttkrp(d, dims, P, subs, vals, n, R, (const double *const *)A, NULL, V);
    if (rc) goto done;

    for (int a = 0; a < R * R; ++a) Gam[a] = 1.0;
    for (int m = 0; m < d; ++m)
        if (m != n)
            for (int a = 0; a < R * R; ++a) Gam[a] *= G[(size_t)m * R * R + a];

    rc = cholesky_lower(R, Gam, L);
    if (rc) goto done;

    /* row k of the new factor solves a Gamma = v, i.e. Gamma a^T = v^T (Gamma symmetric):
     * L y = v (forward), then L^T a = y (backward). */
    for (int64_t k = 0; k < I; ++k) {
        const double *v = V + k * R;
        double *a = A[n] + k * R;
        for (int c = 0; c < R; ++c) {
            double s = v[c];
            for (int q = 0; q < c; ++q) s -= L[c * R + q] * y[q];
            y[c] = s / L[c * R + c];
        }
        for (int c = R - 1; c >= 0; --c) {
            double s = y[c];
            for (int q = c + 1; q < R; ++q) s -= L[q * R + c] * a[q];
            a[c] = s / L[c * R + c];
        }
    }

    for (int j = 0; j < R; ++j) {
        double s = 0.0;
        for (int64_t k = 0; k < I; ++k) s += A[n][k * R + j] * A[n][k * R + j];
        lambda[j] = sqrt(s);
    }
    for (int64_t k = 0; k < I; ++k)
        for (int j = 0; j < R; ++j)
            if (lambda[j] > 0.0) A[n][k * R + j] /= lambda[j];

    rc = oracle_gram(I, R, A[n], G + (size_t)n * R * R);
done:
    free(V);
    free(Gam);
    free(L);
    free(y);
    return rc;
}

int oracle_cp_als_sweep(int d, const int64_t *dims, int64_t P, const int32_t *subs,
                        const double *vals, int R, double *const *A, double *lambda, double *G)
{
    for (int n = 0; n < d; ++n) {
        int rc = oracle_cp_als_mode(d, dims, P, subs, vals, n, R, A, lambda, G);
        if (rc) return rc;
    }
    return ORACLE_OK;
}

int oracle_fit(int d, const int64_t *dims, int64_t P, const int32_t *subs, const double *vals,
               int R, const double *const *A, const double *lambda, double *fit, double *parts)
{
    int rc = check_tensor(d, dims, P, subs);
    if (rc) return rc;
    if (R < 1 || A == NULL || fit == NULL || (P > 0 && vals == NULL)) return ORACLE_EINVAL;
    double *m = (double *)malloc(sizeof(double) * (size_t)(P > 0 ? P : 1));
    double *Gall = (double *)malloc(sizeof(double) * (size_t)R * (size_t)R);
    double *Gm = (double *)malloc(sizeof(double) * (size_t)R * (size_t)R);
    rc = ORACLE_EINVAL;
    if (!m || !Gall || !Gm) goto done;
    rc = oracle_model_values(d, dims, P, subs, R, A, lambda, m);
    if (rc) goto done;

    double xx = 0.0, xm = 0.0, mm = 0.0;
    for (int64_t i = 0; i < P; ++i) {
        xx += vals[i] * vals[i];
        xm += vals[i] * m[i];
    }
    for (int a = 0; a < R * R; ++a) Gall[a] = 1.0;
    for (int q = 0; q < d; ++q) {
        oracle_gram(dims[q], R, A[q], Gm);
        for (int a = 0; a < R * R; ++a) Gall[a] *= Gm[a];
    }
    for (int a = 0; a < R; ++a)
        for (int b = 0; b < R; ++b) {
            double la = lambda ? lambda[a] : 1.0, lb = lambda ? lambda[b] : 1.0;
            mm += la * Gall[a * R + b] * lb;
        }
    double r2 = xx - 2.0 * xm + mm;
    if (r2 < 0.0) r2 = 0.0;
    *fit = 1.0 - sqrt(r2) / sqrt(xx);
    if (parts) {
        parts[0] = xx;
        parts[1] = xm;
        parts[2] = mm;
    }
done:
    free(m);
    free(Gall);
    free(Gm);
    return rc;
}

/* elementwise loss and derivative of the generalized CP losses (plain definitions) */
/* Gamma: the model is the mean, kept positive by the caller (nonnegative factors); the shift
 * ORACLE_GAMMA_EPS guards m = 0 */
#define ORACLE_GAMMA_EPS 1e-10

static double gcp_f(int kind, double x, double m)
{
    switch (kind) {
    case 0: return exp(m) - x * m;
    case 1: return log1p(exp(m)) - x * m;
    case 3: return x / (m + ORACLE_GAMMA_EPS) + log(m + ORACLE_GAMMA_EPS);
    default: return (x - m) * (x - m);
    }
}

static double gcp_df(int kind, double x, double m)
{
    switch (kind) {
    case 0: return exp(m) - x;
    case 1: return 1.0 / (1.0 + exp(-m)) - x;
    case 3: return 1.0 / (m + ORACLE_GAMMA_EPS) - x / ((m + ORACLE_GAMMA_EPS) * (m + ORACLE_GAMMA_EPS));
    default: return 2.0 * (m - x);
    }
}

int oracle_gcp(int d, const int64_t *dims, int64_t P, const int32_t *subs, const double *vals,
               const double *w, int R, const double *const *A, int loss_kind, double *loss,
               double *const *grads)
{
    int rc = check_tensor(d, dims, P, subs);
    if (rc) return rc;
    if (R < 1 || A == NULL || loss == NULL || (P > 0 && vals == NULL) || loss_kind < 0 ||
        loss_kind > 3)
        return ORACLE_EINVAL;
    double *m = (double *)malloc(sizeof(double) * (size_t)(P > 0 ? P : 1));
    double *y = (double *)malloc(sizeof(double) * (size_t)(P > 0 ? P : 1));
    rc = ORACLE_EINVAL;
    if (!m || !y) goto done;
    rc = oracle_model_values(d, dims, P, subs, R, A, NULL, m);
    if (rc) goto done;
    double L = 0.0;
    for (int64_t i = 0; i < P; ++i) {
        double wi = w ? w[i] : 1.0;
        L += wi * gcp_f(loss_kind, vals[i], m[i]);
        y[i] = wi * gcp_df(loss_kind, vals[i], m[i]);
    }
    *loss = L;
    if (grads)
        for (int n = 0; n < d && rc == ORACLE_OK; ++n)
            rc = oracle_mttkrp(d, dims, P, subs, y, n, R, A, NULL, grads[n]);
done:
    free(m);
    free(y);
    return rc;
}

int oracle_gcp_poisson(int d, const int64_t *dims, int64_t P, const int32_t *subs,
                       const double *vals, const double *w, int R, const double *const *A,
                       double *loss, double *const *grads)
{
    return oracle_gcp(d, dims, P, subs, vals, w, R, A, 0, loss, grads);
}

static double bits_to_float_as_double(uint32_t b)
{
    float f;
    memcpy(&f, &b, sizeof f);
    return (double)f;
}

uint16_t oracle_bf16_rne(uint32_t x)
{
    uint32_t sign = x & 0x80000000u;
    uint32_t mag = x & 0x7fffffffu;
    if (mag > 0x7f800000u) /* NaN: keep sign and top payload, force the quiet bit */
        return (uint16_t)((x >> 16) | 0x0040u);
    if (mag == 0x7f800000u) return (uint16_t)(x >> 16); /* +-inf */
    /* the BF16 magnitudes just below (truncation) and just above the input */
    uint32_t lo_bits = mag & 0xffff0000u;
    if (lo_bits == mag) return (uint16_t)((sign | mag) >> 16); /* exactly representable */
    uint32_t hi_bits = lo_bits + 0x00010000u;
    double v = bits_to_float_as_double(mag);
    double lo = bits_to_float_as_double(lo_bits);
    /* the next BF16 above the largest finite one is 2^128, which rounds to infinity */
    double hi = (hi_bits == 0x7f800000u) ? ldexp(1.0, 128) : bits_to_float_as_double(hi_bits);
    double dlo = v - lo, dhi = hi - v; /* exact in double */
    uint32_t pick;
    if (dlo < dhi) pick = lo_bits;
    else if (dhi < dlo) pick = hi_bits;
    else pick = ((lo_bits >> 16) & 1u) ? hi_bits : lo_bits; /* tie: even last bit */
    return (uint16_t)((sign | pick) >> 16);
}

int oracle_bf16_rne_array(int64_t n, const uint32_t *in, uint16_t *out)
{
    if (n < 0 || (n > 0 && (in == NULL || out == NULL))) return ORACLE_EINVAL;
    for (int64_t i = 0; i < n; ++i) out[i] = oracle_bf16_rne(in[i]);
    return ORACLE_OK;
}

uint16_t oracle_bf16_rne_f64(double v)
{
    const uint16_t sign = signbit(v) ? 0x8000u : 0u;
    if (isnan(v)) return (uint16_t)(sign | 0x7fc0u);
    const double a = fabs(v);
    if (isinf(a)) return (uint16_t)(sign | 0x7f80u);
    if (a == 0.0) return sign;
    /* a = f 2^e with f in [0.5, 1): BF16 keeps 8 significant bits, so its step in this binade
     * is 2^(e-8), but never finer than the subnormal step 2^-133 */
    int e;
    frexp(a, &e);
    const int qe = (e - 8 < -133) ? -133 : e - 8;
    const double q = ldexp(1.0, qe);
    const double k = floor(a / q); /* a / q < 256: exact */
    const double lo = k * q, hi = lo + q;
    const double dlo = a - lo, dhi = hi - a; /* exact: multiples of a's ulp below 2^46 of them */
    double pick;
    if (dlo < dhi) pick = lo;
    else if (dhi < dlo) pick = hi;
    else pick = (fmod(k, 2.0) == 0.0) ? lo : hi; /* tie: even last bit */
    if (pick >= ldexp(1.0, 128)) return (uint16_t)(sign | 0x7f80u);
    const float pf = (float)pick; /* at most 8 significant bits inside the FP32 range: exact */
    uint32_t bits;
    memcpy(&bits, &pf, sizeof bits);
    return (uint16_t)(sign | (bits >> 16));
}

int oracle_bf16_rne_f64_array(int64_t n, const double *in, uint16_t *out)
{
    if (n < 0 || (n > 0 && (in == NULL || out == NULL))) return ORACLE_EINVAL;
    for (int64_t i = 0; i < n; ++i) out[i] = oracle_bf16_rne_f64(in[i]);
    return ORACLE_OK;
}

/* ---------------------------------------------------------------------------------------------
 * Stochastic generalized CP (GCP-SGD; generalized CP is the workload Sec. 8 names next).
 * ------------------------------------------------------------------------------------------- */

/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
 * SC'11): ten rounds of two 64x64->128 multiplications on a 4-word counter under a 2-word key
 * bumped by the Weyl constants. */
static void mul_hilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo)
{
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void oracle_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t hi0, lo0, hi1, lo1;
        mul_hilo64(0xD2E7470EE14C6C93ull, c0, &hi0, &lo0);
        mul_hilo64(0xCA5A826395121157ull, c2, &hi1, &lo1);
        uint64_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B97F4A7C15ull;
        k1 += 0xBB67AE8584CAA73Bull;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* floor(r * n / 2^64): a 64-bit random word mapped onto 0..n-1 */
static int64_t scale_index(uint64_t r, int64_t n)
{
    return (int64_t)(((unsigned __int128)r * (unsigned __int128)(uint64_t)n) >> 64);
}

int oracle_gcp_sample(int d, const int64_t *dims, int64_t P, const int32_t *subs,
                      const double *vals, uint64_t seed, int64_t iter, int64_t s_nz,
                      int64_t s_z, int32_t *out_subs, double *out_vals, double *out_w)
{
    int rc = check_tensor(d, dims, P, subs);
    if (rc) return rc;
    if (s_nz < 0 || s_z < 0 || (s_nz > 0 && P == 0) || iter < 0 ||
        (s_nz + s_z > 0 && (out_subs == NULL || out_vals == NULL || out_w == NULL)))
        return ORACLE_EINVAL;
    const uint64_t key[2] = {seed, 0};
    double cells = 1.0;
    for (int m = 0; m < d; ++m) cells *= (double)dims[m];
    const double w_nz = s_nz > 0 ? (double)P / (double)s_nz : 0.0;
    const double w_z = (s_z > 0 && cells > (double)P) ? (cells - (double)P) / (double)s_z : 0.0;
    for (int64_t k = 0; k < s_nz; ++k) {
        const uint64_t ctr[4] = {(uint64_t)k, (uint64_t)iter, 0, 0};
        uint64_t r[4];
        oracle_philox4x64(ctr, key, r);
        const int64_t p = scale_index(r[0], P);
        for (int m = 0; m < d; ++m) out_subs[k * d + m] = subs[p * d + m];
        out_vals[k] = vals[p];
        out_w[k] = w_nz;
    }
    for (int64_t k = 0; k < s_z; ++k) {
        const int64_t e = s_nz + k;
        uint64_t r[8];
        const uint64_t c0[4] = {(uint64_t)k, (uint64_t)iter, 1, 0};
        oracle_philox4x64(c0, key, r);
        if (d > 4) {
            const uint64_t c1[4] = {(uint64_t)k, (uint64_t)iter, 1, 1};
            oracle_philox4x64(c1, key, r + 4);
        }
        for (int m = 0; m < d; ++m) out_subs[e * d + m] = (int32_t)scale_index(r[m], dims[m]);
        out_vals[e] = 0.0;
        out_w[e] = w_z;
    }
    return ORACLE_OK;
}

int oracle_adam(int64_t n, double *x, const double *g, double *m, double *v, double lr,
                double beta1, double beta2, double eps, int64_t t, double lower)
{
    if (n < 0 || t < 1 || (n > 0 && (x == NULL || g == NULL || m == NULL || v == NULL)))
        return ORACLE_EINVAL;
    const double c1 = 1.0 - pow(beta1, (double)t), c2 = 1.0 - pow(beta2, (double)t);
    for (int64_t i = 0; i < n; ++i) {
        m[i] = beta1 * m[i] + (1.0 - beta1) * g[i];
        v[i] = beta2 * v[i] + (1.0 - beta2) * g[i] * g[i];
        const double mh = m[i] / c1, vh = v[i] / c2;
        double xi = x[i] - lr * mh / (sqrt(vh) + eps);
        x[i] = xi < lower ? lower : xi;
    }
    return ORACLE_OK;
}
