/*
 * oracle.h -- declarations of the plain FP64 CPU reference for sparse COO MTTKRP and CP-ALS.
 *
 * TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT PATH.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load or call it.  It shares no code, header, table
 * or helper with the HIP library; the two meet only through the seeded input arrays.
 *
 * Conventions (all functions):
 *   - d-way COO tensor with P entries: subs is P x d row-major int32 (entry i's coordinates are
 *     subs[i*d .. i*d+d-1], 0-based), vals is P FP64 values.  Duplicate coordinates are allowed
 *     and mean "sum of the entries" (MTTKRP is linear in the entries).
 *   - factor matrices A[m] are I_m x R row-major FP64.
 *   - every function returns 0 on success or a negative code (see ORACLE_E*).
 */
#ifndef SPT_ORACLE_H
#define SPT_ORACLE_H

#include <stdint.h>

#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)
#define ORACLE_ERANGE (-2)
#define ORACLE_ESINGULAR (-4)

#ifdef __cplusplus
extern "C" {
#endif

/* Mode-n MTTKRP, eq. (mttkrp) of Section 3.  lambda may be NULL (all ones).  V is I_n x R. */
int oracle_mttkrp(int d, const int64_t *dims, int64_t P, const int32_t *subs, const double *vals,
                  int n, int R, const double *const *A, const double *lambda, double *V);

/* Stable permutation of the entries by their mode-n coordinate (Section 6): perm[q] is the
 * storage position of the q-th entry in increasing mode-n order, ties kept in storage order;
 * skey[q] = subs[perm[q]*d + n].  Either output may be NULL. */
int oracle_perm(int d, const int64_t *dims, int64_t P, const int32_t *subs, int n,
                int32_t *perm, int32_t *skey);

/* Model value of each stored entry, eq. (CP): m_i = sum_j lambda_j prod_m A[m](l_im, j). */
int oracle_model_values(int d, const int64_t *dims, int64_t P, const int32_t *subs, int R,
                        const double *const *A, const double *lambda, double *m);

/* Gram matrix G = A^T A of an I x R factor (R x R, row-major). */
int oracle_gram(int64_t I, int R, const double *A, double *G);

/* One CP-ALS mode update (textbook ALS, Kolda & Bader, cited in Section 3):
 *   V = MTTKRP(X, A, n, lambda = ones); Gamma = Hadamard product of G[m], m != n;
 *   Cholesky Gamma = L L^T (a pivot <= R * eps * max diag(Gamma) is singular -> ORACLE_ESINGULAR);
 *   each row: A[n](k,:) solves A[n](k,:) Gamma = V(k,:) by forward then back substitution;
 *   lambda_j = ||A[n](:,j)||_2; columns with lambda_j > 0 are divided by lambda_j;
 *   G[n] = A[n]^T A[n].
 * A[n], lambda and G[n] are overwritten.  G holds d R x R matrices back to back. */
int oracle_cp_als_mode(int d, const int64_t *dims, int64_t P, const int32_t *subs,
                       const double *vals, int n, int R, double *const *A, double *lambda,
                       double *G);

/* A full sweep: oracle_cp_als_mode for n = 0 .. d-1 in order. */
int oracle_cp_als_sweep(int d, const int64_t *dims, int64_t P, const int32_t *subs,
                        const double *vals, int R, double *const *A, double *lambda, double *G);

/* Fit 1 - ||X - M|| / ||X|| computed from the stored entries only:
 *   ||X||^2 = sum x_i^2, <X,M> = sum x_i m_i, ||M||^2 = lambda^T (Hadamard of all A_m^T A_m) lambda,
 *   ||X - M||^2 = max(0, ||X||^2 - 2<X,M> + ||M||^2).  Requires distinct coordinates. */
int oracle_fit(int d, const int64_t *dims, int64_t P, const int32_t *subs, const double *vals,
               int R, const double *const *A, const double *lambda, double *fit,
               double *parts /* optional out[3] = ||X||^2, <X,M>, ||M||^2 */);

/* Generalized CP with the Poisson log-link loss f(x, m) = exp(m) - x*m over the stored entries
 * (nonzeros and sampled zeros), model without weights lambda:
 *   loss = sum_i w_i f(x_i, m_i);  y_i = w_i (exp(m_i) - x_i);  grad[n] = MTTKRP(Y, A, n).
 * w may be NULL (all ones).  grads may be NULL (loss only); grads[n] is I_n x R. */
int oracle_gcp_poisson(int d, const int64_t *dims, int64_t P, const int32_t *subs,
                       const double *vals, const double *w, int R, const double *const *A,
                       double *loss, double *const *grads);

/* Generalized CP with a choice of elementwise loss f(x, m) and its derivative df/dm:
 *   loss 0, Poisson with log link:  f = exp(m) - x m,          df = exp(m) - x
 *   loss 1, Bernoulli with logit:   f = log(1 + exp(m)) - x m,  df = 1 / (1 + exp(-m)) - x
 *   loss 2, Gaussian:               f = (x - m)^2,              df = 2 (m - x)
 *   loss 3, Gamma (m > 0):          f = x / m' + log m',        df = 1 / m' - x / m'^2,
 *                                   m' = m + 1e-10 (guards m = 0; factors nonnegative)
 * loss = sum_i w_i f(x_i, m_i), grad[n] = MTTKRP(Y, A, n) with y_i = w_i df(x_i, m_i). */
int oracle_gcp(int d, const int64_t *dims, int64_t P, const int32_t *subs, const double *vals,
               const double *w, int R, const double *const *A, int loss_kind, double *loss,
               double *const *grads);

/* Philox4x64-10 counter-based generator (Salmon et al., SC'11): out = philox(ctr, key). */
void oracle_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

/* Stratified sample for stochastic generalized CP, iteration iter, key (seed, 0):
 *   entries 0..s_nz-1: stored entry p = floor(r0 * P / 2^64), r = philox((k, iter, 0, 0)),
 *                      weight P / s_nz;
 *   entries s_nz..s_nz+s_z-1 (k = 0..s_z-1): a uniform cell, subscript m = floor(r_m * I_m /
 *                      2^64) with r = philox((k, iter, 1, 0)) (modes 4.. from (k, iter, 1, 1)),
 *                      value 0, weight (prod I_m - P) / s_z.  Cells that hold a stored entry are
 *                      not rejected (a bias of order P / prod I_m).
 * out_subs: (s_nz + s_z) x d, out_vals and out_w: s_nz + s_z. */
int oracle_gcp_sample(int d, const int64_t *dims, int64_t P, const int32_t *subs,
                      const double *vals, uint64_t seed, int64_t iter, int64_t s_nz,
                      int64_t s_z, int32_t *out_subs, double *out_vals, double *out_w);

/* Adam step t >= 1 (Kingma & Ba): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * x = max(lower, x - lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps)). */
int oracle_adam(int64_t n, double *x, const double *g, double *m, double *v, double lr,
                double beta1, double beta2, double eps, int64_t t, double lower);

/* FP32 -> BF16 round to nearest, ties to even, by comparing the distances to the two
 * neighbouring BF16 values.  NaN maps to a quiet NaN with the same sign and top payload. */
uint16_t oracle_bf16_rne(uint32_t f32_bits);
int oracle_bf16_rne_array(int64_t n, const uint32_t *in, uint16_t *out);

/* FP64 -> BF16 round to nearest, ties to even, in a single rounding (no FP32 step): the value
 * is compared exactly with its two neighbouring BF16 values (8 significant bits, subnormal step
 * 2^-133); half a step or more past the largest finite BF16 gives infinity.  NaN maps to the
 * quiet NaN 0x7fc0 with the same sign.  The BF16 factor store of a CP-ALS update rounds its
 * FP64 solution this way. */
uint16_t oracle_bf16_rne_f64(double v);
int oracle_bf16_rne_f64_array(int64_t n, const double *in, uint16_t *out);

#ifdef __cplusplus
}
#endif
#endif
