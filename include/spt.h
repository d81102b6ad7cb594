/*
 * spt.h -- C ABI of libspt, the MI355X (gfx950) sparse COO tensor library: per-mode
 * permutations and mode-sorted record copies, MTTKRP (atomic, permuted and privatised
 * traversals, batched launches), CP-ALS update and fit, generalized-CP losses with their
 * gradients, and the sampling and Adam steps of stochastic generalized CP.
 *
 * Method: Phipps & Kolda, "Software for Sparse Tensor Decomposition on Emerging Computing
 * Architectures", arXiv 1809.09175.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Pointers documented "device" point to GPU memory owned by the caller (for example torch
 *    tensors).  The library never allocates device memory: every buffer it needs is carved from
 *    a caller-provided workspace whose size the matching *_workspace_bytes() call returns.  The
 *    caller keeps every borrowed buffer alive (and unmodified where stated) while a handle that
 *    refers to it exists.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Calls only enqueue
 *    work on it and return at once, unless documented as synchronising.
 *  - Indices are 0-based.  Subscripts and permutations are int32 (so at most 2^31-1 entries and
 *    mode lengths); sizes and entry counts are int64 in the interface.
 *  - Dense matrices (factors A^(m), MTTKRP results V, Gram matrices) are row-major.  Kernels
 *    address factor rows with 32-bit byte offsets, so every call that reads factor rows of the
 *    tensor's entries (MTTKRP, CP-ALS, fit, model values, generalized CP, batches) returns
 *    SPT_EUNSUPPORTED when one of the matrices it gathers from is 4 GiB or larger.
 *  - Every call returns an spt_status.  Argument errors are found on the host before anything
 *    is enqueued and leave all outputs untouched.  Errors found on the GPU (a subscript out of
 *    range, a singular Gram matrix) set a status word inside the tensor's workspace; they are
 *    returned by the next synchronising call on that tensor (spt_tensor_validate, spt_cp_fit,
 *    spt_tensor_status).
 *  - Thread safety: a tensor handle may be used concurrently by several host threads for
 *    read-only calls (MTTKRP, fit, model values) once its permutations exist; calls that write
 *    into the workspace or the handle (create, permute, sort_copy, deterministic MTTKRP, cp_*
 *    steps, and the first spt_cp_fit_after_mode, which stores ||X||^2 in the handle) must not
 *    overlap on one tensor.
 */
#ifndef SPT_H
#define SPT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum spt_status {
    SPT_OK = 0,
    SPT_EINVAL = -1,       /* invalid argument (null pointer, bad mode, bad size, ...) */
    SPT_ERANGE = -2,       /* a subscript is outside [0, I_m) */
    SPT_EHIP = -3,         /* a HIP runtime call failed */
    SPT_ESINGULAR = -4,    /* a Gram matrix product was not positive definite */
    SPT_EWORKSPACE = -5,   /* workspace too small or misaligned (256-byte alignment) */
    SPT_EUNSUPPORTED = -6, /* valid but unsupported combination (order, rank, dtype) */
    SPT_ESTATE = -7        /* call out of order (e.g. permuted MTTKRP before permute) */
} spt_status;

typedef enum spt_dtype { SPT_F64 = 0, SPT_F32 = 1, SPT_BF16 = 2 } spt_dtype;

typedef enum spt_algo {
    SPT_ALGO_AUTO = 0,     /* library choice (tuned table, else the default heuristic) */
    SPT_ALGO_ATOMIC = 1,   /* storage-order traversal in tiles of up to 1024 entries, each tile
                              sorted by output row in LDS and summed per row, then one atomic
                              per distinct row and column of the tile */
    SPT_ALGO_PERMUTED = 2, /* mode-sorted traversal through the permutation (records gathered),
                              wave segmented reduction */
    SPT_ALGO_PERMUTED_COPY = 3, /* the same traversal reading a mode-sorted copy of the records
                                   (spt_tensor_sort_copy): records stream instead of being
                                   gathered; with a storage-ordered copy the rows are summed in
                                   the order SPT_ALGO_PERMUTED sums them */
    SPT_ALGO_PRIVATIZED = 4 /* storage-order traversal into a per-workgroup LDS copy of the whole
                               output, flushed once per workgroup: the hybrid of atomics and
                               private copies that Sec. 8 proposes for short modes; only when
                               I_n x lanes x columns x 4 (8 for FP64) bytes plus 4-8 KiB of
                               staging fit 64 KiB of LDS (SPT_EUNSUPPORTED otherwise) */
} spt_algo;

/* Launch parameters of one MTTKRP.  Zero fields take the default.  A lane group of
 * lanes_per_nnz lanes evaluates one entry, each lane holding cols_per_lane consecutive rank
 * columns; the product must cover R and cols_per_lane must divide R.  Compiled (lanes, cols)
 * pairs: (4,4) (4,8) (8,1) (8,2) (8,4) (8,8) (16,1) (16,2) (16,4) (16,8) (32,1) (32,2) (32,4)
 * (32,8) (64,1) (64,2) (64,4).  nnz_per_wave: entries one wavefront walks (a multiple of 64); the atomic
 * algorithm gives each workgroup 4 x nnz_per_wave entries rounded up to whole sorted tiles. */
typedef struct spt_tune {
    int32_t algo;
    int32_t lanes_per_nnz;
    int32_t cols_per_lane;
    int32_t nnz_per_wave;
    int32_t flags;   /* SPT_TUNE_DETERMINISTIC: see below */
    int32_t lds_kib; /* reserved: 0 .. 64 accepted (SPT_EINVAL otherwise), no effect on any
                        algorithm */
} spt_tune;

/* spt_tune.flags.  SPT_TUNE_DETERMINISTIC (permuted algorithms only): the rows a wave chunk
 * shares with its neighbours are not added atomically but parked in two scratch slots per chunk
 * and summed by a second pass in sorted order, so the MTTKRP issues no atomic instruction and V
 * is bit-reproducible from run to run (Sec. 6 notes that the segmented reduction can make
 * atomics unnecessary).  The slots live in the tensor's radix-sort scratch: do not overlap with
 * spt_tensor_permute or another deterministic MTTKRP on the same tensor. */
#define SPT_TUNE_DETERMINISTIC 1

typedef struct spt_tensor spt_tensor;

const char *spt_status_string(int status);
int spt_version(void); /* major*10000 + minor*100 + patch */

/* ---------------------------------------------------------------------------------------------
 * Sparse tensor in coordinate (COO) format, Sec. 3: P entries, each a value x_i and subscripts
 * (l_i1 .. l_id).  Duplicate subscripts are allowed and mean the sum of the entries (MTTKRP is
 * linear in the entries); CP fit and the GCP loss assume distinct subscripts.
 * ------------------------------------------------------------------------------------------- */

/* Workspace needed by a tensor of order d (2..5) with the given mode lengths, entry count and
 * value dtype (SPT_F64 or SPT_F32).  It holds the packed entry records, one permutation and one
 * sorted key array per mode (Sec. 6: d extra arrays of P ordinals), the radix-sort scratch and
 * the status word.  Returns 0 for invalid arguments. */
size_t spt_tensor_workspace_bytes(int d, const int64_t *dims, int64_t nnz, int vals_dtype);

/* Builds a tensor handle.
 *   out        receives the host-side handle (free with spt_tensor_destroy)
 *   dims       host, d mode lengths I_m (1 .. 2^31-1)
 *   subs       device, nnz x d int32 row-major subscripts; read only during this call's work
 *   vals       device, nnz values of vals_dtype (SPT_F64 or SPT_F32); read only likewise
 *   ws         device workspace of at least spt_tensor_workspace_bytes(), 256-byte aligned;
 *              owned by the caller, must outlive the handle
 * Enqueues the packing of (subs, vals) into the workspace; subscripts outside [0, I_m) are
 * reported by spt_tensor_validate.  nnz may be 0. */
int spt_tensor_create(spt_tensor **out, int d, const int64_t *dims, int64_t nnz,
                      const int32_t *subs, const void *vals, int vals_dtype, void *ws,
                      size_t ws_bytes, void *stream);

/* The same in pieces, so that moving the entries to the device can overlap with packing them
 * (Sec. 8 proposes building the permutation while the tensor is read): spt_tensor_create_begin
 * takes the arguments of spt_tensor_create without subs and vals; then spt_tensor_append packs
 * entries [first, first + count) from device arrays holding just those entries (subs: count x d
 * int32, vals: count values), in order: first must equal the entries appended so far and be a
 * multiple of 8192, count a multiple of 8192 unless the chunk ends the tensor (SPT_EINVAL /
 * SPT_ESTATE otherwise).  Each append also counts the first radix digit (bits 0-7) of every
 * mode's subscripts over its entries, which spt_tensor_permute then uses instead of a histogram
 * pass of its own.  Until every entry is appended, spt_tensor_permute and the calls that read
 * the entries return SPT_ESTATE.  spt_tensor_create is begin plus one append of all entries.
 * Both enqueue only; the chunk's arrays are read by the enqueued work. */
int spt_tensor_create_begin(spt_tensor **out, int d, const int64_t *dims, int64_t nnz,
                            int vals_dtype, void *ws, size_t ws_bytes, void *stream);
int spt_tensor_append(spt_tensor *X, int64_t first, int64_t count, const int32_t *subs,
                      const void *vals, void *stream);

/* Synchronises `stream`; returns SPT_ERANGE (and the first offending entry index in *bad_entry
 * when not NULL) if a subscript was out of range, else the pending device status. */
int spt_tensor_validate(const spt_tensor *X, int64_t *bad_entry, void *stream);

/* Synchronises `stream` and returns the device status word (then clears it). */
int spt_tensor_status(const spt_tensor *X, void *stream);

/* Builds the mode-`mode` permutation (mode = -1: every mode), Sec. 6: perm_n is the stable
 * order of the entries by their mode-n subscript (ties in storage order) and skey_n the sorted
 * subscripts.  Hand-written LSD radix sort, 8-bit digits.  Enqueued only. */
int spt_tensor_permute(spt_tensor *X, int mode, void *stream);

/* Device pointers of the mode's permutation and sorted keys (valid after spt_tensor_permute's
 * work completes, until the handle is destroyed); SPT_ESTATE if the mode is not permuted. */
int spt_tensor_perm(const spt_tensor *X, int mode, const int32_t **perm, const int32_t **skey);

/* Mode-sorted copies of the packed records (a memory-for-bandwidth trade the paper avoided for
 * 12-16 GB GPUs, Sec. 6), so the permuted MTTKRP streams records instead of gathering them.
 * The copy of mode n holds the records grouped by their mode-n subscript in increasing order;
 * within a group, order selects:
 *   SPT_COPY_STORAGE_ORDER   storage order: position q holds record perm_n[q];
 *   SPT_COPY_BY_SECOND_MODE  increasing subscript of a second mode m, then storage order, where
 *                            m is the other mode with the most rows (lowest index among equals):
 *                            consecutive entries of a row then share or neighbour their mode-m
 *                            factor rows, which raises the cache hit rate of the gathers.  Needs
 *                            mode m permuted as well; the copy carries its own order array
 *                            (4 bytes per entry), used where replacement values are read.
 * Needs spt_tensor_permute(mode) first (SPT_ESTATE otherwise); mode = -1 copies every mode back
 * to back.  ws: device buffer of at least spt_tensor_sorted_copy_bytes(X, mode, order) bytes,
 * 256-byte aligned (any pointer, NULL included, when that size is 0: an empty tensor),
 * caller-owned, kept alive until the copy is dropped or the handle destroyed;
 * the second-mode order also uses the tensor's sort scratch.  A later spt_tensor_permute of a
 * mode drops its copy.  With a copy present, SPT_ALGO_AUTO selects SPT_ALGO_PERMUTED_COPY.
 * SPT_EINVAL for an unknown order (and 0 bytes from the size query). */
typedef enum spt_copy_order {
    SPT_COPY_STORAGE_ORDER = 0,
    SPT_COPY_BY_SECOND_MODE = 1
} spt_copy_order;
size_t spt_tensor_sorted_copy_bytes(const spt_tensor *X, int mode, int order);
int spt_tensor_sort_copy(spt_tensor *X, int mode, int order, void *ws, size_t ws_bytes,
                         void *stream);
int spt_tensor_drop_sorted_copy(spt_tensor *X, int mode);

int spt_tensor_info(const spt_tensor *X, int *d, int64_t *dims, int64_t *nnz, int *vals_dtype);
int spt_tensor_destroy(spt_tensor *X);

/* ---------------------------------------------------------------------------------------------
 * MTTKRP, eq. (mttkrp) of Sec. 3:
 *   V(k, j) = lambda_j * sum_{i : l_in = k} x_i * prod_{m != n} A^(m)(l_im, j)
 *   X        tensor handle (SPT_ALGO_PERMUTED needs spt_tensor_permute(mode) first)
 *   mode     n, 0 <= n < d
 *   R        rank: any value 1 .. 64; even values up to 128; multiples of 4 up to 256
 *            (SPT_EUNSUPPORTED otherwise)
 *   factors  host array of d device pointers, A^(m) is I_m x R row-major of fdtype; the entry
 *            for m == n is not read and may be NULL; each matrix must be smaller than 4 GiB
 *            (SPT_EUNSUPPORTED otherwise: rows are addressed with 32-bit byte offsets)
 *   fdtype   SPT_F64 (needs F64 tensor values), SPT_F32 or SPT_BF16 (need F32 values)
 *   lambda   device R doubles, or NULL for all ones
 *   vals     device, NULL to use the tensor's values, else P replacement values in the tensor's
 *            value dtype, in storage order (the GCP backward passes its derivative tensor here)
 *   V        device I_n x R output, double for SPT_F64 factors, float otherwise; overwritten
 *            (zeroed, then accumulated)
 *   tune     NULL or launch parameters (see spt_tune)
 * Products and accumulation run in FP64 for SPT_F64 and in FP32 otherwise (BF16 factors are
 * widened to FP32 on load). */
int spt_mttkrp(const spt_tensor *X, int mode, int R, const void *const *factors, int fdtype,
               const double *lambda, const void *vals, void *V, const spt_tune *tune,
               void *stream);

/* The launch parameters spt_mttkrp uses for (X, mode, R, fdtype, algo) when tune is NULL. */
int spt_mttkrp_default_tune(const spt_tensor *X, int mode, int R, int fdtype, int algo,
                            spt_tune *out);

/* The GPU vector size and factor block size the paper's register-array MTTKRP uses for rank R
 * (Tab. sizes); the autotuner's candidate list contains the layout it maps to (lanes per entry =
 * vector size, columns per lane = block size / vector size) whenever that layout is compiled. */
int spt_paper_block_sizes(int R, int *vector_size, int *fbs);

/* Autotuner: times the library's default configuration (spt_mttkrp_default_tune, with the
 * chunk its launch uses) and every compiled launch configuration for (X, mode, R, fdtype) on
 * `stream` (algorithm x lanes per entry x columns per lane x entries per wave; layouts that
 * cover R with at most twice R lanes-columns), and returns the fastest in *best and its time
 * per launch in *best_ms (host).  Each candidate runs once untimed, then `reps` launches timed
 * one by one; its time is their median.  V is device scratch of the MTTKRP output size
 * (overwritten).  reps: 0 = 7, at most 64.  Synchronises `stream`. */
enum {
    SPT_TUNE_BATCH_CONFIGS = 1, /* only configurations the batched kernel supports */
    SPT_TUNE_NO_ATOMIC = 2,
    SPT_TUNE_NO_PERMUTED = 4
};
int spt_mttkrp_autotune(const spt_tensor *X, int mode, int R, const void *const *factors,
                        int fdtype, void *V, int flags, int reps, spt_tune *best, float *best_ms,
                        void *stream);

/* ---------------------------------------------------------------------------------------------
 * Batched MTTKRP (beyond the paper): many (tensor, mode) products of uneven sizes in one
 * persistent kernel.  Workgroups take units of 4 wave chunks from a global counter; each
 * product keeps its own algorithm and lane layout.  The output zeroing and the kernel are
 * captured once into a HIP graph that spt_batch_launch replays.
 *   items i = 0..nitems-1: tensors[i] (3-way, F32 values), modes[i], ranks[i],
 *            factors[i] (host array of d device factor pointers), outputs[i] (device
 *            I_n x R floats), tunes[i] (from spt_mttkrp_autotune with SPT_TUNE_BATCH_CONFIGS,
 *            or zeros for the default; must map to a configuration the batched kernel
 *            supports, see spt_batch_supported_tune, else SPT_EUNSUPPORTED)
 *   fdtype   SPT_F32 or SPT_BF16 for every item
 *   ws       device workspace of spt_batch_workspace_bytes(nitems) (item table and counter);
 *            caller-owned, must outlive the batch, as must every tensor, factor and output
 * spt_batch_create synchronises `stream` once (item table upload) and captures on a stream of
 * its own; spt_batch_launch enqueues one graph replay on `stream`.  Replays of one batch must
 * not overlap (they share the work counter). */
typedef struct spt_batch spt_batch;
size_t spt_batch_workspace_bytes(int nitems);
int spt_batch_supported_tune(int d, int fdtype, int algo, int lanes_per_nnz, int cols_per_lane);
int spt_batch_create(spt_batch **out, int nitems, const spt_tensor *const *tensors,
                     const int *modes, const int *ranks, const void *const *const *factors,
                     int fdtype, void *const *outputs, const spt_tune *tunes, void *ws,
                     size_t ws_bytes, void *stream);
int spt_batch_launch(spt_batch *B, void *stream);
int spt_batch_info(const spt_batch *B, int64_t *units, int *smem_bytes);
int spt_batch_destroy(spt_batch *B);

/* ---------------------------------------------------------------------------------------------
 * CP-ALS (Sec. 3 uses alternating least squares and defers the algorithm to Kolda & Bader).
 * One mode update n:
 *   V = MTTKRP(X, A, n, lambda = ones)
 *   Gamma = Hadamard product of G_m, m != n            (FP64, R x R)
 *   Gamma = L L^T (Cholesky; a pivot <= R * eps * max diag(Gamma) sets SPT_ESINGULAR)
 *   row k of A^(n) solves A^(n)(k,:) Gamma = V(k,:)     (FP64 forward/back substitution)
 *   lambda_j = ||A^(n)(:,j)||_2, columns with lambda_j > 0 divided by lambda_j (in FP64), then
 *   stored in fdtype: FP32 by the ordinary FP64 -> FP32 conversion, BF16 by rounding the FP64
 *   value to nearest even in a single step (no FP32 intermediate, so no double rounding; the
 *   rule of spt_f64_to_bf16)
 *   G_n = A^(n)^T A^(n) from the stored values         (FP64)
 * factors: host array of d device pointers (I_m x R, fdtype), A^(n) overwritten.
 * lambda: device R doubles (overwritten).  grams: device d x R x R doubles, G_m for every mode
 * on entry (spt_cp_gram), G_n overwritten.  ws: device workspace of spt_cp_workspace_bytes().
 * R: 1 .. 64 any value (Cholesky in one wavefront, row-parallel substitution); 65 .. 256 as for
 * spt_mttkrp (even up to 128, multiples of 4 above), where the Cholesky factor of Gamma and its
 * inverse are formed by one workgroup and the row solves run as one FP64 product V Gamma^-1
 * (the two agree to about cond(Gamma) times the FP64 rounding unit); SPT_EUNSUPPORTED
 * otherwise.  spt_cp_gram needs ws of R x R x 8 x 1024 bytes up to R = 64, at most R x R x 8 x 768
 * above (spt_cp_workspace_bytes always suffices). */
size_t spt_cp_workspace_bytes(const spt_tensor *X, int R);

int spt_cp_gram(int64_t I, int R, const void *A, int fdtype, double *G, void *ws,
                size_t ws_bytes, void *stream);

int spt_cp_als_mode(spt_tensor *X, int mode, int R, void *const *factors, int fdtype,
                    double *lambda, double *grams, void *ws, size_t ws_bytes,
                    const spt_tune *tune, void *stream);

/* spt_cp_als_mode for n = 0 .. d-1. */
int spt_cp_als_sweep(spt_tensor *X, int R, void *const *factors, int fdtype, double *lambda,
                     double *grams, void *ws, size_t ws_bytes, const spt_tune *tune,
                     void *stream);

/* Device pointer (*Y) to the FP64 solution that the last spt_cp_als_mode(X, n, ...) left in ws:
 * I_n x R row-major doubles, the rows solving A(k,:) Gamma = V(k,:) before normalisation, so the
 * stored factor is Y(k, j) / lambda_j (Y(k, j) where lambda_j = 0) rounded to fdtype.  For
 * checking the precision of the stored factor; valid until the next call that uses ws.  No
 * device work.  SPT_EWORKSPACE if ws is shorter than spt_cp_workspace_bytes(X, R). */
int spt_cp_solution(const spt_tensor *X, int R, const void *ws, size_t ws_bytes,
                    const double **Y);

/* Fit of the model M = sum_j lambda_j a_j^(1) o ... o a_j^(d) (eq. (CP)) from the stored
 * entries: fit = 1 - sqrt(max(0, ||X||^2 - 2<X,M> + ||M||^2)) / ||X|| with ||X||^2 and <X,M>
 * summed over the entries in FP64 and ||M||^2 = lambda^T (Hadamard of all G_m) lambda.
 * Synchronises `stream`; writes the fit to *fit (host) and, if parts != NULL, the three terms
 * to parts[0..2] (host).  Returns a pending device status (e.g. SPT_ESINGULAR) if any. */
int spt_cp_fit(const spt_tensor *X, int R, const void *const *factors, int fdtype,
               const double *lambda, const double *grams, void *ws, size_t ws_bytes,
               double *fit, double *parts, void *stream);

/* spt_cp_fit for callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid allocation): no workspace argument and no allocation.
 * The per-workgroup partial sums go to a fixed scratch array inside the library (about 32 KiB,
 * one copy per GPU, held until the process ends), looked up for the current device at the
 * first call on it: `stream` must belong to the current device.  Every call on one GPU shares
 * that array, so calls that overlap on one GPU (other threads, other streams) race; nothing in
 * it needs clearing between calls.  Same arguments (without ws), result and synchronisation as
 * spt_cp_fit; SPT_EWORKSPACE if the tensor needs more partial sums than the array holds (not
 * reachable at present: the pass uses at most 2048 workgroups). */
int spt_cp_fit_noalloc(const spt_tensor *X, int R, const void *const *factors, int fdtype,
                       const double *lambda, const double *grams, double *fit, double *parts,
                       void *stream);

/* The same fit right after spt_cp_als_mode(X, mode, ...) (typically the last mode of a sweep),
 * without a pass over the entries.  The V that update left in ws is X_(n) times the
 * Khatri-Rao product of the other, normalised factors, so <X,M> = sum_j lambda_j sum_r
 * A^(n)(r, j) V(r, j): an I_n x R inner product of the updated factor with the MTTKRP (FP64
 * sums; V itself carries the MTTKRP's accumulation precision, FP32 for FP32 and BF16 factors).
 * ||M||^2 as in spt_cp_fit; ||X||^2 is summed from the stored values at the handle's first call
 * and kept in the handle (the values never change).  Valid only while ws still holds that
 * update's V and no factor, lambda or Gram changed since: no other call may use ws in between
 * (spt_cp_fit may: it leaves V alone).  Arguments, synchronisation and outputs as spt_cp_fit;
 * factors, lambda and grams are the state the mode update left. */
int spt_cp_fit_after_mode(spt_tensor *X, int mode, int R, const void *const *factors,
                          int fdtype, const double *lambda, const double *grams, void *ws,
                          size_t ws_bytes, double *fit, double *parts, void *stream);

/* Model value of every stored entry, m_i = sum_j lambda_j prod_m A^(m)(l_im, j) (eq. (CP)).
 * out: device P values, double for SPT_F64 factors, float otherwise.  lambda may be NULL. */
int spt_model_values(const spt_tensor *X, int R, const void *const *factors, int fdtype,
                     const double *lambda, void *out, void *stream);

/* ---------------------------------------------------------------------------------------------
 * Generalized CP with the Poisson log-link loss (Sec. 8 names generalized CP, for count and
 * binary data, as the next workload): f(x, m) = exp(m) - x m summed over the stored entries
 * (nonzeros and sampled zeros), model m_i = sum_j prod_m A^(m)(l_im, j) (no weights lambda).
 * fdtype SPT_F64 (tensor values F64; w, m, y double) or SPT_F32 (values F32; w, m, y float).
 *   forward:  m (device P values, out), loss (device 1 double, out) = sum_i w_i f(x_i, m_i),
 *             summed in FP64; ws: device scratch of at least 32 KiB, 256-byte aligned
 *   backward: y_i = g w_i (exp(m_i) - x_i) into y (device P values, scratch), g = *gscale
 *             (device double, the upstream gradient; NULL = 1), then grads[n] = MTTKRP(Y, A, n)
 *             for every mode (host array of d device I_n x R buffers, double for F64 else float)
 * w: device P weights or NULL (all ones).  R as for spt_cp_als_mode (at most 256). */
int spt_gcp_poisson_forward(const spt_tensor *X, int R, const void *const *factors, int fdtype,
                            const void *w, void *m, double *loss, void *ws, size_t ws_bytes,
                            void *stream);
int spt_gcp_poisson_backward(const spt_tensor *X, int R, const void *const *factors, int fdtype,
                             const void *w, const void *m, const double *gscale, void *y,
                             void *const *grads, const spt_tune *tune, void *stream);

/* The same with a choice of elementwise loss (generalized CP for count, binary and real data):
 *   SPT_GCP_POISSON   f = exp(m) - x m,            df/dm = exp(m) - x
 *   SPT_GCP_BERNOULLI f = log(1 + exp(m)) - x m,   df/dm = 1 / (1 + exp(-m)) - x
 *   SPT_GCP_GAUSSIAN  f = (x - m)^2,               df/dm = 2 (m - x)
 *   SPT_GCP_GAMMA     f = x / m' + log m',         df/dm = 1 / m' - x / m'^2,  m' = m + 1e-10
 *                     (positive data, the model is the mean: factors must be nonnegative)
 * Arguments as for the Poisson calls; loss_kind outside these values gives SPT_EINVAL. */
enum { SPT_GCP_POISSON = 0, SPT_GCP_BERNOULLI = 1, SPT_GCP_GAUSSIAN = 2, SPT_GCP_GAMMA = 3 };
int spt_gcp_forward(const spt_tensor *X, int R, const void *const *factors, int fdtype,
                    int loss_kind, const void *w, void *m, double *loss, void *ws,
                    size_t ws_bytes, void *stream);
int spt_gcp_backward(const spt_tensor *X, int R, const void *const *factors, int fdtype,
                     int loss_kind, const void *w, const void *m, const double *gscale, void *y,
                     void *const *grads, const spt_tune *tune, void *stream);

/* Fused forward and backward of the generalized-CP loss with unit weights: for every mode n one
 * pass over the entries in mode-n order (the sorted record copy if built, else the records
 * gathered through the permutation) computes each entry's model value m_i, the derivative
 * y_i = df/dm(x_i, m_i) and y_i's contribution to grads[n] = MTTKRP(Y, A, n), with the permuted
 * MTTKRP's segmented reduction; the derivative tensor is never stored.  The pass over mode 0
 * also sums the loss into *loss (device double; FP64 partials per wave chunk, summed in a fixed
 * order).  grads are scaled by *gscale (device double) when gscale != NULL.  Same losses, types
 * and factor layout as spt_gcp_forward; every mode must be permuted (else SPT_ESTATE); tune (or
 * NULL) supplies lanes/cols/chunk, its algorithm is ignored; SPT_TUNE_DETERMINISTIC is not
 * supported.  Uses the tensor's internal reduction scratch: calls on one tensor must not
 * overlap.  Asynchronous on `stream`. */
int spt_gcp_fused(const spt_tensor *X, int R, const void *const *factors, int fdtype,
                  int loss_kind, double *loss, void *const *grads, const double *gscale,
                  const spt_tune *tune, void *stream);

/* Stochastic generalized CP (GCP-SGD).  spt_gcp_sample draws iteration `iter`'s stratified
 * sample on the device with the Philox4x64-10 counter-based generator (Salmon et al., SC'11),
 * key (seed, 0):
 *   entries 0..s_nz-1:  stored entry p = floor(r0 * P / 2^64), r = philox((k, iter, 0, 0)); its
 *                       subscripts and value; weight P / s_nz
 *   entries s_nz..s_nz+s_z-1 (k = 0..s_z-1): a uniform cell, subscript m = floor(r_m I_m / 2^64),
 *                       r = philox((k, iter, 1, 0)) (modes 4.. from (k, iter, 1, 1)); value 0;
 *                       weight (prod I_m - P) / s_z.  Cells holding a stored entry are not
 *                       rejected (a bias of order P / prod I_m).
 * subs: device (s_nz + s_z) x d int32; vals, w: device s_nz + s_z values of dtype (SPT_F32 or
 * SPT_F64).  The sample feeds spt_tensor_create and spt_gcp_forward / spt_gcp_backward with w.
 * spt_adam_step: one Adam step (Kingma & Ba) on n values of dtype: m = b1 m + (1-b1) g,
 * v = b2 v + (1-b2) g^2, x = max(lower, x - lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps)),
 * t >= 1; x, m, v updated in place (device), g read.  Both asynchronous on `stream`. */
int spt_gcp_sample(const spt_tensor *X, uint64_t seed, int64_t iter, int64_t s_nz, int64_t s_z,
                   int32_t *subs, void *vals, void *w, int dtype, void *stream);
int spt_adam_step(void *x, const void *g, void *m, void *v, int64_t n, int dtype, double lr,
                  double beta1, double beta2, double eps, int64_t t, double lower, void *stream);

/* dst[i] = src[i] * (*g) for n values (dtype SPT_F32 or SPT_F64; src may equal dst; g a device
 * double): the upstream-gradient scaling of a loss computed before its gradient was requested. */
int spt_scale_values(const void *src, void *dst, int64_t n, int dtype, const double *g,
                     void *stream);

/* ---------------------------------------------------------------------------------------------
 * Precision and measurement helpers
 * ------------------------------------------------------------------------------------------- */

/* FP32 -> BF16 bit patterns, round to nearest, ties to even; NaN stays a quiet NaN with its
 * sign.  in: device n floats; out: device n uint16. */
int spt_f32_to_bf16(const float *in, uint16_t *out, int64_t n, void *stream);

/* FP64 -> BF16 bit patterns, round to nearest, ties to even, in a single rounding (the value is
 * narrowed to FP32 with round-to-odd first, which keeps the final rounding correct); NaN maps to
 * the quiet NaN 0x7fc0 with its sign; magnitudes at or past the midpoint between the largest
 * finite BF16 and 2^128 give infinity.  The CP-ALS BF16 factor store uses the same rounding.
 * in: device n doubles; out: device n uint16. */
int spt_f64_to_bf16(const double *in, uint16_t *out, int64_t n, void *stream);

/* STREAM-style triad a[i] = b[i] + s * c[i] over n floats (device), for measuring achievable
 * HBM bandwidth. */
int spt_stream_triad(float *a, const float *b, const float *c, float s, int64_t n, void *stream);

#ifdef __cplusplus
}
#endif
#endif
