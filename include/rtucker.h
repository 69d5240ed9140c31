/*
 * rtucker - randomized Tucker compression on AMD Instinct MI355X (gfx950).
 *
 * C ABI of librtucker.so.  It computes the Tucker approximations of
 * Minster, Saibaba and Kilmer, "Randomized Algorithms for Low-rank Tensor
 * Decompositions in the Tucker Format":
 *   rt_rhosvd            - R-HOSVD, Alg. 2 (§3.1)
 *   rt_rsthosvd          - R-STHOSVD, Alg. 3 (§3.1)
 *   rt_rsthosvd_adaptive - adaptive R-STHOSVD, Alg. 5 (§4)
 *   rt_rhosvd_adaptive   - adaptive R-HOSVD, Alg. 4 (§4)
 *   rt_sp_sthosvd        - structure-preserving STHOSVD, Alg. 6 (§5)
 *   rt_sp_sthosvd_coo    - the same on a sparse tensor in coordinate storage
 * and exposes the steps of their hot path for testing: the on-the-fly Gaussian
 * sketch Y = X_(n) Omega (Alg. 1 step 1), Q = orth(Y) (Alg. 1 step 2) and the
 * projection B = X x_n Q^T (Alg. 1 step 3).
 *
 * Conventions (all calls):
 *  - Tensors are dense, row-major (last index fastest), float32 or float64,
 *    in device memory of the context's device (rt_coo: sparse, coordinate
 *    storage).  Modes are 0-based.
 *  - The mode-n unfolding X_(n) has the mode-n fibres as columns; column c is
 *    the row-major linear index over the remaining modes in increasing order.
 *  - Omega_n[c, k] ~ N(0, 1) comes from Philox4x32-10 with key (seed lo, seed hi)
 *    and counter (c lo, c hi, k / 4, n), words mapped to (w + 1/2) 2^-32 and
 *    through two Box-Muller pairs to columns 4 (k/4) .. 4 (k/4) + 3.  It is never
 *    stored.  R-HOSVD mode n and the first R-STHOSVD step on mode n therefore
 *    see the same Omega.
 *  - Pointers are device pointers unless marked "host".  The caller keeps
 *    ownership of every input; the library never writes an input tensor.
 *  - Work is enqueued on the context's stream.  The fixed-rank decompositions
 *    (rt_rhosvd, rt_rsthosvd, rt_sp_sthosvd, rt_sp_sthosvd_coo) and rt_reconstruct are
 *    asynchronous: they return once their work is enqueued, with the ranks and
 *    the core and factor buffers of the result set; the contents of those
 *    buffers are valid once the stream reaches that point, and the scalars
 *    (norm_x, core_norm, rel_err_est, flags) are filled in by the next rt_sync
 *    on the context (NaN until then), which also returns deferred device
 *    status.  The caller keeps the rt_tucker struct alive until that rt_sync.
 *    The adaptive calls choose ranks on the host from device results, so they
 *    return after the stream has finished their work, with every field set.
 *  - Errors: argument errors return RT_EINVAL before anything is enqueued;
 *    HIP failures return RT_EHIP; rt_last_error() gives a message (thread-local,
 *    valid until the next call on the same thread).
 */
#ifndef RTUCKER_H
#define RTUCKER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RT_OK = 0,
    RT_EINVAL = 1,      /* invalid argument (nothing enqueued) */
    RT_ENOMEM = 2,      /* device allocation failed */
    RT_ENONFINITE = 3,  /* the input holds NaN or Inf */
    RT_ECAP = 4,        /* adaptive: rank cap reached before the tolerance */
    RT_EHIP = 5,        /* a HIP runtime call failed */
    RT_EBUSY = 6,       /* serving: the wait queue is full (nothing queued), or the
                           request to cancel has already been admitted */
    RT_ECANCELLED = 7   /* serving: the request was cancelled before admission */
} rt_status;

typedef enum { RT_F32 = 0, RT_F64 = 1 } rt_dtype;

/* Arithmetic of the hot path.
 *  RT_PREC_F64: float64 input, every step in float64.
 *  RT_PREC_F32: float32 input; sketch and projections in float32 with float32
 *               accumulation; Gram matrices, Cholesky, eigenproblems in float64.
 *  RT_PREC_BF16_SKETCH: as RT_PREC_F32 but the sketch runs in bfloat16 on the
 *               matrix cores (float32 accumulation): each float32 operand of
 *               X and Omega is split into two bfloat16 pieces by truncation,
 *               x = h + m + (|remainder| < 2^-15 |x|), and the three piece
 *               products of weight above 2^-16 (hh, hm, mh) are summed, a
 *               relative accuracy near 2^-15 (bf16x3 of Henry, Tang and
 *               Heinecke, ARITH 2019), enough that the sketch's rounding stays
 *               below the tail a randomized range finder leaves.  Modes the
 *               16x16x32 kernel does not serve (J <= 64, R % 8 != 0) take the
 *               float32 sketch.  Orth, projection and truncation stay
 *               float32/float64.  In the adaptive call a bfloat16 block keeps
 *               directions above 1e-4 of its norm, and once such a block adds
 *               no direction the mode continues with float32 sketches. */
typedef enum { RT_PREC_F64 = 0, RT_PREC_F32 = 1, RT_PREC_BF16_SKETCH = 2 } rt_precision;

#define RT_MAXD 8
#define RT_KEEP (-1) /* rank value: leave this mode uncompressed (factor = identity) */
#define RT_LMAX 64   /* largest sketch width r + p (and adaptive rank) per mode */
#define RT_LMAX_FIXED 128  /* largest r + p of the fixed-rank rt_rhosvd / rt_rsthosvd */

/* flags of rt_tucker */
#define RT_FLAG_PADDED 1u    /* some sketch was numerically rank deficient; its basis
                                was completed with zero-weight orthonormal columns */
#define RT_FLAG_FALLBACK 2u  /* orth used the Householder fallback instead of CholeskyQR2 */
#define RT_FLAG_NONFINITE 4u /* the input held NaN or Inf (the result is not meaningful) */
#define RT_FLAG_BADCOORD 8u  /* a sparse input had a coordinate out of range; those
                                entries were ignored (rt_sync returns RT_EINVAL) */

typedef struct rt_ctx rt_ctx;

/* Optional device allocator: must return `bytes` of device memory on the
 * context's device (or NULL); `user` is passed through.  Without one the
 * library uses hipMalloc / hipFree. */
typedef void* (*rt_alloc_fn)(size_t bytes, void* user);
typedef void (*rt_free_fn)(void* ptr, void* user);

typedef struct {
    int32_t ndim;             /* 2 .. RT_MAXD */
    int64_t dims[RT_MAXD];    /* every dim >= 1 */
    rt_dtype dtype;
    const void* data;         /* device, dense row-major */
} rt_tensor;

#define RT_MAX_POWER_ITERS 16

typedef struct {
    int32_t oversample;       /* p >= 0 */
    uint64_t seed;            /* Omega seed */
    const int32_t* order;     /* host, ndim mode indices (a permutation), or NULL:
                                 largest modes first, ties by index (§3.3) */
    rt_precision prec;        /* must match the input dtype: F64 <-> RT_F64 */
    int32_t power_iters;      /* q in [0, RT_MAX_POWER_ITERS]: steps of randomized
                                 subspace iteration inside every RandSVD of
                                 rt_rhosvd / rt_rsthosvd (the range-finding variant
                                 of §5 and §6: after Q = orth(G_(n) Omega), q times
                                 Q <- orth(G_(n) orth(G_(n)^T Q)), the inner orth by
                                 the eigendecomposition of the fp64 Gram, singular
                                 values below 1e-13 (fp64) / 1e-6 (fp32) of the
                                 largest raised to that floor); 0 = Alg. 1 as printed.
                                 Each step adds two reads of the current core and
                                 one core-sized write.  Must be 0 for the
                                 adaptive calls. */
} rt_opts;

typedef struct {
    int32_t ndim;
    int64_t dims[RT_MAXD];      /* input dims */
    int32_t ranks[RT_MAXD];     /* core dims */
    rt_dtype dtype;
    void* core;                 /* device, row-major ranks[0] x ... x ranks[ndim-1] */
    void* factors[RT_MAXD];     /* device, row-major dims[j] x ranks[j], orthonormal
                                   columns; NULL for an uncompressed mode */
    double norm_x;              /* ||X||_F (fp64 accumulation) */
    double core_norm;           /* ||G||_F */
    double rel_err_est;         /* sqrt(max(0, ||X||^2 - ||G||^2)) / ||X|| (the identity
                                   of orthonormal factors; -1 for rt_sp_sthosvd).  For
                                   float32 data ||G||^2 carries the core's float32
                                   rounding, a few 1e-7 of ||X||^2, so estimates below
                                   about 1e-3 are not resolved and may read 0; a direct
                                   residual decides there */
    uint32_t flags;             /* RT_FLAG_* */
} rt_tucker;

/* Library version string (static storage). */
const char* rt_version(void);

/* Message of the last failed call on this thread ("" if none). */
const char* rt_last_error(void);

/* Create a context on `device` that enqueues on `stream` (a hipStream_t, NULL =
 * the default stream).  alloc/free may be NULL (hipMalloc/hipFree).  The
 * context caches its device workspace between calls; it is not thread-safe. */
rt_status rt_create(rt_ctx** ctx, int device, void* stream, rt_alloc_fn alloc, rt_free_fn free_fn, void* user);

/* Change the stream of a context. */
rt_status rt_set_stream(rt_ctx* ctx, void* stream);

/* Free the workspace and the context. */
rt_status rt_destroy(rt_ctx* ctx);

/* R-HOSVD (Alg. 2, §3.1).  ranks (host, ndim entries): r_j >= 1 or RT_KEEP, with
 * r_j + p <= min(I_j, prod_{i != j} I_i) and r_j + p <= RT_LMAX_FIXED.  Modes
 * with r_j + p > RT_LMAX take a slower path (sketch in column blocks, Householder
 * orth, one-sided Jacobi truncation, all in fp64 by single workgroups) and need
 * opts->power_iters == 0.  On success `out` holds a core and factors allocated
 * with the context's allocator; release them with rt_tucker_release. */
rt_status rt_rhosvd(rt_ctx* ctx, const rt_tensor* X, const int32_t* ranks, const rt_opts* opts, rt_tucker* out);

/* R-STHOSVD (Alg. 3, §3.1): modes in the order opts->order; the core shrinks
 * after each mode.  Arguments as for rt_rhosvd. */
rt_status rt_rsthosvd(rt_ctx* ctx, const rt_tensor* X, const int32_t* ranks, const rt_opts* opts, rt_tucker* out);

/* Structure-preserving STHOSVD (Alg. 6, §5), dense tensors: for every mode in
 * opts->order, Y = G_(n) Omega (ell = r_n + p columns), Q = orth(Y), a selection
 * P of ell rows of Q, A_n = Q (P^T Q)^-1 and G <- P^T G.  The selection is the
 * column-pivoted QR order of Q^T followed by strong rank-revealing QR exchanges
 * (parameter eta = 2) until every entry of A_n is at most 2 in magnitude, so A_n
 * holds the ell x ell identity and ||A_n||_2 <= sqrt(1 + 4 ell (I_n - ell)); the
 * core holds entries of X (dims ell_n; RT_KEEP modes keep theirs).  The factors
 * are not orthonormal: rel_err_est is set to -1.  Other arguments, ownership and
 * errors as rt_rsthosvd (opts->power_iters must be 0). */
rt_status rt_sp_sthosvd(rt_ctx* ctx, const rt_tensor* X, const int32_t* ranks, const rt_opts* opts, rt_tucker* out);

/* Adaptive R-STHOSVD (Alg. 5, §4): the rank of each mode is grown `block`
 * columns at a time until ||G_(n) - Q Q^T G_(n)||_F <= eps_n ||X||_F, with
 * eps_n = eps / sqrt(d) (eps_per_mode == NULL) or eps_per_mode[n] (host array,
 * sum of squares must equal eps^2 to 1e-12 relative; 0 leaves the mode
 * uncompressed), then truncated to the smallest rank whose error estimate
 * still meets eps_n ||X||_F.  max_rank (host, may be NULL) caps each mode
 * (default min(I_n, RT_LMAX_FIXED)); RT_ECAP is returned (with a valid result)
 * when a cap stops a mode before its tolerance.  A basis that grows beyond
 * RT_LMAX columns takes the wide kernels (block Gram-Schmidt in two parts, fp64
 * Gram, one-sided Jacobi).  1 <= block <= RT_LMAX.  opts->oversample is ignored. */
rt_status rt_rsthosvd_adaptive(rt_ctx* ctx, const rt_tensor* X, double eps, const double* eps_per_mode,
                               int32_t block, const int32_t* max_rank, const rt_opts* opts, rt_tucker* out);

/* Adaptive R-HOSVD (Alg. 4, §4): the same block range finder and truncation on
 * the mode-n unfolding of X itself for every mode (tolerance eps_n ||X||_F, so
 * that the error of X x_j A_j A_j^T is at most eps ||X||_F), then the core
 * X x_1 A_1^T ... x_d A_d^T.  Arguments, ownership and errors as for
 * rt_rsthosvd_adaptive (opts->order only sets the order the modes are
 * processed in). */
rt_status rt_rhosvd_adaptive(rt_ctx* ctx, const rt_tensor* X, double eps, const double* eps_per_mode,
                             int32_t block, const int32_t* max_rank, const rt_opts* opts, rt_tucker* out);

/* Release the core and factors of a result produced by this context (waits for
 * the stream; a result not yet filled by rt_sync is dropped from it). */
rt_status rt_tucker_release(rt_ctx* ctx, rt_tucker* t);

/* ---- hot-path steps, exposed for testing --------------------------------------- */

/* Tucker reconstruction (decompression) X_hat = G x_1 A_1 x_2 ... x_d A_d (§2.1,
 * the approximation every decomposition call defines).  t: a result of the calls
 * above or any tensor of the same form (core: row-major ranks[0] x ... x
 * ranks[d-1] in t->dtype, factors[j]: row-major dims[j] x ranks[j], or NULL for a
 * mode kept whole, whose rank must equal its dimension, or of rank 0; norms and
 * flags are ignored; a rank 0 gives a zero result).  out: device buffer of dims[0] x ... x dims[d-1] elements of
 * t->dtype, written in full (row-major).  Float data runs on the MFMA projection
 * kernels with the factor transposed, float64 on the fp64 kernels.  Asynchronous:
 * `out` is complete once the stream reaches this point. */
rt_status rt_reconstruct(rt_ctx* ctx, const rt_tucker* t, void* out);

/* Y = X_(mode) Omega_mode[:, col0 : col0 + ell] (Alg. 1 step 1) for a row-major
 * tensor X, written to Y (device, float64, dims[mode] x ell, row-major).
 * prec selects the arithmetic (F64 needs an RT_F64 tensor).  If nrm2 is not NULL
 * it receives ||X||_F^2 (device, one float64).  1 <= ell <= RT_LMAX. */
rt_status rt_sketch(rt_ctx* ctx, const rt_tensor* X, int32_t mode, int32_t ell, int64_t col0, uint64_t seed,
                    rt_precision prec, double* Y, double* nrm2);

/* rt_sketch for callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * result, plan and kernels, with every temporary (split-K partial sums, norm
 * partials, reduction temporaries) in a static device array of 64 MiB that each
 * GPU holds from library load until the process ends; it calls no allocator.
 * Enqueues on the context's stream and returns without waiting (Y and *nrm2 are
 * valid once the stream has reached that point).  A shape whose temporaries
 * exceed 64 MiB (float64 sketches of width above about 32 over many columns,
 * or float sketches of width near 64 over long, non-x8 modes) returns RT_EINVAL
 * before anything is enqueued.  All calls on one GPU share the array: calls that
 * overlap on one GPU (other streams or threads) race and must be serialised by
 * the caller. */
rt_status rt_sketch_noalloc(rt_ctx* ctx, const rt_tensor* X, int32_t mode, int32_t ell, int64_t col0,
                            uint64_t seed, rt_precision prec, double* Y, double* nrm2);

/* Q = orth(Y) (Alg. 1 step 2): Y (device, float64, rows x ell, row-major) is
 * overwritten by an orthonormal Q with range(Y) inside range(Q).  *flags (host)
 * receives RT_FLAG_* bits.  ell <= rows, ell <= RT_LMAX. */
rt_status rt_orth(rt_ctx* ctx, double* Y, int64_t rows, int32_t ell, uint32_t* flags);

/* B = X x_mode Q^T (Alg. 1 step 3): Q (device, dims[mode] x ell, row-major,
 * dtype qtype), B (device, X's dims with dims[mode] replaced by ell, X's dtype).
 * qtype may be RT_F64 for an RT_F32 tensor (fp64 accumulation).  If gram is not
 * NULL it receives B_(mode) B_(mode)^T (device, ell x ell float64). */
rt_status rt_project(rt_ctx* ctx, const rt_tensor* X, int32_t mode, const void* Q, rt_dtype qtype, int32_t ell,
                     void* B, double* gram);

/* Omega_mode[c0 + i, col0 + j] for i < nrows, j < ncols into out (device,
 * row-major, float32 or float64 transform). */
rt_status rt_omega(rt_ctx* ctx, uint64_t seed, int32_t mode, int64_t c0, int64_t nrows, int64_t col0,
                   int32_t ncols, rt_dtype dtype, void* out);

/* Raw Philox4x32-10 words of the Omega stream: out[4 i + t] = word t of the block
 * at counter (c0 + i, q, mode) and key seed (device, uint32). */
rt_status rt_philox_words(rt_ctx* ctx, uint64_t seed, int32_t mode, int64_t c0, int64_t n, uint32_t q,
                          uint32_t* out);

/* ---- tile table (autotuning) ----------------------------------------------------- */
/* The launch shape of the sketch (which kernel variant, its row blocking, and
 * how many workgroups the split over the unfolding's columns aims for) comes
 * from a process-wide table when an entry matches, else from built-in rules.
 * The table is written by the project's tuner, which times the candidate shapes
 * of representative problems on the device (paper_1905_07311_amd/tune.py, table
 * in paper_1905_07311_amd/tuning/); the Python binding installs it at load.  An
 * entry applies to sketches of tensors of `dtype` at precision `prec` whose
 * mode-n unfolding has J in [j_lo, j_hi] rows and K in [k_lo, k_hi] columns,
 * width ell in [ell_lo, ell_hi], and stride class `stride`; the first matching
 * entry wins.  An entry whose variant does not serve the shape, or would lower
 * the precision (the bfloat16 sketch for RT_PREC_F32), is skipped. */
#define RT_TUNE_SKETCH 0
#define RT_STRIDE_FIRST 0   /* mode 0: the unfolding's columns are contiguous rows of X */
#define RT_STRIDE_INNER 1   /* 0 < n < d - 1 */
#define RT_STRIDE_LAST 2    /* the last mode: X_(n) is read along its rows */
typedef struct {
    int32_t op;               /* RT_TUNE_SKETCH */
    rt_dtype dtype;
    rt_precision prec;
    int32_t stride;           /* RT_STRIDE_* */
    int64_t j_lo, j_hi;
    int64_t k_lo, k_hi;
    int32_t ell_lo, ell_hi;
    int32_t kind;             /* RT_SKETCH_* variant */
    int32_t rb, rw;           /* row blocking: RT_SKETCH_SPLIT_BF16 / BF16X3: rb in {1, 2, 4}
                                 (16-row blocks per wave); RT_SKETCH_MFMA_F32: (rb, rw) in
                                 {(1,1), (2,1), (2,2)}; 0 = the built-in rule */
    int32_t wgs;              /* workgroups the column split aims for (0 = built-in) */
} rt_tune_entry;

/* Replace the process-wide table with n entries (copied); n = 0 clears it. */
rt_status rt_tuning_set(const rt_tune_entry* entries, int32_t n);

/* The launch shape the sketch of mode `mode` of a tensor of `dims` (host, ndim
 * values) would use at width ell (col0 = 0, 16-byte aligned data): *out gets
 * the variant and its parameters (bounds = the shape itself, wgs = the
 * workgroups of the launch); *from_table is 1 when a table entry chose it. */
rt_status rt_tuning_plan(rt_dtype dtype, rt_precision prec, const int64_t* dims, int32_t ndim, int32_t mode,
                         int32_t ell, rt_tune_entry* out, int32_t* from_table);

/* ---- timing log --------------------------------------------------------------- */

/* Kernel kinds of the timing log. */
#define RT_KIND_SKETCH 0    /* Y = X_(n) Omega, bytes = X read, flops = 2 ell N */
#define RT_KIND_PROJECT 1   /* B = X x_n Q^T, bytes = X read + B written, flops = 2 ell N */
#define RT_KIND_ORTH 2      /* single-workgroup orth(Y) */
#define RT_KIND_TRUNCATE 3  /* single-workgroup eigensolver + factor */
#define RT_KIND_GRAM 4      /* fp64 Gram of B for the truncation (unfused variant) */
#define RT_KIND_REDUCE 5    /* fixed-order sum of a sketch's split-K partials, bytes = partials read */

/* Set the per-launch timing log and clear it.  `kinds` is a bit mask over the
 * RT_KIND_* values (bit k records launches of kind k; 0 turns the log off,
 * RT_TIMING_ALL records every kind).  A recorded launch is bracketed by HIP
 * events on the context's stream. */
#define RT_TIMING_ALL 0x3f
rt_status rt_timing(rt_ctx* ctx, int32_t kinds);

/* Number of entries in the timing log. */
rt_status rt_timing_count(rt_ctx* ctx, int64_t* n);

/* Entry i of the timing log (host outputs): kind (RT_KIND_*), elapsed
 * milliseconds between the bracketing events, algorithmic bytes and flops of the
 * launch, rows (J) and columns (K) of the unfolding, and the sketch width. */
rt_status rt_timing_entry(rt_ctx* ctx, int64_t i, int32_t* kind, double* ms, double* bytes, double* flops,
                          int64_t* rows, int64_t* cols, int32_t* ell);

/* Kernel variant of entry i of the timing log (host output).  For sketches:
 * RT_SKETCH_GENERIC (LDS-staged vector ALU), RT_SKETCH_MFMA_F32 (float32
 * MFMA), RT_SKETCH_SPLIT_BF16 (float32 products formed from three bfloat16
 * pieces per operand, six piece products on the 16x16x32 bfloat16 MFMA, float32
 * accuracy), RT_SKETCH_BF16X3 (the bfloat16 sketch: two bfloat16 pieces per
 * operand, three piece products on the same MFMA), RT_SKETCH_COO (the sketch of
 * a sparse tensor); 0 for the other kinds. */
#define RT_SKETCH_GENERIC 0
#define RT_SKETCH_MFMA_F32 1
#define RT_SKETCH_SPLIT_BF16 3
#define RT_SKETCH_BF16X3 4
#define RT_SKETCH_COO 5       /* sparse (coordinate) sketch, atomic fp64 adds */
rt_status rt_timing_variant(rt_ctx* ctx, int64_t i, int32_t* variant);

/* Block until the context's stream is idle, then fill the scalars of every
 * result of an asynchronous call made since the last rt_sync.  Returns
 * RT_ENONFINITE if the input of any of them held NaN or Inf (that result's
 * flags carry RT_FLAG_NONFINITE), RT_EINVAL if a sparse input had a coordinate
 * out of range (RT_FLAG_BADCOORD), RT_EHIP if the stream failed, else RT_OK. */
rt_status rt_sync(rt_ctx* ctx);

/* ---- sparse tensors: structure-preserving STHOSVD (Alg. 6, §5) ---------------- */
/* A d-way tensor in coordinate (COO) storage: entry e has coordinates
 * idx[m * nnz + e] (0 <= idx < dims[m]) and value vals[e].  Coordinates should
 * be distinct; repeated ones act as one entry holding their sum, except that
 * norm_x is then sqrt(sum of vals^2) rather than ||X||_F. */
typedef struct {
    int32_t ndim;             /* 2 .. RT_MAXD */
    int64_t dims[RT_MAXD];    /* 1 .. 2^31 - 1 */
    int64_t nnz;              /* >= 0 */
    rt_dtype dtype;
    const int32_t* idx;       /* device, ndim x nnz int32, mode-major */
    const void* vals;         /* device, nnz values of dtype */
} rt_coo;

/* SP-STHOSVD (Alg. 6) of a sparse tensor.  Every intermediate core stays in
 * coordinate storage: step n sketches the current core, Y = G_(n) Omega_n
 * (cost O(nnz ell), §5), selects ell = r_n + p rows P of Q = orth(Y) as
 * rt_sp_sthosvd does, and keeps the entries of the selected mode-n slices,
 * renumbered by their position in the selection (G_(n) <- P^T G_(n)), so the
 * core holds entries of X only and never grows.  The result is laid out as
 * rt_sp_sthosvd's on the dense tensor: a dense core (ell_1 x ... x ell_d) of
 * entries of X, factors A_n = Q (P^T Q)^-1 (dims[n] x ell_n) that contain the
 * ell x ell identity, rel_err_est = -1.  opts->prec: RT_PREC_F64 for RT_F64
 * values, RT_PREC_F32 for RT_F32 (sketch in fp64 accumulation either way);
 * power_iters must be 0.  Asynchronous as the other fixed-rank calls; entries
 * with a coordinate out of range are ignored and rt_sync then returns
 * RT_EINVAL.  The sketch adds into Y with atomic operations, so results are
 * reproducible to fp64 rounding rather than bitwise. */
rt_status rt_sp_sthosvd_coo(rt_ctx* ctx, const rt_coo* X, const int32_t* ranks, const rt_opts* opts,
                            rt_tucker* out);

/* Y = X_(mode) Omega_mode[:, col0 : col0 + ell] of a sparse tensor (the sketch
 * step of Alg. 6), Y device float64 dims[mode] x ell; Omega is the generator of
 * rt_sketch in the precision of the values (float32 normals for RT_F32, float64
 * for RT_F64).  nrm2 (device, optional) receives the sum of vals^2.  Waits for
 * the stream; RT_EINVAL if some coordinate is out of range (those entries are
 * skipped).  1 <= ell <= RT_LMAX. */
rt_status rt_sketch_coo(rt_ctx* ctx, const rt_coo* X, int32_t mode, int32_t ell, int64_t col0, uint64_t seed,
                        double* Y, double* nrm2);

/* ---- serving: continuous batching of many requests --------------------------- */
/* A server runs adaptive R-STHOSVD (Alg. 5, §4) on a stream of float32 tensors of
 * uneven shapes, and decompressions (rt_server_submit_reconstruct) beside them.  Requests wait in arrival order and are admitted as soon as a
 * slot is free and their device memory fits in `hbm_budget`.
 *
 * RT_SERVE_GROUPED (default): one executor drives every admitted request through
 * the method's steps in lock-step iterations.  In each iteration the requests in
 * their block phase share one launch of each step (the block sketch, its sums,
 * the block orthonormalisation, the projection) and the requests whose mode has
 * stopped growing share the truncation launches (Gram, eigensolver with rank
 * choice and factor, core update); the iteration is one captured HIP graph
 * (descriptor copy plus the launches, replayed every iteration) followed by one
 * wait, after which the host advances every request (next block, truncation,
 * next mode, done).  While an iteration runs, the host copies out the results
 * of requests finished by the previous one and admits new requests, whose
 * inputs cross on two copy streams and join the next iteration.  A request's footprint is the exact
 * workspace of its shape (input, basis, projections, cores, factors).  A request
 * whose block step does not fit the grouped kernel (a mode longer than 910 rows
 * for blocks of 8) runs alone through rt_rsthosvd_adaptive, and so is a request
 * redone whose basis would grow past RT_LMAX columns (the shared kernels' cap;
 * the single-request path grows to RT_LMAX_FIXED).  Float32 sketches.
 * RT_SERVE_SLOTS: every slot runs whole requests through rt_rsthosvd_adaptive
 * on a stream of its own (float32 or bfloat16 sketches).
 *
 * Either way a request's result does not depend on what else is in flight (the
 * work of a request is split by its own shape and every sum has a fixed order). */
typedef struct rt_server rt_server;

#define RT_SERVE_GROUPED 0
#define RT_SERVE_SLOTS 1

typedef struct {
    int32_t max_inflight;     /* requests in flight (slots): 1 .. 64 */
    size_t hbm_budget;        /* bytes; 0 = 3/4 of the device memory free at creation */
    rt_precision prec;        /* RT_PREC_F32 (either mode) or RT_PREC_BF16_SKETCH (slots) */
    double eps;               /* relative tolerance of every request (eps_n = eps / sqrt(d)) */
    int32_t block;            /* adaptive block size, 1 .. RT_LMAX (grouped: 1 .. 16) */
    int32_t mode;             /* RT_SERVE_GROUPED or RT_SERVE_SLOTS */
    int32_t max_queued;       /* requests waiting for admission; 0 = unbounded.  A
                                 submission beyond it returns RT_EBUSY and queues
                                 nothing (back-pressure for the caller) */
} rt_server_opts;

typedef struct {
    rt_status status;         /* of the request's computation */
    int32_t ndim;
    int64_t dims[RT_MAXD];
    int32_t ranks[RT_MAXD];
    const float* core;        /* host, row-major core, owned by the server until rt_server_release */
    const float* factors[RT_MAXD];  /* host, row-major dims[j] x ranks[j] */
    double norm_x, core_norm, rel_err_est;
    uint32_t flags;
    double queue_s;           /* submission -> admission, seconds */
    double latency_s;         /* submission -> result on the host, seconds */
} rt_result;

/* Start a server on `device` (its threads and streams live until destroy). */
rt_status rt_server_create(rt_server** srv, int device, const rt_server_opts* opts);

/* Queue a request.  X->data is HOST memory (float32, dense row-major) that must
 * stay valid and unchanged until the request completes; page-locked memory lets
 * the copy to the device overlap other work.  *ticket identifies the request. */
rt_status rt_server_submit(rt_server* srv, const rt_tensor* X, uint64_t seed, uint64_t* ticket);

/* A Tucker decomposition in host memory, float32 (a served result, or any). */
typedef struct {
    int32_t ndim;
    int64_t dims[RT_MAXD];
    int32_t ranks[RT_MAXD];
    const float* core;              /* host, row-major ranks[0] x ... x ranks[ndim-1] */
    const float* factors[RT_MAXD];  /* host, row-major dims[j] x ranks[j]; NULL: the
                                       mode is kept (ranks[j] == dims[j]) or ranks[j] == 0 */
} rt_tucker_host;

/* Queue a decompression: X_hat = G x_1 A_1 ... x_d A_d (rt_reconstruct) written to
 * `out` (host, prod(dims) float32, row-major).  t's arrays and `out` stay owned
 * by the caller and must stay valid until the request completes.  The request
 * takes a slot like a compression; its rt_result carries status, dims, ranks
 * and the times (core and factors NULL).  In the grouped mode it runs on the
 * executor between iterations. */
rt_status rt_server_submit_reconstruct(rt_server* srv, const rt_tucker_host* t, float* out, uint64_t* ticket);

/* *done = 1 and *out filled when the request has completed, else *done = 0. */
rt_status rt_server_poll(rt_server* srv, uint64_t ticket, int32_t* done, rt_result* out);

/* Block until the request has completed, then fill *out. */
rt_status rt_server_wait(rt_server* srv, uint64_t ticket, rt_result* out);

/* Free the host result of a completed request (its pointers become invalid). */
rt_status rt_server_release(rt_server* srv, uint64_t ticket);

/* Withdraw a request that is still waiting for admission: it leaves the queue
 * and completes at once with status RT_ECANCELLED (poll and wait report it;
 * release it like any other).  A request already admitted, running or done is
 * not touched: RT_EBUSY.  An unknown ticket: RT_EINVAL. */
rt_status rt_server_cancel(rt_server* srv, uint64_t ticket);

/* Counters of the grouped executor since creation (slots mode: zeros apart
 * from `completed`).  Per iteration the executor launches, then does the host
 * work that does not feed this iteration (result copies of the last one,
 * admission of new requests: overlap_s), then blocks on the device (wait_s);
 * host_s is its remaining time (descriptors, launch, readback), which the
 * device spends idle.  The three add up to the executor's wall time while
 * requests are in flight. */
typedef struct {
    int64_t iterations;       /* grouped iterations launched */
    int64_t request_steps;    /* requests advanced, summed over iterations */
    int64_t completed;        /* requests completed */
    double wait_s;
    double host_s;
    double overlap_s;
} rt_server_stats;
rt_status rt_server_get_stats(rt_server* srv, rt_server_stats* out);

/* Finish the queued requests, stop the threads, free all memory. */
rt_status rt_server_destroy(rt_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* RTUCKER_H */
