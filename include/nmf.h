/*
 * nmf.h -- C ABI of the MI355X (gfx950) alternating-updating NMF library.
 *
 * Problem (Section 1, Eq. (1)): given a nonnegative m x n matrix A and a rank
 * k, find W (m x k) >= 0 and H (k x n) >= 0 that reduce ||A - W H||_F.
 * Method (Algorithm 1, AU-NMF): repeat { update W from H H^T and A H^T;
 * update H from W^T W and W^T A } for a fixed number of iterations, the
 * stopping rule of Section 6.1.3. The local update is one of
 *   NMF_MU   -- multiplicative update, Section 4.1, Eq. (3);
 *   NMF_HALS -- hierarchical alternating least squares, Section 4.2, Eq. (5);
 *   NMF_ABPP -- exact nonnegative least squares by block principal pivoting,
 *               Section 4.3, Eqs. (6)-(7).
 * The relative error ||A - W H||_F / ||A||_F of Section 6.2 can be reported
 * after every iteration.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All matrix arguments are DEVICE pointers on the context's GPU, row-major,
 *   with the leading dimension (elements between consecutive rows) given
 *   where stated and otherwise equal to the number of columns. Host pointers
 *   are marked "host".
 * - The caller owns every array it passes. The library reads A (and the CSR
 *   arrays), reads and overwrites W and H in place, and writes outputs.
 *   The context owns only its workspace, which it frees in nmf_destroy.
 * - Work is enqueued on the context's HIP stream. A call returns once its
 *   work is enqueued, except that a call given a host rel_err or stats
 *   pointer, or one that must check a device-side error flag (ABPP, input
 *   checks), synchronises the stream before returning.
 * - Errors are reported as nmf_status codes only; no exception or abort
 *   crosses the ABI. Argument checks run on the host before any device
 *   work, so an NMF_EINVAL return has touched no device memory.
 *   nmf_last_error() describes the most recent failure on a context.
 * - Element types: NMF_F64 runs everything in double; NMF_F32 stores A, W, H
 *   in float and accumulates the large products in float on the matrix
 *   cores, with the Gram split-sums and the objective accumulated in double.
 *   NMF_BF16 (dense A only) stores A as bfloat16 (each element the 16 bits
 *   of the value, row pitch lda a multiple of 8 elements, rows 16-byte
 *   aligned) with W, H and every other array in float: the two large
 *   products run on the BF16 matrix cores with float accumulation, the
 *   factor operand rounded to bfloat16 (nearest even) for each product;
 *   Grams, updates and the objective are as for NMF_F32. This is the
 *   reduced-precision variant of the products the paper's Section 6.3.1
 *   breakdown calls MM.
 *   NMF_FP8_E4M3 (dense A only) is the same with A stored as FP8 E4M3 (one
 *   byte each: sign, 4 exponent bits with bias 7, 3 fraction bits; largest
 *   finite 448, bits S.1111.111 NaN; lda a multiple of 16, rows 16-byte
 *   aligned): the products run on the FP8 matrix cores with float
 *   accumulation; for each product every rank column j of the factor operand
 *   is divided by s_j, the smallest power of two with max |column j| <=
 *   448 s_j (1 for a zero column), rounded to E4M3 (nearest even), and the
 *   output column is multiplied by s_j. Any scaling of A itself is the
 *   caller's: the factorisation of c A is c times that of A.
 * - m, n >= 1 and 1 <= k <= NMF_MAX_K; k may exceed min(m, n). NMF_ABPP and
 *   the unrolled-iteration gradients take k <= 64 (NMF_EINVAL otherwise).
 *   With k > min(m, n) a Gram is singular, so ABPP can return NMF_ENUMERIC
 *   or NMF_ENOTCONV there; MU and HALS are defined for any k.
 * - Calls on one context must not overlap: they share its workspace. A
 *   context runs on one stream at a time; nmf_set_stream orders the new
 *   stream after the work already enqueued on the old one.
 */
#ifndef NMF_MI355X_H
#define NMF_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NMF_MAX_K 128

typedef enum {
  NMF_OK = 0,
  NMF_EINVAL = 1,    /* bad argument (null pointer, size, enum, layout)      */
  NMF_ENOMEM = 2,    /* device allocation failed                             */
  NMF_EDEVICE = 3,   /* a HIP call failed                                    */
  NMF_ENUMERIC = 4,  /* NaN/Inf/negative input (check_input) or a singular   */
                     /* passive-set system in ABPP                           */
  NMF_ENOTCONV = 5   /* ABPP: pivot cap reached before the KKT conditions    */
} nmf_status;

typedef enum { NMF_MU = 0, NMF_HALS = 1, NMF_ABPP = 2 } nmf_algo;

typedef enum { NMF_F64 = 0, NMF_F32 = 1, NMF_BF16 = 2, NMF_FP8_E4M3 = 3 } nmf_dtype;

typedef enum {
  NMF_STOP_ITERS = 0,  /* run exactly opts->iters iterations               */
  NMF_STOP_PGRAD = 1,  /* also stop after iteration t once the projected   */
                       /* gradient (see nmf_projected_gradient_sq) has     */
                       /* fallen to ||pg(W_t,H_t)|| <= tol ||pg(W_0,H_0)|| */
  NMF_STOP_RELERR = 2  /* also stop after iteration t once the relative    */
                       /* error improves by less than tol: e_{t-1} - e_t < */
                       /* tol e_{t-1} (needs opts->objective)              */
} nmf_stop;

typedef enum {
  NMF_OBJ_NONE = 0,    /* do not evaluate the objective                    */
  NMF_OBJ_DIRECT = 1   /* ||A - W H||_F from the residual: dense A forms   */
                       /* A - W H tile by tile; CSR A sums (a - wh)^2 -    */
                       /* wh^2 over stored entries plus <W^T W, H H^T>     */
} nmf_objective;

typedef struct {
  int algo;          /* nmf_algo                                             */
  int iters;         /* number of AU-NMF iterations (>= 0)                   */
  double eps_mu;     /* MU: added to every denominator (Eq. (3) has no zero  */
                     /* guard); 1e-16 is the documented default             */
  int max_pivots;    /* ABPP: cap on passive-set solves per right-hand side; */
                     /* <= 0 selects 50 k                                    */
  int objective;     /* nmf_objective, evaluated at start and after each it. */
  int timers;        /* nonzero: fill the per-phase times in nmf_stats       */
  int check_input;   /* nonzero: scan A for NaN/Inf/negative entries and the */
                     /* CSR arrays for out-of-range or unsorted columns      */
  int transpose_a;   /* dense A: 0 (default) keeps a transposed copy of A in */
                     /* device memory for the call when it fits (both large  */
                     /* products then stream A row by row); -1 never does.   */
                     /* NMF_BF16 and NMF_FP8_E4M3 A always need the copy: */
                     /* -1 is rejected and                                  */
                     /* a copy that does not fit returns NMF_ENOMEM          */
  double tol;        /* tolerance of the stopping test (>= 0)                */
  int stop;          /* nmf_stop. Section 6.2: the iteration count together  */
                     /* with a tolerance on a quality metric. With a metric, */
                     /* iters is the cap and the call synchronises once per  */
                     /* iteration to read it                                 */
} nmf_opts;

typedef struct {
  double ms_total;   /* wall time of the iterations (hipEvents)              */
  double ms_mm;      /* large products A H^T, W^T A (Section 6.3.1 "MM")     */
  double ms_luc;     /* local update computations ("LUC")                    */
  double ms_gram;    /* H H^T and W^T W ("Gram")                             */
  double ms_obj;     /* objective evaluations                                */
  double ms_setup;   /* layout copies, CSR transpose                         */
  long long bpp_pivots; /* ABPP: total passive-set solves over all RHS       */
  double ms_mm_aht;  /* the A H^T part of ms_mm (one launch group per iter.) */
  double ms_mm_wta;  /* the W^T A part of ms_mm                              */
  long long iters_done; /* iterations performed (< iters when a stop fired)  */
  double pgrad_ratio;   /* NMF_STOP_PGRAD: ||pg(W,H)|| / ||pg(W_0,H_0)|| at the */
                        /* returned factors; otherwise NaN                    */
  /* ABPP (Section 4.3) work, summed over both half-steps of every iteration.
   * Each passive-set solve eliminates the smaller of two equivalent systems
   * (ns unknowns, ns <= 32); four right-hand sides share a wavefront and
   * eliminate together at the size of the largest of them, rounded up to a
   * size class (8, 12, 16, 18, 20, ..., 30 or 32). */
  long long bpp_solves;       /* eliminations performed                    */
  double bpp_flops;           /* their algorithmic flops: ns^3 - ns (Gauss- */
                              /* Jordan, one right-hand side) + 2 k ns (the */
                              /* other half of the KKT pair) each, plus     */
                              /* 2 k^2 per right-hand side forming G^-1 p   */
  double bpp_size_mean;       /* mean ns                                    */
  double bpp_size_max_mean;   /* mean over the same eliminations of the     */
                              /* largest ns of the wavefront                */
  double bpp_size_class_mean; /* mean size the eliminations ran at          */
} nmf_stats;

typedef struct nmf_ctx nmf_ctx;

/* Fills *opts with the defaults: MU, 0 iterations, eps_mu 1e-16,
 * max_pivots 0 (= 50 k), no objective, no timers, no input check,
 * transpose_a 0, tol 0, stop NMF_STOP_ITERS. */
void nmf_default_opts(nmf_opts* opts);

/* Creates a context bound to HIP device `device` and the HIP stream
 * `hip_stream` (a hipStream_t; NULL means the default stream).
 * device = -1 creates a context bound to no device: every call on it runs
 * its argument checks and then returns NMF_EDEVICE (argument checking on a
 * machine without a GPU). */
nmf_status nmf_create(nmf_ctx** out, int device, void* hip_stream);
void nmf_destroy(nmf_ctx* ctx);
/* Rebinds the context to another stream on the same device. Work the
 * context has already enqueued on the old stream may still be using its
 * workspace, so the new stream is made to wait for it (an event recorded on
 * the old stream) before anything enqueued on it later. */
nmf_status nmf_set_stream(nmf_ctx* ctx, void* hip_stream);

const char* nmf_status_str(nmf_status s);
const char* nmf_last_error(const nmf_ctx* ctx);

/* Full AU-NMF on a dense A (Algorithm 1).
 *   A       m x n, leading dimension lda >= n, element type dtype.
 *   W       m x k (leading dimension k), element type dtype (float for
 *           NMF_BF16 and NMF_FP8_E4M3): the initial W on
 *           entry (read by MU and HALS; ABPP's W step is an exact solve that
 *           only takes its starting passive sets from it), the final W.
 *   H       k x n (leading dimension n): initial H on entry, final H on return.
 *   rel_err host array of iters+1 doubles or NULL; requires opts->objective.
 *           Entries after the last iteration performed (a stop fired) are NaN.
 *   stats   host pointer or NULL.
 * HALS returns W with unit-norm nonzero columns, the scale carried by H. */
nmf_status nmf_dense(nmf_ctx* ctx, nmf_dtype dtype, int64_t m, int64_t n,
                     const void* A, int64_t lda, int k, const nmf_opts* opts,
                     void* W, void* H, double* rel_err, nmf_stats* stats);

/* Full AU-NMF on a sparse A in CSR form, float32 values.
 *   rowptr  m+1 int64, rowptr[0] = 0, rowptr[m] = nnz, nondecreasing.
 *   colidx  nnz int32 column ids in [0, n), increasing within each row.
 *   m, n <= 2^31 - 1 (A^T is built with int32 column ids too), nnz < 2^32.
 *   Rows (of A or A^T) longer than 4096 stored entries are split into
 *   chunks for the products, so power-law row lengths stay balanced.
 *   vals    nnz floats >= 0.
 * W (m x k) and H (k x n) are float32 as for nmf_dense. The transpose of A
 * (needed for W^T A) is built once per call on the device. */
nmf_status nmf_csr(nmf_ctx* ctx, int64_t m, int64_t n, int64_t nnz,
                   const int64_t* rowptr, const int32_t* colidx, const float* vals,
                   int k, const nmf_opts* opts, float* W, float* H,
                   double* rel_err, nmf_stats* stats);

/* ---- Per-step entry points (one phase of Algorithm 1 each) --------------
 * These use the same row layout as the iteration driver: the fixed factor
 * is given with one row per row (W, m x k) or per column (H^T, n x k) of A,
 * so the two half-steps of Algorithm 1 are the same calls with A and A^T.
 */

/* G = X^T X for X rows x k (leading dimension ldx >= k); G is k x k.
 * With X = W this is W^T W; with X = H^T it is H H^T (Algorithm 1). */
nmf_status nmf_gram(nmf_ctx* ctx, nmf_dtype dtype, int64_t rows, int k,
                    const void* X, int64_t ldx, void* G);

/* P = A F for dense A (m x n, lda) and F (n x k, ldf): with F = H^T this is
 * the A H^T of the W update. Output P is m x k (leading dimension k).
 * NMF_BF16: A bfloat16 (lda a multiple of 8), F and P float; F is rounded
 * to bfloat16 for the product, as in nmf_dense. NMF_FP8_E4M3 likewise (lda
 * a multiple of 16; F scaled per column and rounded to E4M3 as in
 * nmf_dense). */
nmf_status nmf_dense_AF(nmf_ctx* ctx, nmf_dtype dtype, int64_t m, int64_t n,
                        const void* A, int64_t lda, int k, const void* F,
                        int64_t ldf, void* P);

/* R = A^T F for dense A (m x n, lda) and F (m x k, ldf): with F = W this is
 * (W^T A)^T of the H update. Output R is n x k (leading dimension k).
 * NMF_BF16 and NMF_FP8_E4M3 as for nmf_dense_AF (the call makes a
 * transposed copy of A). */
nmf_status nmf_dense_AtF(nmf_ctx* ctx, nmf_dtype dtype, int64_t m, int64_t n,
                         const void* A, int64_t lda, int k, const void* F,
                         int64_t ldf, void* R);

/* P = A F for CSR A (m x n, float32) and dense F (n x k, float32, leading
 * dimension k). With the CSR arrays of A^T this computes A^T W instead. */
nmf_status nmf_csr_AF(nmf_ctx* ctx, int64_t m, int64_t n, int64_t nnz,
                      const int64_t* rowptr, const int32_t* colidx,
                      const float* vals, int k, const float* F, float* P);

/* CSR of A^T (n rows) from CSR of A: rowptr_t has n+1 entries, colidx_t and
 * vals_t have nnz; columns within each output row are increasing. */
nmf_status nmf_csr_transpose(nmf_ctx* ctx, int64_t m, int64_t n, int64_t nnz,
                             const int64_t* rowptr, const int32_t* colidx,
                             const float* vals, int64_t* rowptr_t,
                             int32_t* colidx_t, float* vals_t);

/* One local update of X (rows x k, leading dimension k) in place, given the
 * Gram G (k x k) of the fixed factor and the product P (rows x k) of A with
 * it: row r of X is the row of W (or of H^T) that Algorithm 1 updates from
 * G and row r of P.
 *   NMF_MU:   x <- x .* p ./ (x G + eps_mu)                      (Eq. (3))
 *   NMF_HALS: for i = 1..k in order: if G_ii > 0,
 *             x_i <- max(0, x_i + (p_i - x G_:i) / G_ii)        (Eq. (5))
 *             (no normalisation here; see nmf_hals_normalize)
 *   NMF_ABPP: x <- argmin_{x >= 0} 1/2 x^T G x - p^T x          (Eqs. (6)-(7))
 *             by block principal pivoting. The support of the incoming row
 *             of X is only the starting passive set; the result is the
 *             unique minimiser whatever X holds (G positive definite).
 *             pivots (host, nullable) receives the total number of
 *             passive-set solves. */
nmf_status nmf_update(nmf_ctx* ctx, nmf_algo algo, nmf_dtype dtype,
                      int64_t rows, int k, const void* G, const void* P,
                      void* X, const nmf_opts* opts, long long* pivots);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * update as nmf_update, with the same arguments, kernels and results, whose
 * scratch (padded copies of G, P and X, the ABPP counters and inverse Gram)
 * lives in a fixed device array of NMF_NOALLOC_SCRATCH_BYTES that each GPU
 * holds from the first context created on it until the process ends. The
 * call never allocates or frees memory and issues no hipMemset; the caller
 * still owns G, P and X.
 *   Size limit: with KP = k rounded up to 16 and e = sizeof(element), the
 *   call needs 2 rows KP e + KP^2 (e + 8) bytes plus at most 1024 of
 *   alignment, which must not exceed NMF_NOALLOC_SCRATCH_BYTES (F32,
 *   k <= 64: about 130,000 rows; F64, k = 128: about 32,600); larger calls
 *   return NMF_EINVAL before any device work.
 *   Sharing: every call on one GPU, from any context or stream, uses that
 *   GPU's one array, which keeps the last call's contents (each call clears
 *   what must start at zero). Calls that overlap on one GPU race; serialise
 *   them.
 *   Synchronisation: as nmf_update (MU and HALS only enqueue work; ABPP
 *   synchronises the stream to read its status and pivot count). */
#define NMF_NOALLOC_SCRATCH_BYTES (64u << 20)
nmf_status nmf_update_noalloc(nmf_ctx* ctx, nmf_algo algo, nmf_dtype dtype,
                              int64_t rows, int k, const void* G, const void* P,
                              void* X, const nmf_opts* opts, long long* pivots);

/* HALS column normalisation with compensation (Section 4.2): for every
 * i < k with s_i = ||w^i||_2 > 0, w^i <- w^i / s_i and h_i <- s_i h_i, so
 * W H is unchanged. W is m x k, Ht = H^T is n x k (both leading dimension
 * k), both updated in place. S (k x k, nullable) receives W^T W of the
 * normalised W; norms (k entries, nullable, device) receives s. */
nmf_status nmf_hals_normalize(nmf_ctx* ctx, nmf_dtype dtype, int64_t m,
                              int64_t n, int k, void* W, void* Ht, void* S,
                              void* norms);

/* Relative error ||A - W H||_F / ||A||_F of Section 6.2 for dense A, with W
 * (m x k) and Ht = H^T (n x k). Residual formed explicitly, squares summed
 * in double. Result written to the host double *out (synchronises).
 * NMF_BF16 / NMF_FP8_E4M3: A in that format, W and Ht float. */
nmf_status nmf_dense_relerr(nmf_ctx* ctx, nmf_dtype dtype, int64_t m,
                            int64_t n, const void* A, int64_t lda, int k,
                            const void* W, const void* Ht, double* out);

/* Same for CSR A: sum over stored entries of (a - wh)^2 - wh^2, plus
 * <W^T W, H H^T> for the zeros. */
nmf_status nmf_csr_relerr(nmf_ctx* ctx, int64_t m, int64_t n, int64_t nnz,
                          const int64_t* rowptr, const int32_t* colidx,
                          const float* vals, int k, const float* W,
                          const float* Ht, double* out);

/* Stationarity measure of Section 6.2 for one factor: with X rows x k (the
 * rows of W, or of H^T), P = A F (rows x k, the product with the other
 * factor) and G = F^T F (k x k), the gradient of 1/2 ||A - W H||_F^2 in X is
 * X G - P; its projection onto the feasible directions keeps an entry where
 * x > 0 and only its negative part where x = 0. *out (host) receives the sum
 * of the squared projected entries (accumulated in double); the norm of
 * nmf_opts' NMF_STOP_PGRAD test is the square root of the W and H sums. */
nmf_status nmf_projected_gradient_sq(nmf_ctx* ctx, nmf_dtype dtype, int64_t rows,
                                     int k, const void* X, const void* P,
                                     const void* G, double* out);

/* ---- Differentiation through unrolled MU iterations -------------------------
 * The map (A, W_0, H_0) -> (W_T, H_T) of T iterations of Algorithm 1 with the
 * MU rule of Section 4.1, Eq. (3) (W step, then H step; eps added to every
 * denominator), and its reverse-mode gradient for any scalar loss of
 * (W_T, H_T). Dense A, NMF_F32 or NMF_F64, 1 <= k <= 64.
 *
 * Checkpoints: the forward pass stores the factors entering iterations
 * 0, c, 2c, ... (c = ckpt_every >= 1) in a device buffer of
 * nmf_mu_ckpt_elems(m, n, k, T, c) elements of dtype (the library's internal
 * padded row layout; opaque to the caller). The backward pass recomputes each
 * segment of c iterations from its checkpoint and runs the adjoint through
 * it in reverse, so its memory grows with c, not with T. It must be given the
 * same m, n, A, k, T, eps and c as the forward pass that wrote the buffer.
 * The gradients of W_0 and H_0 do not depend on c, bit for bit; dL/dA is
 * summed one segment at a time, so its float rounding does.
 */

/* Elements of dtype in the checkpoint buffer, or -1 for invalid sizes. */
int64_t nmf_mu_ckpt_elems(int64_t m, int64_t n, int k, int iters, int ckpt_every);

/* W (m x k, leading dimension k) and H (k x n, leading dimension n): W_0 and
 * H_0 on entry, W_T and H_T on return. ckpt: device buffer as above, or NULL
 * when no backward pass will follow. */
nmf_status nmf_mu_unrolled_forward(nmf_ctx* ctx, nmf_dtype dtype, int64_t m,
                                   int64_t n, const void* A, int64_t lda, int k,
                                   int iters, double eps, int ckpt_every,
                                   void* W, void* H, void* ckpt);

/* Given gW = dL/dW_T (m x k) and gH = dL/dH_T (k x n), writes
 * gW0 = dL/dW_0 (m x k), gH0 = dL/dH_0 (k x n) and, if gA is not NULL,
 * gA = dL/dA (m x n, leading dimension ldga >= n; overwritten). */
nmf_status nmf_mu_unrolled_backward(nmf_ctx* ctx, nmf_dtype dtype, int64_t m,
                                    int64_t n, const void* A, int64_t lda, int k,
                                    int iters, double eps, int ckpt_every,
                                    const void* ckpt, const void* gW,
                                    const void* gH, void* gA, int64_t ldga,
                                    void* gW0, void* gH0);

/* ---- Differentiation through unrolled HALS iterations -----------------------
 * The map (A, W_0, H_0) -> (W_T, H_T) of T iterations of Algorithm 1 with the
 * HALS rules of Section 4.2, Eq. (5), exactly as nmf_dense runs them (the
 * exact block minimiser of each column, the columns of W normalised after
 * the sweep with H rescaled to compensate, then the sweep over the rows of
 * H), and its reverse-mode gradient for any scalar loss of (W_T, H_T). The
 * map is piecewise smooth: the gradient is that of the piece the forward
 * pass is on (an entry clipped to zero carries none; a column with a zero
 * Gram diagonal, which the sweep skips, passes its gradient through). Dense
 * A, NMF_F32 or NMF_F64, 1 <= k <= 64. The checkpoint buffer has
 * nmf_mu_ckpt_elems(m, n, k, T, c) elements, as for MU, and the backward
 * pass must be given the same m, n, A, k, T and c as the forward pass. */
nmf_status nmf_hals_unrolled_forward(nmf_ctx* ctx, nmf_dtype dtype, int64_t m,
                                     int64_t n, const void* A, int64_t lda, int k,
                                     int iters, int ckpt_every, void* W, void* H,
                                     void* ckpt);

/* As nmf_mu_unrolled_backward, for the HALS map. */
nmf_status nmf_hals_unrolled_backward(nmf_ctx* ctx, nmf_dtype dtype, int64_t m,
                                      int64_t n, const void* A, int64_t lda, int k,
                                      int iters, int ckpt_every, const void* ckpt,
                                      const void* gW, const void* gH, void* gA,
                                      int64_t ldga, void* gW0, void* gH0);

#ifdef __cplusplus
}
#endif

#endif /* NMF_MI355X_H */
