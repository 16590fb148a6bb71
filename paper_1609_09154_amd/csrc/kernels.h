// Host-side interface between the C ABI (api.hip) and the kernel files.
// Every function enqueues work on the given stream and returns the launch
// status; none of them allocates memory.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nmfk {

enum class GemmKind { NN, TN, TN_GRAM };

// D (M x N) = X * Y (NN, X is M x K) or X^T * Y (TN, X is K x M). Y is
// K x N, or, with yt set, its transpose N x K (ldy between its N rows; then
// Y must be 16-byte aligned with ldy a multiple of 16 bytes). N must be a
// multiple of 16 between 16 and 128.
template <typename T> struct GemmArgs {
  const T* X; int64_t ldx;
  const T* Y; int64_t ldy;
  T* D; int64_t ldd;
  int64_t M, N, K;
  bool yt;
  int nvalid;  // output columns that matter (0: all N); columns >= nvalid may be 0
  T* Dt;       // nullable: also receives D transposed (Dt[j * M + i]; Grams only)
};

// `part` must hold splits * M * N elements when splits > 1. splits <= 0 picks
// the split count automatically (gemm_auto_splits, at most
// MAX_PRODUCT_SPLITS for the products: 32, so that products with few output
// rows still fill the chip).
constexpr int64_t MAX_PRODUCT_SPLITS = 32;
// With nsplit set, a split product is not summed: the slabs stay in part
// (slab s at part + s M N, ld N) and *nsplit receives their count, for a
// consumer that adds them itself (Split below); *nsplit = 1 means D holds
// the product.
template <typename T>
hipError_t gemm_run(GemmKind kind, const GemmArgs<T>& a, int64_t splits, T* part,
                    hipStream_t st, int* nsplit = nullptr);

// A product handed over as n slabs of rows x KP (slab q at p + q stride),
// whose entries the consumer sums in slab order in double and rounds once,
// as reduce_splits does (n = 1: p is the product itself). p == nullptr: no
// product.
template <typename T> struct Split {
  const T* p;
  int n;
  int64_t stride;
};
template <typename T>
int64_t gemm_auto_splits(GemmKind kind, int64_t M, int64_t N, int64_t K);
// D[i][j] (ld ldd) = sum over s of part[s * dsplit + i * ldp + j], in the
// order s = 0, 1, ... with double sums, for i < M, j < N.
template <typename T>
hipError_t reduce_splits(const T* part, int splits, int64_t dsplit, int64_t M, int N,
                         int64_t ldd, T* D, int64_t ldp, hipStream_t st, T* Dt = nullptr);

// Reduced-precision products: D (M x N float, ld ldd) = X Y^T for X (M x K)
// and Y (N x K) stored as bfloat16 bits (uint16_t) or FP8 E4M3 bits
// (uint8_t), K contiguous in both (rows 16-byte aligned, ldx and ldy whole
// multiples of 16 bytes), N a multiple of 16 up to 128, float accumulation.
// The FP8 form multiplies output column j by colscale[j]. `part` must hold
// gemm_lp_splits(M, K) * M * N floats when that count exceeds 1.
hipError_t gemm_bf16_nt(const uint16_t* X, int64_t ldx, const uint16_t* Y, int64_t ldy, float* D,
                        int64_t ldd, int64_t M, int N, int64_t K, float* part, hipStream_t st);
hipError_t gemm_fp8_nt(const uint8_t* X, int64_t ldx, const uint8_t* Y, int64_t ldy,
                       const float* colscale, float* D, int64_t ldd, int64_t M, int N, int64_t K,
                       float* part, hipStream_t st);
int64_t gemm_lp_splits(int64_t M, int64_t K);
// Ft (KP x rows, row pitch ldt) = F^T rounded to bfloat16 (nearest even), for
// F rows x KP float.
hipError_t pack_bf16_t(const float* F, int64_t rows, int KP, uint16_t* Ft, int64_t ldt,
                       hipStream_t st);
// Ft = FP8 E4M3 of F^T with column j divided by colscale[j] = 2^p_j, the
// smallest power of two with max_r |F[r][j]| <= 448 2^p_j (1 for a zero
// column); round to nearest even. maxbits: KP unsigned of scratch. KP <= 128.
hipError_t pack_fp8_t(const float* F, int64_t rows, int KP, uint8_t* Ft, int64_t ldt,
                      float* colscale, unsigned* maxbits, hipStream_t st);

// Local updates on rows x KP row-major factors (leading dimension KP); k is
// the true rank, entries k..KP-1 are zero padding and stay zero.
// mu_rows and hals_rows write the updated rows of X to Xn (Xn == X: in
// place) and, when Xt is set (KP <= 64), their transpose Xt[i * rows + r] as
// well; P is summed from its slabs (mu_rows: Pout, nullable, receives the
// sum). Gslab (nullable, KP <= 64) receives the row blocks' shares of
// Xn^T Xn, one KP x KP slab per block of share_rows rows (cdiv(rows,
// share_rows) of them), for an ordered sum (reduce_splits).
// mu_rows' gn (KP <= 64 when above 1): G is given as gn KP x KP shares at
// stride KP * KP, which the update adds in order as it stages them.
template <typename T>
hipError_t mu_rows(const T* X, T* Xn, Split<T> P, const T* G, int64_t rows, int k, int KP, T eps,
                   T* Xt, T* Pout, T* Gslab, hipStream_t st, int gn = 1);
// hals_rows' Xs (nullable, KP entries): the incoming rows are scaled first,
// x_i *= Xs[i] where Xs[i] > 0 (the normalisation's compensation of H).
template <typename T>
hipError_t hals_rows(const T* X, T* Xn, Split<T> P, const T* G, int64_t rows, int k, int KP,
                     T* Xt, T* Gslab, hipStream_t st, const T* Xs = nullptr);
// Rows per block of an update's Gram shares (0: the update writes none at
// this KP): mu_rows at any row count, hals_rows at `rows` rows.
enum class ShareOf { MU, HALS };
int share_rows(ShareOf u, int64_t rows, int KP);
// Whether the update at `rows` rows takes a product's split slabs without
// losing occupancy (the HALS sweep's slab sums need registers that its
// many-row forms share out among more waves).
bool takes_slabs(ShareOf u, int64_t rows);
// The same shares of X^T X over blocks of rpb rows (a share_rows value) for
// a factor that no update produced (KP <= 64).
template <typename T>
hipError_t gram_shares(const T* X, int64_t rows, int KP, int rpb, T* Gslab, hipStream_t st);

// HALS normalisation: s_i = sqrt(S[i][i]); W[:, i] /= s_i, Ht[:, i] *= s_i and
// S[i][j] /= s_i s_j for s_i > 0. norms receives s. Wt (nullable, KP <= 64,
// m a multiple of 16 / sizeof(T)) receives the transpose of the rescaled W,
// Wt[i * m + r].
template <typename T>
hipError_t hals_normalize(const T* W, T* Wn, int64_t m, const T* Ht, T* Htn, int64_t n, T* S,
                          T* norms, int k, int KP, hipStream_t st, T* Wt = nullptr);

// Copies between the caller's layouts (ld = k) and the padded row layout.
template <typename T>
hipError_t pad_rows(const T* src, int64_t rows, int k, T* dst, int KP, hipStream_t st);
template <typename T>
hipError_t unpad_rows(const T* src, int64_t rows, int k, int KP, T* dst, hipStream_t st);
// At (n x m, row pitch ldt >= m) = A^T for A (m x n, lda). T is float,
// double, uint16_t (bfloat16 bits) or uint8_t (FP8 bits).
template <typename T>
hipError_t transpose_full(const T* A, int64_t lda, int64_t m, int64_t n, T* At, int64_t ldt,
                          hipStream_t st);
// src (rows x KP, row major) -> dst (KP x rows, row major), all KP rows.
template <typename T>
hipError_t transpose_rows(const T* src, int64_t rows, int KP, T* dst, hipStream_t st);
// H (k x n, ld n) -> Ht (n x KP) and back.
template <typename T>
hipError_t transpose_in(const T* H, int k, int64_t n, T* Ht, int KP, hipStream_t st);
template <typename T>
hipError_t transpose_out(const T* Ht, int k, int64_t n, int KP, T* H, hipStream_t st);

// Objective pieces. Each writes one double partial per block into `partial`
// (capacity given by *_partials) and a final reduce sums them in order.
template <typename T>
int64_t residual_partials(int64_t m, int64_t n);
// residual_sq: A is stored as TA (T, or with float factors uint16_t bfloat16
// bits or uint8_t FP8 E4M3 bits). sumsq and check_dense take all four.
template <typename T, typename TA = T>
hipError_t residual_sq(const TA* A, int64_t lda, int64_t m, int64_t n, const T* W, const T* Ht,
                       int KP, double* partial, hipStream_t st);
template <typename T>
int64_t sumsq_partials(int64_t m, int64_t n);
template <typename T>
hipError_t sumsq(const T* A, int64_t lda, int64_t m, int64_t n, double* partial,
                 hipStream_t st);
// Squares of the projected gradient of 1/2 ||A - W H||^2 in the factor whose
// rows are X (rows x KP): g = x G - p per row, kept where x > 0, negative part
// where x = 0; one double per block: pgrad_blocks<T>(rows, KP) of them, at
// most pgrad_partials(rows).
int64_t pgrad_partials(int64_t rows);
template <typename T>
int64_t pgrad_blocks(int64_t rows, int KP);
template <typename T>
hipError_t pgrad_sq(const T* X, const T* P, const T* G, int64_t rows, int k, int KP,
                    double* partial, hipStream_t st);
// out[slot] = sqrt(max(0, sum(partial[0..np)) + add) / ref) where add is the
// <G1, G2> Frobenius product of two KP x KP matrices (nullable) and ref the
// double at *ref_sq (nullable: out = the sum itself, no sqrt).
template <typename T>
hipError_t finish_relerr(const double* partial, int64_t np, const T* G1, const T* G2, int KP,
                         const double* ref_sq, double* out, hipStream_t st);

// Sparse (CSR, float32 values).
// Rows with more than a fixed number of stored entries (csr_long_rows, in
// scratch of csr_long_work_bytes(nnz, KP) bytes; synchronises the stream to
// read two counts) are computed in chunks by csr_spmm when lr describes them.
struct CsrLongRows {
  int64_t nlong = 0, nchunks = 0;
  const int64_t* ids = nullptr;        // the long rows
  const int64_t* chunk_off = nullptr;  // nlong + 1 chunk offsets
  float* part = nullptr;               // nchunks x KP partial sums
};
size_t csr_long_work_bytes(int64_t nnz, int KP);
hipError_t csr_long_rows(const int64_t* rowptr, int64_t m, int64_t nnz, int KP, void* work,
                         CsrLongRows* out, hipStream_t st);
// P (m x KP) = A F; lr nullable (then every row is one wave's work).
hipError_t csr_spmm(const int64_t* rowptr, const int32_t* colidx, const float* vals, int64_t m,
                    const float* F, int KP, float* P, const CsrLongRows* lr, hipStream_t st);
// `work` holds csr_transpose_work_bytes(m, n, nnz) bytes of scratch.
hipError_t csr_transpose(const int64_t* rowptr, const int32_t* colidx, const float* vals,
                         int64_t m, int64_t n, int64_t nnz, int64_t* rowptr_t,
                         int32_t* colidx_t, float* vals_t, void* work, hipStream_t st);
size_t csr_transpose_work_bytes(int64_t m, int64_t n, int64_t nnz);
int64_t csr_residual_partials(int64_t m);
hipError_t csr_residual_sq(const int64_t* rowptr, const int32_t* colidx, const float* vals,
                           int64_t m, const float* W, const float* Ht, int KP, double* partial,
                           hipStream_t st);
hipError_t csr_sumsq(const float* vals, int64_t nnz, double* partial, int64_t np,
                     hipStream_t st);
// Reverse mode through unrolled multiplicative updates (row layout, KP in
// {16, 32, 48, 64}). For Xn = X * N / (X G + eps), with the gradient reaching
// Xn taken as g = gXn + Y + Xn (M + M^T) (Y and M nullable: the terms that
// the next half-step's product and Gram pass back): gN = g * X / D,
// gD = -g * Xn / D, gX = g * N / D + gD G^T (D = X G + eps). Gt and Mt are
// the transposes of G and M (as the Gram's reduction writes them). gNt
// (nullable) receives gN transposed, gNt[i * rows + r].
// Gslab (nullable) receives the Gram gradient dL/dG = X^T gD as one KP x KP
// slab per row block (mu_adjoint_blocks of them), to be summed in order.
template <typename T>
hipError_t mu_adjoint_rows(const T* X, const T* Xn, const T* N, const T* G, const T* Gt,
                           const T* gXn, Split<T> Y, const T* M, const T* Mt, int64_t rows, int k,
                           int KP, T eps, T* gN, T* gNt, T* gD, T* gX, T* Gslab, hipStream_t st);
template <typename T>
int64_t mu_adjoint_blocks(int64_t rows, int KP);
// Reverse of the HALS sweep on rows x KP rows (KP in {16, 32, 48, 64}): from
// the sweep's output Xnew, the Gram G and gXnew = dL/dXnew, writes
// gXold = dL/dX (input) and Delta = dL/dP (one delta per row and column);
// Dt (nullable) receives Delta transposed, Dt[i * rows + r]. With Xold (the
// sweep's input) and Tslab set, the row blocks' shares of Xnew^T Delta and
// Xold^T Delta go to Tslab: hals_adjoint_blocks slabs of KP x KP each, then as
// many again, to be summed in order.
template <typename T>
hipError_t hals_adjoint_rows(const T* Xnew, const T* G, const T* gXnew, int64_t rows, int k,
                             int KP, T* gXold, T* Delta, T* Dt, const T* Xold, T* Tslab,
                             hipStream_t st);
template <typename T>
int64_t hals_adjoint_blocks(int64_t rows, int KP);
// M = S + S^T, S[a][b] = -(a <= b ? T1[a][b] : T2[a][b]) (the sweep's Gram
// gradient from T1 = Xnew^T Delta and T2 = Xold^T Delta, given as the nb
// per-block slabs of each that hals_adjoint_rows writes).
template <typename T>
hipError_t hals_gram_grad(const T* slabs, int nb, int KP, T* M, hipStream_t st);
// Column dot products of two pairs in one pass: out[c] = sum_r X1[r][c]
// Y1[r][c] over rows1 rows and out[KP + c] the same for X2, Y2 over rows2
// (double, fixed order); part holds coldot_partials(KP) doubles.
int64_t coldot_partials(int KP);
template <typename T>
hipError_t coldot2(const T* X1, const T* Y1, int64_t rows1, const T* X2, const T* Y2,
                   int64_t rows2, int KP, double* part, double* out, hipStream_t st);
// Adjoint of the HALS normalisation (Wn = W' / s, Hc = s H per column):
// gWp = dL/dW', gHt = dL/dH^T (pre-scaling) from gWn, gHc; dots[c] =
// <gWn_c, Wn_c>, dots[KP + c] = <gHc_c, Ht_c>.
template <typename T>
hipError_t hals_norm_adjoint(const T* gWn, const T* Wn, int64_t m, const T* gHc, int64_t n,
                             const T* norms, const double* dots, int k, int KP, T* gWp, T* gHt,
                             hipStream_t st);
// Out[r] = (Out[r] + Y[r]) + X[r] M (M KP x KP), columns < k; Y (a product's
// slabs) may be empty.
template <typename T>
hipError_t rowmm_add(const T* X, const T* M, int64_t rows, int k, int KP, T* Out,
                     hipStream_t st, Split<T> Y = Split<T>{nullptr, 0, 0});
// M = G + G^T.
template <typename T>
hipError_t symmetrize(const T* G, int KP, T* M, hipStream_t st);
// Y += X (n elements).
template <typename T>
hipError_t add_to(T* Y, const T* X, int64_t n, hipStream_t st);
// D (m x n, ldd) = beta D + sum_{t < L} (X1_t Y1_t^T + X2_t Y2_t^T), beta 0 or
// 1, with X*_t = X* + t m KP (m x KP) and Y*_t = Y* + t n KP (n x KP): the L
// rank-2KP terms of one checkpoint segment in one pass over D (X2 may be
// null).
template <typename T>
hipError_t rank_update(T* D, int64_t ldd, int64_t m, int64_t n, const T* X1, const T* Y1,
                       const T* X2, const T* Y2, int KP, int L, int beta, hipStream_t st);

// Input checks: sets *flag (device int) nonzero on a bad entry.
template <typename T>
hipError_t check_dense(const T* A, int64_t lda, int64_t m, int64_t n, int* flag,
                       hipStream_t st);
// flag bit 1: bad value; bit 2: bad structure (row bounds, column range or order).
hipError_t check_csr(const int64_t* rowptr, const int32_t* colidx, const float* vals, int64_t m,
                     int64_t n, int64_t nnz, int* flag, hipStream_t st);

// Batched NNLS by block principal pivoting: each row x of X (rows x KP)
// becomes argmin_{x>=0} 1/2 x^T G x - p^T x. With warm set, the support of
// the incoming row starts the pivoting. Ginv: KP*KP doubles of scratch,
// ginv_ok: one device int. status (device int) |= 1 on a singular system,
// |= 2 on pivot-cap exhaustion. pivots (device, BPP_TALLIES counters) adds
// up, over all right-hand sides: [BPP_T_PIVOTS] passive sets tried (the
// pivot cap counts these); [BPP_T_SOLVES] eliminations; [BPP_T_FLOPS] their
// algorithmic flops (ns^3 - ns for Gauss-Jordan on ns unknowns and one
// right-hand side, 2 k ns for the other half of the optimality pair, 2 k^2
// per right-hand side that forms G^-1 p); [BPP_T_SIZE] the sizes ns;
// [BPP_T_SIZE_MAX] the largest size of the same form in the wavefront at
// that elimination (the four right-hand sides of a wavefront eliminate
// together); [BPP_T_SIZE_CLASS] the size the elimination ran at.
enum { BPP_T_PIVOTS = 0, BPP_T_SOLVES, BPP_T_FLOPS, BPP_T_SIZE, BPP_T_SIZE_MAX,
       BPP_T_SIZE_CLASS, BPP_TALLIES = 8 };
template <typename T>
hipError_t bpp_rows_compact(T* X, const T* P, const T* G, int64_t rows, int k, int KP,
                            int max_pivots, int warm, double* Ginv, int* ginv_ok, int* status,
                            unsigned long long* pivots, hipStream_t st);

}  // namespace nmfk
