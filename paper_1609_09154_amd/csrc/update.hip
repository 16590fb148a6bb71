// Local update computations (LUC) of Algorithm 1 on the row layout: a row x
// of the factor being updated (a row of W, or a row of H^T, i.e. a column of
// H) is independent of every other row (Section 5: rows of W and columns of H
// can be updated in parallel). HALS gives each row a group of lanes that
// share the sequential sweep (each lane owns a slice of x; the dot product of
// every step is summed across the group with lane permutations); MU splits
// each row's outputs over several threads; both stage G in LDS.
//
//   MU   (Section 4.1, Eq. (3)):  x_i <- x_i p_i / ((x G)_i + eps), all i at once
//   HALS (Section 4.2, Eq. (5)):  i = 1..k in order, newest values:
//        x_i <- max(0, x_i + (p_i - (x G)_i) / G_ii)   (skipped if G_ii = 0)
//
// Padding entries k..KP-1 of x are zero on entry and stay zero.
#include "common.h"
#include "grid.h"
#include "rowtile.h"
#include "kernels.h"

namespace nmfk {

// HALS sweep with a group of TPR lanes per row: lane `sub` of a group owns
// entries sub*R .. sub*R + R - 1 of the row (R = KP / TPR) and the matching
// products. Step i forms (x G)_i from the owners' partial sums (group_sum,
// the same bits on every lane of the group) and the owner of entry i updates
// it. G is staged in LDS with column i contiguous (Gs[i][j] = G[j][i]), so a
// lane reads its R entries of the column with one vector load. Rows past the
// end run on a clamped copy of the last row (every lane must join the group
// sums) and store nothing. TPR (4, 8 or 16 lanes per row) is chosen from the
// number of rows: many rows fill the chip with small groups, which take fewer
// permutation steps per column; few rows need larger groups to fill it.
// With TILE (KP <= 64), after the sweep the LDS that held G takes the
// block's new rows (zero past the end) for their transposed copy (Xt,
// nullable) and the block's share of Xn^T Xn (Gslab + blockIdx.x * KP * KP,
// nullable), formed on the matrix cores. The tile shares G's space; only at
// 64 rows per block does its padding need more (17 KB against 16 KB at KP =
// 64), which the form without TILE, for calls that want neither output,
// does not take.
// Xs (nullable) scales the incoming rows first, x_i *= Xs[i] where Xs[i] > 0
// (the normalisation's compensation of H, applied as the sweep reads the rows
// rather than by a pass of its own; the same product, so the same bits).
template <typename T, int KP, int TPR, bool SLABS, bool TILE>
__global__ __launch_bounds__(256) void hals_rows_grp_kernel(const T* X, T* Xn, Split<T> P,
                                                            const T* __restrict__ G,
                                                            int64_t rows, int k,
                                                            T* __restrict__ Xt,
                                                            T* __restrict__ Gslab,
                                                            const T* __restrict__ Xscale) {
  constexpr int R = KP / TPR, ROWS = 256 / TPR;
  constexpr int VEC = Tr<T>::VEC;
  constexpr int XLD = KP + VEC;
  constexpr int TS = TILE && KP <= 64 ? ROWS * XLD : 0;
  constexpr int LS = KP * KP > TS ? KP * KP : TS;
  __shared__ __attribute__((aligned(16))) T Ls[LS];
  T* Gs = Ls;
  const int sub = threadIdx.x % TPR;
  const int64_t rb = (int64_t)blockIdx.x * ROWS;
  const int64_t r = rb + threadIdx.x / TPR;
  const int64_t rr = r < rows ? r : rows - 1;
  // G's loads, the row's x and its entries of P (summed from the slabs in
  // slab order in double), all in flight together
  SquareStage<T, KP, 256> gst;
  gst.load(G, nullptr);
  T x[R], p[R];
#pragma unroll
  for (int q = 0; q < R; ++q) x[q] = X[rr * KP + sub * R + q];
  if (Xscale) {
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const T sc = Xscale[sub * R + q];
      if (sc > T(0)) x[q] = x[q] * sc;
    }
  }
  if constexpr (SLABS) {
    double ps[R];
#pragma unroll
    for (int q = 0; q < R; ++q) ps[q] = 0.0;
    slab_sum<T, R>(P.p + rr * KP + sub * R, P.n, P.stride, ps);
#pragma unroll
    for (int q = 0; q < R; ++q) p[q] = (T)ps[q];
  } else {
    // one slab: the product itself (a sum of one term rounds to itself)
#pragma unroll
    for (int q = 0; q < R; ++q) p[q] = P.p[rr * KP + sub * R + q];
  }
  gst.store_t(Gs);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < KP; ++i) {
    if (i < k) {
      const T gii = Gs[i * KP + i];
      if (gii > T(0)) {
        const T* gc = &Gs[i * KP + sub * R];
        T part = T(0);
#pragma unroll
        for (int q = 0; q < R; ++q) part = fma(x[q], gc[q], part);
        const T s = group_sum<TPR>(part);
        if (sub == i / R) {
          const T t = x[i % R] + (p[i % R] - s) / gii;
          x[i % R] = t > T(0) ? t : T(0);
        }
      }
    }
  }
  if (r < rows) {
#pragma unroll
    for (int q = 0; q < R; ++q) Xn[r * KP + sub * R + q] = x[q];
  }
  if constexpr (TILE && KP <= 64) {
    if (Xt == nullptr && Gslab == nullptr) return;  // uniform over the block
    __syncthreads();  // every read of G is done
    const bool in = r < rows;
#pragma unroll
    for (int q = 0; q < R; ++q) Ls[(threadIdx.x / TPR) * XLD + sub * R + q] = in ? x[q] : T(0);
    __syncthreads();
    if (Gslab) block_gram_partial<T, KP, ROWS, XLD>(Ls, Ls, Gslab + (int64_t)blockIdx.x * KP * KP);
    if (Xt) store_rows_transposed<T, KP, ROWS, XLD>(Ls, rb, rows, Xt);
  }
}

// MU with several threads per row: the KP outputs of a row are split over
// TPR threads of RPT outputs each, and a block of 256 threads covers 256 / TPR
// rows. G and the block's rows of x are staged in LDS first (so an in-place
// update, Xn = X, reads nothing a lane has already written) and read with
// 16-byte loads. Xn receives every entry of the new rows (entries k..KP-1
// copied from X); Xt (nullable) receives their transpose, Xt[i * rows + r],
// the layout the next product reads the factor in, and Gslab (nullable) the
// block's share of Xn^T Xn, formed on the matrix cores from the same staged
// rows. P arrives as the product's slabs, summed here in slab order in double
// (Pout, nullable, receives the sum), so that a split product needs no pass
// of its own to add them.
template <int KP> struct RowSplit {
  static constexpr int TPR = KP == 48 ? 4 : KP / 8;
  static constexpr int RPT = KP / TPR;
  static constexpr int ROWS = 256 / TPR;
};

// GSUM: G arrives as gn KP x KP shares, summed while staged (in slab order
// in double, as the separate ordered sum would).
template <typename T, int KP, bool SLABS, bool GSUM>
__global__ __launch_bounds__(256) void mu_rows_tpr_kernel(const T* X, T* Xn, Split<T> P,
                                                          const T* __restrict__ G, int64_t rows,
                                                          int k, T eps, T* __restrict__ Xt,
                                                          T* __restrict__ Pout,
                                                          T* __restrict__ Gslab, int gn) {
  constexpr int TPR = RowSplit<KP>::TPR, RPT = RowSplit<KP>::RPT, ROWS = RowSplit<KP>::ROWS;
  constexpr int VEC = Tr<T>::VEC;
  static_assert(RPT % VEC == 0, "16-byte reads of G");
  constexpr int XLD = KP + VEC;
  __shared__ __attribute__((aligned(16))) T Gs[KP * KP];
  __shared__ __attribute__((aligned(16))) T Xs[ROWS * XLD];
  const int64_t rb = (int64_t)blockIdx.x * ROWS;
  const int lr = threadIdx.x / TPR;
  const int64_t r = rb + lr;
  const bool live = r < rows;
  const int i0 = (threadIdx.x % TPR) * RPT;
  // the staging loads, then the row's entries of P (independent of them),
  // all in flight together
  SquareStage<T, KP, 256> gst;
  RowStage<T, KP, ROWS, XLD, 256> xst;
  if constexpr (GSUM) gst.load_sum(G, gn, (int64_t)KP * KP);
  else gst.load(G, nullptr);
  xst.load(X, rb, rows);
  double ps[RPT];
#pragma unroll
  for (int ii = 0; ii < RPT; ++ii) ps[ii] = 0.0;
  if (live) {
    if constexpr (SLABS) {
      slab_sum<T, RPT>(P.p + r * KP + i0, P.n, P.stride, ps);
    } else {
      // one slab: the product itself (a sum of one term rounds to itself)
#pragma unroll
      for (int ii = 0; ii < RPT; ++ii) ps[ii] = (double)P.p[r * KP + i0 + ii];
    }
  }
  gst.store(Gs);
  xst.store(Xs, rb, rows);
  __syncthreads();
  const T* xs = &Xs[lr * XLD];
  T d[RPT];
#pragma unroll
  for (int ii = 0; ii < RPT; ++ii) d[ii] = T(0);
#pragma unroll 8
  for (int j = 0; j < KP; ++j) {
    const T xj = xs[j];
#pragma unroll
    for (int q = 0; q < RPT / VEC; ++q) {
      const V16<T> v = load16<T>(&Gs[j * KP + i0 + q * VEC]);
#pragma unroll
      for (int w = 0; w < VEC; ++w) d[q * VEC + w] = fma(xj, v.v[w], d[q * VEC + w]);
    }
  }
  T out[RPT];
#pragma unroll
  for (int ii = 0; ii < RPT; ++ii) out[ii] = xs[i0 + ii];
  if (live) {
#pragma unroll
    for (int ii = 0; ii < RPT; ++ii) {
      const int i = i0 + ii;
      const T pv = (T)ps[ii];
      if (Pout) Pout[r * KP + i] = pv;
      if (i < k) out[ii] = xs[i] * pv / (d[ii] + eps);
      Xn[r * KP + i] = out[ii];
    }
  }
  if (Xt == nullptr && Gslab == nullptr) return;  // uniform over the block
  __syncthreads();            // every read of the staged rows is done
#pragma unroll
  for (int ii = 0; ii < RPT; ++ii) Xs[lr * XLD + i0 + ii] = out[ii];
  __syncthreads();
  // the block's share of Xn^T Xn (rows past the end are zero)
  if (Gslab) block_gram_partial<T, KP, ROWS, XLD>(Xs, Xs, Gslab + (int64_t)blockIdx.x * KP * KP);
  if (Xt) store_rows_transposed<T, KP, ROWS, XLD>(Xs, rb, rows, Xt);
}

// The block's share of X^T X for the rows x KP factor X (slab blockIdx.x,
// KP x KP) over blocks of ROWS rows, staged and multiplied as the updates
// stage and multiply theirs (mu_rows_tpr_kernel, hals_rows_grp_kernel), so
// that either gives the same Gram after the ordered sum.
template <typename T, int KP, int ROWS>
__global__ __launch_bounds__(256) void gram_rows_kernel(const T* __restrict__ X, int64_t rows,
                                                        T* __restrict__ Gslab) {
  constexpr int XLD = KP + Tr<T>::VEC;
  __shared__ __attribute__((aligned(16))) T Xs[ROWS * XLD];
  const int64_t rb = (int64_t)blockIdx.x * ROWS;
  stage_rows<T, KP, ROWS, XLD, 256>(Xs, X, rb, rows);
  __syncthreads();
  block_gram_partial<T, KP, ROWS, XLD>(Xs, Xs, Gslab + (int64_t)blockIdx.x * KP * KP);
}

// MU at ranks above 64: each thread's row kept in LDS (column tid of a
// [KP][64] array, so accesses are bank-conflict free) and runtime loops,
// instead of fully unrolled register code. G is symmetric, so G[i*KP + j] is
// read along j with uniform loads.
constexpr int LDS_ROWS = 64;
template <typename T>
__global__ __launch_bounds__(LDS_ROWS) void mu_rows_lds_kernel(const T* X, T* Xn, Split<T> P,
                                                               const T* __restrict__ G,
                                                               int64_t rows, int k, int KP,
                                                               T eps, T* __restrict__ Pout) {
  __shared__ T xs[NMF_MAX_K * LDS_ROWS];
  const int t = threadIdx.x;
  const int64_t r = (int64_t)blockIdx.x * LDS_ROWS + t;
  if (r >= rows) return;  // no barriers below: each thread touches only its column
  for (int j = 0; j < KP; ++j) xs[j * LDS_ROWS + t] = X[r * KP + j];
  for (int i = 0; i < k; ++i) {
    T d = T(0);
    for (int j = 0; j < k; ++j) d = fma(xs[j * LDS_ROWS + t], G[i * KP + j], d);
    double ps = 0.0;
    for (int q = 0; q < P.n; ++q) ps += (double)P.p[q * P.stride + r * KP + i];
    const T pv = (T)ps;
    if (Pout) Pout[r * KP + i] = pv;
    Xn[r * KP + i] = xs[i * LDS_ROWS + t] * pv / (d + eps);
  }
  for (int i = k; i < KP; ++i) {
    if (Pout) Pout[r * KP + i] = T(0);
    Xn[r * KP + i] = xs[i * LDS_ROWS + t];
  }
}

#define KP_SWITCH(KPV, CALL, FALLBACK)                         \
  switch (KPV) {                                               \
    case 16: { constexpr int KPc = 16; CALL; } break;          \
    case 32: { constexpr int KPc = 32; CALL; } break;          \
    case 48: { constexpr int KPc = 48; CALL; } break;          \
    case 64: { constexpr int KPc = 64; CALL; } break;          \
    default:                                                   \
      if (KPV > NMF_MAX_K || KPV % 16) return hipErrorInvalidValue; \
      FALLBACK;                                                \
  }

// One slab (the product as it came) needs no double accumulation: that form
// keeps fewer registers live.
template <typename T, int KP, bool GSUM>
void launch_mu_rows_tpr_g(const T* X, T* Xn, Split<T> P, const T* G, int64_t rows, int k, T eps,
                          T* Xt, T* Pout, T* Gslab, int gn, hipStream_t st) {
  const unsigned nb = (unsigned)cdiv(rows, RowSplit<KP>::ROWS);
  if (P.n > 1)
    mu_rows_tpr_kernel<T, KP, true, GSUM><<<nb, 256, 0, st>>>(X, Xn, P, G, rows, k, eps, Xt,
                                                                Pout, Gslab, gn);
  else
    mu_rows_tpr_kernel<T, KP, false, GSUM><<<nb, 256, 0, st>>>(X, Xn, P, G, rows, k, eps, Xt,
                                                                 Pout, Gslab, gn);
}

template <typename T, int KP>
void launch_mu_rows_tpr(const T* X, T* Xn, Split<T> P, const T* G, int64_t rows, int k, T eps,
                        T* Xt, T* Pout, T* Gslab, int gn, hipStream_t st) {
  if (gn > 1) launch_mu_rows_tpr_g<T, KP, true>(X, Xn, P, G, rows, k, eps, Xt, Pout, Gslab, gn, st);
  else launch_mu_rows_tpr_g<T, KP, false>(X, Xn, P, G, rows, k, eps, Xt, Pout, Gslab, 1, st);
}

template <typename T>
hipError_t mu_rows(const T* X, T* Xn, Split<T> P, const T* G, int64_t rows, int k, int KP, T eps,
                   T* Xt, T* Pout, T* Gslab, hipStream_t st, int gn) {
  if (rows <= 0) return hipSuccess;
  if (((Xt || Gslab || gn > 1) && KP > 64) || !P.p || P.n < 1 || gn < 1)
    return hipErrorInvalidValue;
  KP_SWITCH(KP, (launch_mu_rows_tpr<T, KPc>(X, Xn, P, G, rows, k, eps, Xt, Pout, Gslab, gn, st)),
            (mu_rows_lds_kernel<T><<<(unsigned)cdiv(rows, LDS_ROWS), LDS_ROWS, 0, st>>>(
                X, Xn, P, G, rows, k, KP, eps, Pout)));
  return NMF_LAUNCH_CHECK();
}

static int hals_tpr(int64_t rows) { return rows >= 65536 ? 4 : (rows >= 16384 ? 8 : 16); }

bool takes_slabs(ShareOf u, int64_t rows) { return u == ShareOf::MU || hals_tpr(rows) == 16; }

int share_rows(ShareOf u, int64_t rows, int KP) {
  if (KP > 64 || KP % 16 || KP < 16) return 0;
  if (u == ShareOf::HALS) return 256 / hals_tpr(rows);
  switch (KP) {
    case 16: return RowSplit<16>::ROWS;
    case 32: return RowSplit<32>::ROWS;
    case 48: return RowSplit<48>::ROWS;
    default: return RowSplit<64>::ROWS;
  }
}

template <typename T, int KP>
static bool launch_gram_rows(const T* X, int64_t rows, int rpb, T* Gslab, hipStream_t st) {
  const unsigned nb = (unsigned)cdiv(rows, rpb);
  switch (rpb) {
    case 16: gram_rows_kernel<T, KP, 16><<<nb, 256, 0, st>>>(X, rows, Gslab); return true;
    case 32: gram_rows_kernel<T, KP, 32><<<nb, 256, 0, st>>>(X, rows, Gslab); return true;
    case 64: gram_rows_kernel<T, KP, 64><<<nb, 256, 0, st>>>(X, rows, Gslab); return true;
    case 128:
      if constexpr (KP == 16) {
        gram_rows_kernel<T, KP, 128><<<nb, 256, 0, st>>>(X, rows, Gslab);
        return true;
      }
      return false;
    default: return false;
  }
}

template <typename T>
hipError_t gram_shares(const T* X, int64_t rows, int KP, int rpb, T* Gslab, hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  bool ok = false;
  switch (KP) {
    case 16: ok = launch_gram_rows<T, 16>(X, rows, rpb, Gslab, st); break;
    case 32: ok = launch_gram_rows<T, 32>(X, rows, rpb, Gslab, st); break;
    case 48: ok = launch_gram_rows<T, 48>(X, rows, rpb, Gslab, st); break;
    case 64: ok = launch_gram_rows<T, 64>(X, rows, rpb, Gslab, st); break;
    default: break;
  }
  if (!ok) return hipErrorInvalidValue;
  return NMF_LAUNCH_CHECK();
}

template <typename T, int KP, bool SLABS, bool TILE>
void launch_hals_grp_t(const T* X, T* Xn, Split<T> P, const T* G, int64_t rows, int k, int tpr,
                       T* Xt, T* Gslab, const T* Xs, hipStream_t st) {
  if (tpr == 4)
    hals_rows_grp_kernel<T, KP, 4, SLABS, TILE><<<(unsigned)cdiv(rows, 64), 256, 0, st>>>(
        X, Xn, P, G, rows, k, Xt, Gslab, Xs);
  else if (tpr == 8)
    hals_rows_grp_kernel<T, KP, 8, SLABS, TILE><<<(unsigned)cdiv(rows, 32), 256, 0, st>>>(
        X, Xn, P, G, rows, k, Xt, Gslab, Xs);
  else
    hals_rows_grp_kernel<T, KP, 16, SLABS, TILE><<<(unsigned)cdiv(rows, 16), 256, 0, st>>>(
        X, Xn, P, G, rows, k, Xt, Gslab, Xs);
}

// One slab (the product as it came) needs no double accumulation: that form
// keeps the small register footprint that lets many blocks share a CU.
template <typename T, int KP>
void launch_hals_grp(const T* X, T* Xn, Split<T> P, const T* G, int64_t rows, int k, int tpr,
                     T* Xt, T* Gslab, const T* Xs, hipStream_t st) {
  if constexpr (KP <= 64) {
    if (Xt || Gslab) {
      if (P.n > 1)
        launch_hals_grp_t<T, KP, true, true>(X, Xn, P, G, rows, k, tpr, Xt, Gslab, Xs, st);
      else
        launch_hals_grp_t<T, KP, false, true>(X, Xn, P, G, rows, k, tpr, Xt, Gslab, Xs, st);
      return;
    }
  }
  if (P.n > 1) launch_hals_grp_t<T, KP, true, false>(X, Xn, P, G, rows, k, tpr, Xt, Gslab, Xs, st);
  else launch_hals_grp_t<T, KP, false, false>(X, Xn, P, G, rows, k, tpr, Xt, Gslab, Xs, st);
}

template <typename T>
hipError_t hals_rows(const T* X, T* Xn, Split<T> P, const T* G, int64_t rows, int k, int KP,
                     T* Xt, T* Gslab, hipStream_t st, const T* Xs) {
  if (rows <= 0) return hipSuccess;
  if (((Xt || Gslab) && KP > 64) || !P.p || P.n < 1) return hipErrorInvalidValue;
  const int tpr = hals_tpr(rows);
  // every padded rank up to NMF_MAX_K takes the grouped sweep; G (KP x KP)
  // is staged in LDS, at most 64 KB (float) or 128 KB (double) at KP = 128
  switch (KP) {
    case 16: launch_hals_grp<T, 16>(X, Xn, P, G, rows, k, tpr, Xt, Gslab, Xs, st); break;
    case 32: launch_hals_grp<T, 32>(X, Xn, P, G, rows, k, tpr, Xt, Gslab, Xs, st); break;
    case 48: launch_hals_grp<T, 48>(X, Xn, P, G, rows, k, tpr, Xt, Gslab, Xs, st); break;
    case 64: launch_hals_grp<T, 64>(X, Xn, P, G, rows, k, tpr, Xt, Gslab, Xs, st); break;
    case 80: launch_hals_grp<T, 80>(X, Xn, P, G, rows, k, tpr, Xt, Gslab, Xs, st); break;
    case 96: launch_hals_grp<T, 96>(X, Xn, P, G, rows, k, tpr, Xt, Gslab, Xs, st); break;
    case 112: launch_hals_grp<T, 112>(X, Xn, P, G, rows, k, tpr, Xt, Gslab, Xs, st); break;
    case 128: launch_hals_grp<T, 128>(X, Xn, P, G, rows, k, tpr, Xt, Gslab, Xs, st); break;
    default: return hipErrorInvalidValue;
  }
  return NMF_LAUNCH_CHECK();
}

// --- HALS normalisation ----------------------------------------------------
// One block: norms s_i = sqrt(S_ii) (0 if S_ii <= 0), then S <- D^-1 S D^-1
// on the entries whose norms are positive.
// The entries of S a thread rescales are loaded in batches of NB before any
// is written, so the block waits for one memory latency per batch rather
// than one per entry.
template <typename T>
__global__ void hals_norms_kernel(T* __restrict__ S, T* __restrict__ norms, int k, int KP) {
  constexpr int NB = 16;
  __shared__ double s_sh[NMF_MAX_K];
  for (int i = threadIdx.x; i < KP; i += blockDim.x) {
    const T d = S[i * KP + i];
    const double s = (i < k && d > T(0)) ? sqrt((double)d) : 0.0;
    s_sh[i] = s;
    norms[i] = (T)s;
  }
  __syncthreads();
  const int total = KP * KP, step = (int)blockDim.x;
  for (int e0 = threadIdx.x; e0 < total; e0 += NB * step) {
    T v[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int e = e0 + u * step;
      v[u] = S[e < total ? e : 0];
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int e = e0 + u * step;
      if (e < total) {
        const int i = e / KP, j = e - i * KP;
        const double si = s_sh[i], sj = s_sh[j];
        if (si > 0.0 && sj > 0.0) S[e] = (T)((double)v[u] / (si * sj));
      }
    }
  }
}

// Wn[:, i] = W[:, i] / s_i (rows 0..m-1), Htn[:, i] = Ht[:, i] * s_i (rows
// m..m+n-1 of the grid); columns with s_i = 0 (and the padding) are copied.
// Wn and Htn may be W and Ht. Each thread takes one 16-byte run of a row (KP
// is a multiple of 16, so runs never cross rows); in place, runs whose
// columns all keep their values (the padding, zero columns) are skipped.
template <typename T>
__global__ void hals_scale_kernel(const T* W, T* Wn, int64_t m, const T* Ht, T* Htn, int64_t n,
                                  const T* __restrict__ norms, int k, int KP) {
  constexpr int VEC = Tr<T>::VEC;
  const int CPR = KP / VEC;
  const int64_t total = (m + n) * CPR, stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int64_t r = e / CPR;
    const int i0 = (int)(e - r * CPR) * VEC;
    T s[VEC];
    bool any = false;
#pragma unroll
    for (int q = 0; q < VEC; ++q) {
      s[q] = i0 + q < k ? norms[i0 + q] : T(0);
      any = any || s[q] > T(0);
    }
    const bool w = r < m;
    const T* src = w ? W + r * KP + i0 : Ht + (r - m) * KP + i0;
    T* dst = w ? Wn + r * KP + i0 : Htn + (r - m) * KP + i0;
    if (!any && dst == src) continue;
    V16<T> v = load16<T>(src);
#pragma unroll
    for (int q = 0; q < VEC; ++q)
      if (s[q] > T(0)) v.v[q] = w ? v.v[q] / s[q] : v.v[q] * s[q];
    store16<T>(dst, v);
  }
}

// The same rescaling by tiles of SCALE_ROWS rows (W's tiles, then Ht's), for
// KP <= 64 with W's transposed copy: each tile of Wn also goes through LDS
// and out as Wt[i * m + r], the layout the next product reads, so that copy
// needs no launch of its own.
constexpr int SCALE_ROWS = 64;
template <typename T, int KP>
__global__ __launch_bounds__(256) void hals_scale_t_kernel(const T* W, T* Wn, int64_t m,
                                                           const T* Ht, T* Htn, int64_t n,
                                                           const T* __restrict__ norms, int k,
                                                           T* __restrict__ Wt) {
  constexpr int VEC = Tr<T>::VEC, CPR = KP / VEC, XLD = KP + VEC;
  __shared__ __attribute__((aligned(16))) T tile[SCALE_ROWS * XLD];
  const int64_t tw = cdiv(m, SCALE_ROWS), tt = tw + cdiv(n, SCALE_ROWS);
  for (int64_t tb = blockIdx.x; tb < tt; tb += gridDim.x) {
    const bool w = tb < tw;  // uniform over the block
    const int64_t rb = (w ? tb : tb - tw) * SCALE_ROWS, rows = w ? m : n;
    for (int e = threadIdx.x; e < SCALE_ROWS * CPR; e += blockDim.x) {
      const int q = e / CPR, i0 = (e % CPR) * VEC;
      const int64_t r = rb + q;
      if (r >= rows) continue;
      T s[VEC];
      bool any = false;
#pragma unroll
      for (int u = 0; u < VEC; ++u) {
        s[u] = i0 + u < k ? norms[i0 + u] : T(0);
        any = any || s[u] > T(0);
      }
      const T* src = (w ? W : Ht) + r * KP + i0;
      T* dst = (w ? Wn : Htn) + r * KP + i0;
      V16<T> v = load16<T>(src);
#pragma unroll
      for (int u = 0; u < VEC; ++u)
        if (s[u] > T(0)) v.v[u] = w ? v.v[u] / s[u] : v.v[u] * s[u];
      if (any || dst != src) store16<T>(dst, v);
      if (w) {
#pragma unroll
        for (int u = 0; u < VEC; ++u) tile[q * XLD + i0 + u] = v.v[u];
      }
    }
    if (w) {
      __syncthreads();
      store_rows_transposed<T, KP, SCALE_ROWS, XLD>(tile, rb, m, Wt);
      __syncthreads();  // the tile is rewritten by the block's next W tile
    }
  }
}

template <typename T>
hipError_t hals_normalize(const T* W, T* Wn, int64_t m, const T* Ht, T* Htn, int64_t n, T* S,
                          T* norms, int k, int KP, hipStream_t st, T* Wt) {
  hals_norms_kernel<T><<<1, 256, 0, st>>>(S, norms, k, KP);
  hipError_t e = NMF_LAUNCH_CHECK();
  if (e != hipSuccess) return e;
  const int64_t total = (m + n) * (KP / Tr<T>::VEC);
  if (total == 0) return hipSuccess;
  if (Wt) {
    const unsigned nb = capped_grid(cdiv(m, SCALE_ROWS) + cdiv(n, SCALE_ROWS));
    switch (KP) {
      case 16: hals_scale_t_kernel<T, 16><<<nb, 256, 0, st>>>(W, Wn, m, Ht, Htn, n, norms, k, Wt); break;
      case 32: hals_scale_t_kernel<T, 32><<<nb, 256, 0, st>>>(W, Wn, m, Ht, Htn, n, norms, k, Wt); break;
      case 48: hals_scale_t_kernel<T, 48><<<nb, 256, 0, st>>>(W, Wn, m, Ht, Htn, n, norms, k, Wt); break;
      case 64: hals_scale_t_kernel<T, 64><<<nb, 256, 0, st>>>(W, Wn, m, Ht, Htn, n, norms, k, Wt); break;
      default: return hipErrorInvalidValue;
    }
    return NMF_LAUNCH_CHECK();
  }
  hals_scale_kernel<T><<<capped_grid(cdiv(total, 256)), 256, 0, st>>>(W, Wn, m, Ht, Htn, n, norms,
                                                                      k, KP);
  return NMF_LAUNCH_CHECK();
}

// --- layout copies ---------------------------------------------------------
template <typename T>
__global__ void pad_rows_kernel(const T* __restrict__ src, int64_t rows, int k,
                                T* __restrict__ dst, int KP) {
  const int64_t total = rows * KP, stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int64_t r = e / KP;
    const int i = (int)(e - r * KP);
    dst[e] = i < k ? src[r * k + i] : T(0);
  }
}

template <typename T>
__global__ void unpad_rows_kernel(const T* __restrict__ src, int64_t rows, int k, int KP,
                                  T* __restrict__ dst) {
  const int64_t total = rows * k, stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int64_t r = e / k;
    const int i = (int)(e - r * k);
    dst[e] = src[r * KP + i];
  }
}

// Ht[j][i] = H[i][j] (i < k), 0 for k <= i < KP. Tiled through LDS.
template <typename T>
__global__ void transpose_in_kernel(const T* __restrict__ H, int k, int64_t n,
                                    T* __restrict__ Ht, int KP) {
  __shared__ T tile[32][33];
  const int64_t j0 = (int64_t)blockIdx.x * 32;
  const int i0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int yy = ty; yy < 32; yy += 8) {
    const int i = i0 + yy;
    const int64_t j = j0 + tx;
    tile[yy][tx] = (i < k && j < n) ? H[(int64_t)i * n + j] : T(0);
  }
  __syncthreads();
  for (int yy = ty; yy < 32; yy += 8) {
    const int64_t j = j0 + yy;
    const int i = i0 + tx;
    if (j < n && i < KP) Ht[j * KP + i] = tile[tx][yy];
  }
}

template <typename T>
__global__ void transpose_out_kernel(const T* __restrict__ Ht, int k, int64_t n, int KP,
                                     T* __restrict__ H) {
  __shared__ T tile[32][33];
  const int64_t j0 = (int64_t)blockIdx.x * 32;
  const int i0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int yy = ty; yy < 32; yy += 8) {
    const int64_t j = j0 + yy;
    const int i = i0 + tx;
    tile[tx][yy] = (j < n && i < k) ? Ht[j * KP + i] : T(0);
  }
  __syncthreads();
  for (int yy = ty; yy < 32; yy += 8) {
    const int i = i0 + yy;
    const int64_t j = j0 + tx;
    if (i < k && j < n) H[(int64_t)i * n + j] = tile[yy][tx];
  }
}

// Full transpose of a dense matrix (A, m x n, lda) into At (n x m, ld m),
// 64 x 64 tiles through LDS so both the reads and the writes are 256-byte
// row segments. With vec set (16-byte aligned A and At, lda and ldt
// multiples of the 16-byte element count) a tile that lies wholly inside the
// matrix moves as 16-byte runs both ways: each lane reads one run of a row of
// A, and writes one run of a row of At gathered from the tile's column.
template <typename T>
__global__ __launch_bounds__(256) void transpose_full_kernel(const T* __restrict__ A,
                                                             int64_t lda, int64_t m, int64_t n,
                                                             T* __restrict__ At, int64_t ldt,
                                                             int vec) {
  __shared__ T tile[64][65];
  const int64_t c0 = (int64_t)blockIdx.x * 64, r0 = (int64_t)blockIdx.y * 64;
  if constexpr (sizeof(T) >= 4) {
  constexpr int VEC = Tr<T>::VEC;        // elements per 16 bytes
  constexpr int CPR = 64 / VEC;          // 16-byte runs per 64-element row
  constexpr int RPP = 256 / CPR;         // rows per pass
  if (vec && r0 + 64 <= m && c0 + 64 <= n) {
    const int q = threadIdx.x % CPR, rr = threadIdx.x / CPR;
#pragma unroll
    for (int i = rr; i < 64; i += RPP) {
      const V16<T> v = load16_stream<T>(A + (r0 + i) * lda + c0 + VEC * q);
#pragma unroll
      for (int e = 0; e < VEC; ++e) tile[i][VEC * q + e] = v.v[e];
    }
    __syncthreads();
#pragma unroll
    for (int i = rr; i < 64; i += RPP) {
      T* dst = At + (c0 + i) * ldt + r0 + VEC * q;
      if constexpr (sizeof(T) == 4) {
        *reinterpret_cast<float4*>(dst) = make_float4(tile[4 * q][i], tile[4 * q + 1][i],
                                                      tile[4 * q + 2][i], tile[4 * q + 3][i]);
      } else {
        *reinterpret_cast<double2*>(dst) = make_double2(tile[2 * q][i], tile[2 * q + 1][i]);
      }
    }
    return;
  }
  }
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int i = ty; i < 64; i += 4) {
    const int64_t r = r0 + i, c = c0 + tx;
    tile[i][tx] = (r < m && c < n) ? __builtin_nontemporal_load(A + r * lda + c) : T(0);
  }
  __syncthreads();
  for (int i = ty; i < 64; i += 4) {
    const int64_t c = c0 + i, r = r0 + tx;
    if (c < n && r < m) At[c * ldt + r] = tile[tx][i];
  }
}

// Byte and 16-bit matrices (FP8 and bfloat16 A) move 4-byte words both
// ways: a TR x 128 tile (TR = 128 rows for bytes, 64 for 16-bit elements, so
// that every output word run is 128 bytes and the tile stays near 16 KB of
// LDS) is read as whole words of each row and written as whole words of each
// output row, an output word gathering one element from each of
// 4 / sizeof(T) consecutive input rows. Needs lda, ldt and n multiples of the
// elements per word and 4-byte aligned pointers, so that a word read at a
// column below n and a word written at a row below m stay inside the row
// pitches.
template <typename T> struct WordTile {
  static constexpr int EPW = 4 / (int)sizeof(T);   // elements per word
  static constexpr int TR = 32 * EPW;              // tile rows
};
template <typename T>
__global__ __launch_bounds__(256) void transpose_words_kernel(const T* __restrict__ A,
                                                              int64_t lda, int64_t m, int64_t n,
                                                              T* __restrict__ At, int64_t ldt) {
  constexpr int EPW = WordTile<T>::EPW;
  constexpr int TR = WordTile<T>::TR;
  constexpr int WPR = 128 / EPW;            // words per tile row (128 columns)
  constexpr int RPP = 256 / WPR;            // tile rows read per pass
  constexpr int OW = TR / EPW;              // words per output row (32)
  constexpr int OPP = 256 / OW;             // output rows written per pass
  constexpr int EB = 8 * (int)sizeof(T);    // bits per element
  constexpr uint32_t MASK = (1u << EB) - 1u;
  __shared__ uint32_t tile[TR][WPR + 1];
  const int64_t c0 = (int64_t)blockIdx.x * 128, r0 = (int64_t)blockIdx.y * TR;
  {
    const int tx = threadIdx.x % WPR, ty = threadIdx.x / WPR;
    for (int i = ty; i < TR; i += RPP) {
      const int64_t r = r0 + i, c = c0 + EPW * tx;
      tile[i][tx] = (r < m && c < n) ? __builtin_nontemporal_load(
                                           reinterpret_cast<const uint32_t*>(A + r * lda + c))
                                     : 0u;
    }
  }
  __syncthreads();
  const int ox = threadIdx.x % OW, oy = threadIdx.x / OW;
  for (int j = oy; j < 128; j += OPP) {
    const int64_t c = c0 + j, r = r0 + EPW * ox;
    if (c < n && r < m) {
      const int w = j / EPW, sh = EB * (j % EPW);
      uint32_t out = 0;
#pragma unroll
      for (int b = 0; b < EPW; ++b) out |= ((tile[EPW * ox + b][w] >> sh) & MASK) << (EB * b);
      *reinterpret_cast<uint32_t*>(At + c * ldt + r) = out;
    }
  }
}

template <typename T>
hipError_t transpose_full(const T* A, int64_t lda, int64_t m, int64_t n, T* At, int64_t ldt,
                          hipStream_t st) {
  if constexpr (sizeof(T) < 4) {
    constexpr int EPW = 4 / (int)sizeof(T);
    if (lda % EPW == 0 && ldt % EPW == 0 && n % EPW == 0 && (uintptr_t)A % 4 == 0 &&
        (uintptr_t)At % 4 == 0) {
      dim3 grid((unsigned)cdiv(n, 128), (unsigned)cdiv(m, WordTile<T>::TR));
      transpose_words_kernel<T><<<grid, 256, 0, st>>>(A, lda, m, n, At, ldt);
      return NMF_LAUNCH_CHECK();
    }
  }
  constexpr int VEC = 16 / (int)sizeof(T);
  const int vec = sizeof(T) >= 4 && lda % VEC == 0 && ldt % VEC == 0 &&
                  (uintptr_t)A % 16 == 0 && (uintptr_t)At % 16 == 0;
  dim3 grid((unsigned)cdiv(n, 64), (unsigned)cdiv(m, 64));
  transpose_full_kernel<T><<<grid, 256, 0, st>>>(A, lda, m, n, At, ldt, vec);
  return NMF_LAUNCH_CHECK();
}

template <typename T>
hipError_t transpose_rows(const T* src, int64_t rows, int KP, T* dst, hipStream_t st) {
  dim3 grid((unsigned)cdiv(rows, 32), (unsigned)cdiv(KP, 32));
  transpose_out_kernel<T><<<grid, 256, 0, st>>>(src, KP, rows, KP, dst);
  return NMF_LAUNCH_CHECK();
}

template <typename T>
hipError_t pad_rows(const T* src, int64_t rows, int k, T* dst, int KP, hipStream_t st) {
  const int64_t total = rows * KP;
  if (total == 0) return hipSuccess;
  pad_rows_kernel<T><<<capped_grid(cdiv(total, 256)), 256, 0, st>>>(src, rows, k, dst, KP);
  return NMF_LAUNCH_CHECK();
}

template <typename T>
hipError_t unpad_rows(const T* src, int64_t rows, int k, int KP, T* dst, hipStream_t st) {
  const int64_t total = rows * k;
  if (total == 0) return hipSuccess;
  unpad_rows_kernel<T><<<capped_grid(cdiv(total, 256)), 256, 0, st>>>(src, rows, k, KP, dst);
  return NMF_LAUNCH_CHECK();
}

template <typename T>
hipError_t transpose_in(const T* H, int k, int64_t n, T* Ht, int KP, hipStream_t st) {
  dim3 grid((unsigned)cdiv(n, 32), (unsigned)cdiv(KP, 32));
  transpose_in_kernel<T><<<grid, 256, 0, st>>>(H, k, n, Ht, KP);
  return NMF_LAUNCH_CHECK();
}

template <typename T>
hipError_t transpose_out(const T* Ht, int k, int64_t n, int KP, T* H, hipStream_t st) {
  dim3 grid((unsigned)cdiv(n, 32), (unsigned)cdiv(k, 32));
  transpose_out_kernel<T><<<grid, 256, 0, st>>>(Ht, k, n, KP, H);
  return NMF_LAUNCH_CHECK();
}

#define INST(T)                                                                             \
  template hipError_t mu_rows<T>(const T*, T*, Split<T>, const T*, int64_t, int, int, T, T*, \
                                 T*, T*, hipStream_t, int); \
  template hipError_t gram_shares<T>(const T*, int64_t, int, int, T*, hipStream_t); \
  template hipError_t hals_rows<T>(const T*, T*, Split<T>, const T*, int64_t, int, int, T*, \
                                   T*, hipStream_t, const T*);                              \
  template hipError_t hals_normalize<T>(const T*, T*, int64_t, const T*, T*, int64_t, T*, T*, \
                                        int, int, hipStream_t, T*);                         \
  template hipError_t pad_rows<T>(const T*, int64_t, int, T*, int, hipStream_t);            \
  template hipError_t unpad_rows<T>(const T*, int64_t, int, int, T*, hipStream_t);          \
  template hipError_t transpose_in<T>(const T*, int, int64_t, T*, int, hipStream_t);        \
  template hipError_t transpose_out<T>(const T*, int, int64_t, int, T*, hipStream_t);         \
  template hipError_t transpose_rows<T>(const T*, int64_t, int, T*, hipStream_t);            \
  template hipError_t transpose_full<T>(const T*, int64_t, int64_t, int64_t, T*, int64_t,      \
                                        hipStream_t);
INST(float)
INST(double)
#undef INST
template hipError_t transpose_full<uint16_t>(const uint16_t*, int64_t, int64_t, int64_t,
                                             uint16_t*, int64_t, hipStream_t);
template hipError_t transpose_full<uint8_t>(const uint8_t*, int64_t, int64_t, int64_t, uint8_t*,
                                            int64_t, hipStream_t);

}  // namespace nmfk
