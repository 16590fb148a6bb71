// Batched nonnegative least squares by block principal pivoting (Section 4.3,
// Eqs. (6)-(7)): for every row p of P solve
//     min_{x >= 0} 1/2 x^T G x - p^T x,    y = G x - p,
// until x_F >= 0 and y off F >= 0 (F the passive set). All right-hand sides
// share G (the Gram of the fixed factor), so one launch covers all of them:
// one wavefront per right-hand side, lane i <-> index i (k <= 64), the
// passive set a 64-bit mask and the infeasible set a ballot.
//
// The exchange rule is Kim and Park's (the method the paper cites): swap all
// of V while |V| keeps falling, at most three times without progress, then
// only the largest index of V. Factorisation, solves and sign tests run in
// double for every storage type: with float arithmetic, rounding noise on
// entries whose exact value is zero flips their sign from one pivot to the
// next and the pivoting can cycle. A non-positive pivot sets status |= 1;
// reaching the pivot cap sets status |= 2.
#include "common.h"
#include "kernels.h"


// ===========================================================================
// Compact solver. The passive-set system only involves the |F| indices of F,
// and the KKT conditions give an equivalent system on the active set A:
//     y = G x - p,  x_A = 0,  y_F = 0   =>   x = G^-1 (p + y),
//     (G^-1)_AA y_A = -(G^-1 p)_A,       x_F = (G^-1 p)_F + (G^-1)_FA y_A.
// With k <= 64 one of |F|, |A| is at most 32, so each solve eliminates at
// most 32 pivots. The solved set S (F, or A) is moved to lanes 0..|S|-1 and
// the other indices to the lanes after it (one cross-lane permute); every
// lane c holds row c of [M_{.,S} | rhs] in double registers, and Gauss-Jordan
// elimination over the pivots of S (pivot rows broadcast with readlane)
// leaves the solution on S in lanes c < |S| and, in the other lanes, the
// right-hand side with S eliminated: p - G_{.F} x_F = -y for the passive
// system; for the active one, with right-hand side G^-1 p, the solution on
// A is -y_A and the other lanes hold x_F. So one elimination gives both halves of
// the KKT pair, with no LDS traffic and no waits inside the solve. Each
// right-hand side starts from the support of the incoming X (warm start);
// the solution is unique, so the start only changes how many exchanges are
// needed.
// ===========================================================================
namespace nmfk {

constexpr int BPP_WAVES = 4;   // right-hand sides in flight per workgroup
constexpr int CNF = 32;        // largest eliminated set

__device__ __forceinline__ double rdl(double v, int q) {
  const unsigned long long b = __double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_readlane((unsigned)(b & 0xffffffffu), q);
  const unsigned hi = __builtin_amdgcn_readlane((unsigned)(b >> 32), q);
  return __longlong_as_double(((unsigned long long)hi << 32) | lo);
}

// v from lane `src` (any lane, per-lane source).
__device__ __forceinline__ double pull(double v, int src) {
  const unsigned long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_ds_bpermute(src << 2, (int)(unsigned)(b & 0xffffffffu));
  const int hi = __builtin_amdgcn_ds_bpermute(src << 2, (int)(unsigned)(b >> 32));
  return __longlong_as_double(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Gauss-Jordan elimination of the first ns <= NS columns (lane c holds row c
// of the matrix in a[] and its right-hand side b): returns the solution in
// lanes c < ns and the eliminated right-hand side in the other lanes; a
// non-positive pivot sets bad. Columns ns..NS-1 hold zeros, so the column
// loops need no bounds tests.
template <int NS>
__device__ __forceinline__ double gj_eliminate(double (&a)[CNF], double b, int ns, int lane,
                                               bool& bad) {
  double dq = 1.0;
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    if (q < ns) {
      double pv = rdl(a[q], q);
      if (!(pv > 0.0)) { bad = true; pv = 1.0; }
      const double f = (lane == q) ? 0.0 : a[q] / pv;
      if (lane == q) dq = pv;
      b = fma(-f, rdl(b, q), b);
#pragma unroll
      for (int j = q + 1; j < NS; ++j) a[j] = fma(-f, rdl(a[j], q), a[j]);
    }
  }
  return lane < ns ? b / dq : b;
}

// Ginv (KP x KP, double) = inverse of G restricted to the indices i < k with
// G_ii > 0 (zero rows and columns elsewhere), by Gauss-Jordan elimination in
// double with one workgroup; *ok = 0 when a pivot of that block is not
// positive (the block is not numerically positive definite). An index with
// G_ii = 0 belongs to a zero column of the fixed factor: its right-hand side
// entry is exactly 0 too, so it stays active with x_i = y_i = 0.
template <typename TS, int KP>
__global__ __launch_bounds__(256) void gram_inverse_kernel(const TS* __restrict__ G, int k,
                                                           double* __restrict__ Ginv,
                                                           int* __restrict__ ok) {
  __shared__ double M[KP][2 * KP + 1];
  __shared__ double piv;
  const int t = threadIdx.x;
  for (int e = t; e < KP * 2 * KP; e += blockDim.x) {
    const int i = e / (2 * KP), j = e % (2 * KP);
    const bool li = i < k && G[i * KP + i] > TS(0);
    const bool lj = (j % KP) < k && G[(j % KP) * KP + (j % KP)] > TS(0);
    double v = 0.0;
    if (j < KP) v = (li && lj) ? (double)G[i * KP + j] : (i == j ? 1.0 : 0.0);
    else v = (j - KP == i) ? 1.0 : 0.0;
    M[i][j] = v;
  }
  __syncthreads();
  int good = 1;
  for (int q = 0; q < k; ++q) {
    if (t == 0) piv = M[q][q];
    __syncthreads();
    const double pv = piv;
    if (!(pv > 0.0)) { good = 0; break; }
    for (int j = t; j < 2 * KP; j += blockDim.x) M[q][j] /= pv;
    __syncthreads();
    for (int e = t; e < KP * 2 * KP; e += blockDim.x) {
      const int i = e / (2 * KP), j = e % (2 * KP);
      if (i != q) {
        const double f = M[i][q];
        if (j != q) M[i][j] = fma(-f, M[q][j], M[i][j]);
      }
    }
    __syncthreads();
    for (int i = t; i < KP; i += blockDim.x)
      if (i != q) M[i][q] = 0.0;
    __syncthreads();
  }
  for (int e = t; e < KP * KP; e += blockDim.x) {
    const int i = e / KP, j = e % KP;
    const bool li = i < k && G[i * KP + i] > TS(0);
    const bool lj = j < k && G[j * KP + j] > TS(0);
    Ginv[e] = (li && lj) ? M[i][KP + j] : 0.0;
  }
  if (t == 0) *ok = good;
}

template <typename TS, int KP>
__global__ __launch_bounds__(64 * BPP_WAVES) void bpp_compact_kernel(
    TS* __restrict__ X, const TS* __restrict__ P, const TS* __restrict__ G,
    const double* __restrict__ Ginv, const int* __restrict__ ginv_ok, int64_t rows, int k,
    int max_pivots, int warm, int* __restrict__ status, unsigned long long* __restrict__ pivots) {
  static_assert(KP <= 64, "one lane per index");
  constexpr int LD = KP + 1;
  __shared__ TS Gs[KP * LD];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int e = threadIdx.x; e < KP * KP; e += blockDim.x) Gs[(e / KP) * LD + (e % KP)] = G[e];
  __syncthreads();
  // live: index in range with a nonzero Gram diagonal (see gram_inverse_kernel)
  const bool act = lane < k && Gs[lane * LD + lane] > TS(0);
  const uint64_t all = __ballot(act);
  const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const bool have_ginv = k > CNF && *ginv_ok != 0;
  unsigned long long my_pivots = 0;
  int my_status = 0;

  for (int64_t r = (int64_t)blockIdx.x * BPP_WAVES + wv; r < rows;
       r += (int64_t)gridDim.x * BPP_WAVES) {
    const double p = (lane < k) ? (double)P[r * KP + lane] : 0.0;
    uint64_t F = 0;
    if (warm) F = __ballot(act && X[r * KP + lane] > TS(0)) & all;
    double x = 0.0, y = -p, cp = 0.0;
    bool have_cp = false, bad = false;
    int budget = 3, best = k + 1, npiv = 0;
    bool first = F != 0;  // the warm-start set is solved before any test
    const bool from_warm = first;
    for (;;) {
      if (!first) {
        const bool inF = (F >> lane) & 1ull;
        const bool infeas = act && (inF ? (x < 0.0) : (y < 0.0));
        const uint64_t V = __ballot(infeas);
        if (V == 0) break;
        if (npiv >= max_pivots) { my_status |= 2; break; }
        const int nv = __popcll(V);
        uint64_t E;
        if (nv < best) { best = nv; budget = 3; E = V; }
        else if (budget >= 1) { --budget; E = V; }
        else { E = 1ull << (63 - __clzll(V)); }
        F ^= E;
      }
      first = false;
      ++npiv;
      const int nf = __popcll(F);
      const bool fi = (F >> lane) & 1ull;
      if (nf == 0) { x = 0.0; y = -p; continue; }
      const bool passive = nf <= CNF;
      if (!passive && !have_ginv) { bad = true; break; }  // G^-1 unavailable (G singular)
      if (!passive && !have_cp) {
        // cp = G^-1 p, once per right-hand side
        double s = 0.0;
        const int grow = act ? lane : 0;
        for (int j = 0; j < k; ++j) s = fma(Ginv[grow * KP + j], rdl(p, j), s);
        cp = act ? s : 0.0;
        have_cp = true;
      }
      const uint64_t S = passive ? F : (all & ~F);
      const int ns = __popcll(S);
      const bool si = (S >> lane) & 1ull;
      // compact position: S in increasing index order, then the other lanes
      const int pos = si ? __popcll(S & below) : ns + __popcll(~S & below);
      const int ci0 = __builtin_amdgcn_ds_permute(pos << 2, lane);  // index held by lane
      const int ci = ci0 < k ? ci0 : 0;
      const double bv = pull(passive ? p : cp, ci0);
      const double b = bv;
      double a[CNF];
      uint64_t bits = S;
#pragma unroll
      for (int d = 0; d < CNF; ++d) {
        double v = 0.0;
        if (d < ns) {
          const int j = __builtin_ctzll(bits);
          bits &= bits - 1;
          v = passive ? (double)Gs[ci * LD + j] : Ginv[ci * KP + j];
        }
        a[d] = v;
      }
      double sol;
      switch ((ns + 7) >> 3) {
        case 1: sol = gj_eliminate<8>(a, b, ns, lane, bad); break;
        case 2: sol = gj_eliminate<16>(a, b, ns, lane, bad); break;
        case 3: sol = gj_eliminate<24>(a, b, ns, lane, bad); break;
        default: sol = gj_eliminate<32>(a, b, ns, lane, bad); break;
      }
      if (bad && npiv == 1 && from_warm) {
        // The warm-start set was not positive definite: start over from F = {}.
        bad = false;
        F = 0;
        x = 0.0;
        y = -p;
        continue;
      }
      if (bad) break;
      const double val = pull(sol, pos);
      if (passive) {
        x = fi ? val : 0.0;
        y = (fi || !act) ? 0.0 : -val;
      } else {
        // (G^-1)_AA z = (G^-1 p)_A gives z = -y_A; the other lanes hold
        // (G^-1 p)_F - (G^-1)_FA z = x_F
        y = si ? -val : 0.0;
        x = fi ? val : 0.0;
      }
    }
    if (bad) my_status |= 1;
    my_pivots += (unsigned long long)npiv;
    if (lane < KP) X[r * KP + lane] = (lane < k) ? (TS)(x > 0.0 ? x : 0.0) : TS(0);
  }
  if (lane == 0) {
    atomicAdd(pivots, my_pivots);
    if (my_status) atomicOr(status, my_status);
  }
}

template <typename T>
hipError_t bpp_rows_compact(T* X, const T* P, const T* G, int64_t rows, int k, int KP,
                            int max_pivots, int warm, double* Ginv, int* ginv_ok, int* status,
                            unsigned long long* pivots, hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  const int64_t maxb = 256 * 16;
  const unsigned blocks = (unsigned)std::min<int64_t>(maxb, cdiv(rows, BPP_WAVES));
#define CASE(K)                                                                          \
  case K:                                                                                \
    if (k > CNF) gram_inverse_kernel<T, K><<<1, 256, 0, st>>>(G, k, Ginv, ginv_ok);      \
    bpp_compact_kernel<T, K><<<blocks, 64 * BPP_WAVES, 0, st>>>(                         \
        X, P, G, Ginv, ginv_ok, rows, k, max_pivots, warm, status, pivots);              \
    break;
  switch (KP) {
    CASE(16) CASE(32) CASE(48) CASE(64)
    default: return hipErrorInvalidValue;
  }
#undef CASE
  return NMF_LAUNCH_CHECK();
}

template hipError_t bpp_rows_compact<float>(float*, const float*, const float*, int64_t, int, int,
                                            int, int, double*, int*, int*, unsigned long long*,
                                            hipStream_t);
template hipError_t bpp_rows_compact<double>(double*, const double*, const double*, int64_t, int,
                                             int, int, int, double*, int*, int*,
                                             unsigned long long*, hipStream_t);

}  // namespace nmfk
