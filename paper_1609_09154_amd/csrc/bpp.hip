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
// With k <= 64 one of |F|, |A| is at most 32, so every factorisation here is
// at most 32 x 32: lane c holds compact row c in double registers, pivots are
// broadcast with readlane, each factor column goes through LDS once, and L is
// transposed through LDS for the backward solve. Each right-hand side starts
// from the support of the incoming X (warm start); the solution is unique, so
// the start only changes how many exchanges are needed.
// ===========================================================================
namespace nmfk {

constexpr int BPP_WAVES = 4;   // right-hand sides in flight per workgroup
constexpr int CNF = 32;        // largest compact system
constexpr int CLD = CNF + 1;

__device__ __forceinline__ double rdl(double v, int q) {
  const unsigned long long b = __double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_readlane((unsigned)(b & 0xffffffffu), q);
  const unsigned hi = __builtin_amdgcn_readlane((unsigned)(b >> 32), q);
  return __longlong_as_double(((unsigned long long)hi << 32) | lo);
}

// Orders this wave's LDS writes before its later reads (lanes read what
// other lanes of the same wave wrote).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Solves M s = b for the ns x ns SPD matrix whose row `lane` is in a[]
// (lanes >= ns and columns >= ns are ignored). Returns s in lane c < ns and
// sets *bad on a non-positive pivot. bw: 64 doubles of LDS, Lw: CNF x CLD.
__device__ __forceinline__ double chol_solve(double (&a)[CNF], double b, int ns, int lane,
                                             double* bw, double* Lw, bool* bad) {
  double dd = 1.0;
#pragma unroll
  for (int q = 0; q < CNF; ++q) {
    if (q < ns) {
      double d = rdl(a[q], q);
      if (!(d > 0.0)) { *bad = true; d = 1.0; }
      const double inv = 1.0 / sqrt(d);
      const double l = a[q] * inv;
      a[q] = lane >= q ? l : 0.0;
      if (lane == q) dd = inv;
      const double lq = (lane > q && lane < ns) ? l : 0.0;
      bw[lane] = lq;
      wave_sync();
#pragma unroll
      for (int j = q + 1; j < CNF; ++j)
        if (j < ns) a[j] = fma(-lq, bw[j], a[j]);
      wave_sync();
    }
  }
  if (lane < CNF) {
#pragma unroll
    for (int j = 0; j < CNF; ++j) Lw[lane * CLD + j] = a[j];
  }
  wave_sync();
  // forward: L z = b
  double rz = b, z = 0.0;
#pragma unroll
  for (int q = 0; q < CNF; ++q) {
    if (q < ns) {
      const double zq = rdl(rz, q) * rdl(dd, q);
      if (lane == q) z = zq;
      rz = fma(-a[q], zq, rz);
    }
  }
  // backward: L^T s = z (lane c reads column c of L from LDS)
  double rs = z, s = 0.0;
#pragma unroll
  for (int q = CNF - 1; q >= 0; --q) {
    if (q < ns) {
      const double sq = rdl(rs, q) * rdl(dd, q);
      if (lane == q) s = sq;
      const double lqc = lane < CNF ? Lw[q * CLD + lane] : 0.0;
      rs = fma(-lqc, sq, rs);
    }
  }
  wave_sync();
  return s;
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
  __shared__ double Ls[BPP_WAVES][CNF * CLD];
  __shared__ double Bs[BPP_WAVES][64];
  __shared__ double Xs[BPP_WAVES][64];
  __shared__ int Is[BPP_WAVES][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int e = threadIdx.x; e < KP * KP; e += blockDim.x) Gs[(e / KP) * LD + (e % KP)] = G[e];
  __syncthreads();
  double* bw = Bs[wv];
  double* xw = Xs[wv];
  double* Lw = Ls[wv];
  int* iw = Is[wv];
  // live: index in range with a nonzero Gram diagonal (see gram_inverse_kernel)
  const bool act = lane < k && Gs[lane * LD + lane] > TS(0);
  const uint64_t all = __ballot(act);
  const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
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
      if (!passive && !*ginv_ok) { bad = true; break; }  // G^-1 unavailable (G singular)
      if (!passive && !have_cp) {
        // cp = G^-1 p, once per right-hand side
        xw[lane] = p;
        wave_sync();
        double s = 0.0;
        if (act)
          for (int j = 0; j < k; ++j) s = fma(Ginv[j * KP + lane], xw[j], s);
        cp = s;
        have_cp = true;
        wave_sync();
      }
      const uint64_t Sset = passive ? F : (all & ~F);
      const int ns = __popcll(Sset);
      const bool si = (Sset >> lane) & 1ull;
      const int rank = __popcll(Sset & below);
      if (si) iw[rank] = lane;
      xw[lane] = passive ? p : cp;
      wave_sync();
      const int ci = lane < ns ? iw[lane] : 0;
      double a[CNF];
#pragma unroll
      for (int d = 0; d < CNF; ++d) {
        double v = (lane == d) ? 1.0 : 0.0;
        if (d < ns) {
          const int j = iw[d];
          if (lane < ns) v = passive ? (double)Gs[ci * LD + j] : Ginv[ci * KP + j];
        }
        a[d] = v;
      }
      const double b = lane < ns ? (passive ? xw[ci] : -xw[ci]) : 0.0;
      wave_sync();
      const double sol = chol_solve(a, b, ns, lane, bw, Lw, &bad);
      if (bad && npiv == 1 && from_warm) {
        // The warm-start set was not positive definite: start over from F = {}.
        bad = false;
        F = 0;
        x = 0.0;
        y = -p;
        wave_sync();
        continue;
      }
      if (bad) break;
      // scatter the compact solution back to original indices
      bw[lane] = sol;
      wave_sync();
      const double mine = si ? bw[rank] : 0.0;
      wave_sync();
      if (passive) {
        x = fi ? mine : 0.0;
        xw[lane] = x;
        wave_sync();
        double gx = 0.0;
        const int grow = lane < k ? lane : 0;
        for (int d = 0; d < ns; ++d) {
          const int j = iw[d];
          gx = fma((double)Gs[grow * LD + j], xw[j], gx);
        }
        y = fi ? 0.0 : gx - p;
      } else {
        // mine = y on A; x_F = cp_F + Ginv_FA y_A
        y = si ? mine : 0.0;
        xw[lane] = y;
        wave_sync();
        double gy = 0.0;
        const int grow = lane < k ? lane : 0;
        for (int d = 0; d < ns; ++d) {
          const int j = iw[d];
          gy = fma(Ginv[grow * KP + j], xw[j], gy);
        }
        x = fi ? cp + gy : 0.0;
        y = fi ? 0.0 : y;
      }
      wave_sync();
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
