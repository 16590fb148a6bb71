// Batched nonnegative least squares by block principal pivoting (Section 4.3,
// Eqs. (6)-(7)): for every row p of P solve
//     min_{x >= 0} 1/2 x^T G x - p^T x,    y = G x - p,
// until x_F >= 0 and y off F >= 0 (F the passive set). All right-hand sides
// share G (the Gram of the fixed factor), so one launch covers all of them.
//
// One wavefront per right-hand side, lane i <-> index i (k <= 64):
//   * the passive set is a 64-bit mask; the infeasible set V is a ballot;
//   * the exchange rule is Kim and Park's (the method the paper cites): swap
//     all of V while |V| keeps falling, at most three times without
//     progress, then only the largest index of V;
//   * the passive-set system G_FF x_F = p_F is solved on the full KP x KP
//     matrix D G D + (I - D), D = diag(F), by Cholesky: lane i keeps row i
//     in registers, each column of the factor is broadcast through LDS, and
//     the factor's rows go to LDS once for the backward solve.
// The factorisation, the solves and the sign tests run in double for every
// storage type: with float arithmetic, rounding noise on entries whose exact
// value is zero flips their sign from one pivot to the next and the pivoting
// can cycle. A non-positive pivot (G_FF not numerically positive definite)
// sets status |= 1; reaching the pivot cap sets status |= 2.
#include "common.h"
#include "kernels.h"

namespace nmfk {

template <typename TS, int KP>
__global__ __launch_bounds__(64) void bpp_kernel(TS* __restrict__ X, const TS* __restrict__ P,
                                                 const TS* __restrict__ G, int64_t rows, int k,
                                                 int max_pivots, int* __restrict__ status,
                                                 unsigned long long* __restrict__ pivots) {
  static_assert(KP <= 64, "one lane per index");
  typedef double T;  // compute type
  constexpr int LD = KP + 1;
  __shared__ T Gs[KP * LD];
  __shared__ T Ls[KP * LD];
  __shared__ T bc[KP];
  __shared__ T dinv[KP];
  const int i = threadIdx.x;
  const bool lanei = i < KP;
  const bool act = i < k;
  for (int e = i; e < KP * KP; e += 64) Gs[(e / KP) * LD + (e % KP)] = (T)G[e];
  __syncthreads();

  unsigned long long my_pivots = 0;
  int my_status = 0;
  for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
    const T p = act ? (T)P[r * KP + i] : T(0);
    T x = T(0), y = -p;
    uint64_t F = 0;
    int budget = 3, best = k + 1, npiv = 0;
    bool bad = false;
    for (;;) {
      const bool inF = (F >> i) & 1ull;
      const bool infeas = act && (inF ? (x < T(0)) : (y < T(0)));
      const uint64_t V = __ballot(infeas);
      if (V == 0) break;
      if (npiv >= max_pivots) { my_status |= 2; break; }
      const int nv = __popcll(V);
      uint64_t E;
      if (nv < best) { best = nv; budget = 3; E = V; }
      else if (budget >= 1) { --budget; E = V; }
      else { E = 1ull << (63 - __clzll(V)); }
      F ^= E;
      ++npiv;

      // Row i of M = D G D + (I - D).
      const bool fi = (F >> i) & 1ull;
      T a[KP];
#pragma unroll
      for (int j = 0; j < KP; ++j) {
        const bool fj = (F >> j) & 1ull;
        a[j] = (lanei && fi && fj) ? Gs[i * LD + j] : ((i == j) ? T(1) : T(0));
      }
      // Right-looking Cholesky, M = L L^T; lane i ends with row i of L in a[0..i].
#pragma unroll
      for (int q = 0; q < KP; ++q) {
        T dq = __shfl(a[q], q, 64);
        // A non-positive pivot is flagged; the factorisation continues on a
        // unit pivot so that control flow stays uniform and unrolled.
        if (!(dq > T(0))) { bad = true; dq = T(1); }
        const T s = sqrt(dq);
        const T l = a[q] / s;
        a[q] = (i >= q) ? l : T(0);
        if (i == 0) dinv[q] = T(1) / s;
        if (lanei) bc[i] = (i > q) ? l : T(0);
        __syncthreads();
        const T lq = (i > q) ? l : T(0);
#pragma unroll
        for (int j = q + 1; j < KP; ++j) a[j] -= lq * bc[j];
        __syncthreads();
      }
      if (bad) { my_status |= 1; break; }
      if (lanei) {
#pragma unroll
        for (int j = 0; j < KP; ++j) Ls[i * LD + j] = a[j];
      }
      __syncthreads();
      // Forward: L z = b, b = D p.
      T rz = fi ? p : T(0);
      T z = T(0);
#pragma unroll
      for (int q = 0; q < KP; ++q) {
        const T zq = __shfl(rz, q, 64) * dinv[q];
        if (i == q) z = zq;
        rz -= a[q] * zq;
      }
      // Backward: L^T x = z.
      T rx = z;
      T xi = T(0);
#pragma unroll
      for (int q = KP - 1; q >= 0; --q) {
        const T xq = __shfl(rx, q, 64) * dinv[q];
        if (i == q) xi = xq;
        const T lqi = lanei ? Ls[q * LD + i] : T(0);
        rx -= lqi * xq;
      }
      x = fi ? xi : T(0);
      // y = G x - p off F, 0 on F.
      if (lanei) bc[i] = x;
      __syncthreads();
      T gx = T(0);
      if (lanei) {
#pragma unroll
        for (int j = 0; j < KP; ++j) gx += Gs[i * LD + j] * bc[j];
      }
      y = fi ? T(0) : gx - p;
      __syncthreads();
    }
    my_pivots += (unsigned long long)npiv;
    if (lanei) X[r * KP + i] = act ? (TS)(x > T(0) ? x : T(0)) : TS(0);
  }
  if (i == 0) {
    atomicAdd(pivots, my_pivots);
    if (my_status) atomicOr(status, my_status);
  }
}

template <typename T>
hipError_t bpp_rows(T* X, const T* P, const T* G, int64_t rows, int k, int KP, int max_pivots,
                    int* status, unsigned long long* pivots, hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  const int64_t maxb = 256 * 32;
  const unsigned blocks = (unsigned)(rows < maxb ? rows : maxb);
  switch (KP) {
    case 16: bpp_kernel<T, 16><<<blocks, 64, 0, st>>>(X, P, G, rows, k, max_pivots, status, pivots); break;
    case 32: bpp_kernel<T, 32><<<blocks, 64, 0, st>>>(X, P, G, rows, k, max_pivots, status, pivots); break;
    case 48: bpp_kernel<T, 48><<<blocks, 64, 0, st>>>(X, P, G, rows, k, max_pivots, status, pivots); break;
    case 64: bpp_kernel<T, 64><<<blocks, 64, 0, st>>>(X, P, G, rows, k, max_pivots, status, pivots); break;
    default: return hipErrorInvalidValue;
  }
  return NMF_LAUNCH_CHECK();
}

template hipError_t bpp_rows<float>(float*, const float*, const float*, int64_t, int, int, int,
                                    int*, unsigned long long*, hipStream_t);
template hipError_t bpp_rows<double>(double*, const double*, const double*, int64_t, int, int,
                                     int, int*, unsigned long long*, hipStream_t);

}  // namespace nmfk
