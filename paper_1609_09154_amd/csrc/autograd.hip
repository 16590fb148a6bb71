// Reverse mode through T unrolled multiplicative updates (Section 4.1,
// Eq. (3)). On the row layout both half-steps have the form
//     Xn = X * N / D,   D = X G + eps   (elementwise * and /),
// with (X, N, G) = (W, A H^T, H H^T) for the W step and (H^T, A^T W, W^T W)
// for the H step. Given gXn = dL/dXn, the step's local adjoint is
//     dL/dN = gXn * X / D,   dL/dD = -gXn * Xn / D,
//     dL/dX = gXn * N / D + (dL/dD) G,   dL/dG = X^T (dL/dD),
// and the products that formed N and G pass the rest on to A and to the
// other factor (done by the driver with the product and Gram kernels).
// This file holds the row kernel of that local adjoint, the rank update that
// accumulates dL/dA, and the small row-times-matrix update.
#include "common.h"
#include "kernels.h"

namespace nmfk {

// Rows are split over TPR threads (a power of two, whole rows per wave) of
// RPT outputs each; 256 threads cover 256 / TPR rows; G is staged in LDS.
template <int KP> struct AdjSplit {
  static constexpr int TPR = KP == 48 ? 4 : KP / 8;
  static constexpr int RPT = KP / TPR;
  static constexpr int ROWS = 256 / TPR;
};

// Local adjoint of Xn = X * N / (X G + eps) for the rows of one block: writes
// gN, gD (= dL/dD) and gX; entries k..KP-1 are 0. G, the block's rows of X
// and dL/dD (shared between a row's threads for the (dL/dD) G^T term) live in
// LDS.
template <typename T, int KP>
__global__ __launch_bounds__(256) void mu_adjoint_rows_kernel(
    const T* __restrict__ X, const T* __restrict__ Xn, const T* __restrict__ N,
    const T* __restrict__ G, const T* __restrict__ gXn, int64_t rows, int k, T eps,
    T* __restrict__ gN, T* __restrict__ gD, T* __restrict__ gX) {
  constexpr int TPR = AdjSplit<KP>::TPR, RPT = AdjSplit<KP>::RPT, ROWS = AdjSplit<KP>::ROWS;
  constexpr int VEC = Tr<T>::VEC;
  constexpr int DLD = KP + VEC;
  __shared__ __attribute__((aligned(16))) T Gs[KP * KP];
  __shared__ __attribute__((aligned(16))) T Xs[ROWS * DLD];
  __shared__ __attribute__((aligned(16))) T Ds[ROWS * DLD];
  for (int e = threadIdx.x; e < KP * KP; e += 256) Gs[e] = G[e];
  const int64_t rb = (int64_t)blockIdx.x * ROWS;
  for (int e = threadIdx.x; e < ROWS * KP; e += 256) {
    const int q = e / KP, j = e % KP;
    Xs[q * DLD + j] = rb + q < rows ? X[(rb + q) * KP + j] : T(0);
  }
  __syncthreads();
  const int lr = threadIdx.x / TPR;
  const int64_t r = rb + lr;
  const bool live = r < rows;
  const int i0 = (threadIdx.x % TPR) * RPT;
  const T* xs = &Xs[lr * DLD];
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
#pragma unroll
  for (int ii = 0; ii < RPT; ++ii) {
    const int i = i0 + ii;
    T dd = T(0);
    if (live) {
      const int64_t e = r * KP + i;
      if (i < k) {
        const T den = d[ii] + eps;
        const T g = gXn[e];
        gN[e] = g * xs[i] / den;
        dd = -g * Xn[e] / den;
        gX[e] = g * N[e] / den;  // direct term; (dL/dD) G^T is added below
      } else {
        gN[e] = T(0);
        gX[e] = T(0);
      }
      gD[e] = dd;
    }
    Ds[lr * DLD + i] = dd;
  }
  __syncthreads();
  if (!live) return;
  // D_i = sum_j x_j G[j][i], so dL/dx_i picks up sum_j dd_j G[i][j]
#pragma unroll
  for (int ii = 0; ii < RPT; ++ii) {
    const int i = i0 + ii;
    if (i < k) {
      T acc = T(0);
#pragma unroll 4
      for (int q = 0; q < KP / VEC; ++q) {
        const V16<T> gv = load16<T>(&Gs[i * KP + q * VEC]);
        const V16<T> dv = load16<T>(&Ds[lr * DLD + q * VEC]);
#pragma unroll
        for (int w = 0; w < VEC; ++w) acc = fma(dv.v[w], gv.v[w], acc);
      }
      gX[r * KP + i] += acc;
    }
  }
}

// Out[r] += X[r] M for rows x KP X and KP x KP M.
template <typename T, int KP>
__global__ __launch_bounds__(256) void rowmm_add_kernel(const T* __restrict__ X,
                                                        const T* __restrict__ M, int64_t rows,
                                                        int k, T* __restrict__ Out) {
  constexpr int TPR = AdjSplit<KP>::TPR, RPT = AdjSplit<KP>::RPT, ROWS = AdjSplit<KP>::ROWS;
  constexpr int VEC = Tr<T>::VEC;
  constexpr int XLD = KP + VEC;
  __shared__ __attribute__((aligned(16))) T Ms[KP * KP];
  __shared__ __attribute__((aligned(16))) T Xs[ROWS * XLD];
  for (int e = threadIdx.x; e < KP * KP; e += 256) Ms[e] = M[e];
  const int64_t rb = (int64_t)blockIdx.x * ROWS;
  for (int e = threadIdx.x; e < ROWS * KP; e += 256) {
    const int q = e / KP, j = e % KP;
    Xs[q * XLD + j] = rb + q < rows ? X[(rb + q) * KP + j] : T(0);
  }
  __syncthreads();
  const int lr = threadIdx.x / TPR;
  const int64_t r = rb + lr;
  if (r >= rows) return;
  const int i0 = (threadIdx.x % TPR) * RPT;
  const T* xs = &Xs[lr * XLD];
  T s[RPT];
#pragma unroll
  for (int ii = 0; ii < RPT; ++ii) s[ii] = T(0);
#pragma unroll 8
  for (int j = 0; j < KP; ++j) {
    const T xj = xs[j];
#pragma unroll
    for (int q = 0; q < RPT / VEC; ++q) {
      const V16<T> v = load16<T>(&Ms[j * KP + i0 + q * VEC]);
#pragma unroll
      for (int w = 0; w < VEC; ++w) s[q * VEC + w] = fma(xj, v.v[w], s[q * VEC + w]);
    }
  }
#pragma unroll
  for (int ii = 0; ii < RPT; ++ii)
    if (i0 + ii < k) Out[r * KP + i0 + ii] += s[ii];
}

// M = G + G^T (KP x KP).
template <typename T>
__global__ void symmetrize_kernel(const T* __restrict__ G, int KP, T* __restrict__ M) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= KP * KP) return;
  const int i = e / KP, j = e % KP;
  M[e] = G[i * KP + j] + G[j * KP + i];
}

// Y += X elementwise (n elements).
template <typename T>
__global__ void add_kernel(T* __restrict__ Y, const T* __restrict__ X, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) Y[e] += X[e];
}

// D (m x n, ld ldd) += X1 Y1^T + X2 Y2^T with X* m x KP and Y* n x KP (row
// layout, KP contiguous). Each wave forms a 64 x 64 tile on the matrix cores
// (16 x 16 x 4 tiles, the reduction index permuted so every operand load is
// 16 bytes) and adds it to D; a workgroup is 64 rows x 256 columns.
constexpr int RU = 64;
template <typename T>
__global__ __launch_bounds__(256) void rank_update_kernel(T* __restrict__ D, int64_t ldd,
                                                          int64_t m, int64_t n,
                                                          const T* __restrict__ X1,
                                                          const T* __restrict__ Y1,
                                                          const T* __restrict__ X2,
                                                          const T* __restrict__ Y2, int KP) {
  constexpr int VEC = Tr<T>::VEC;
  typedef typename Tr<T>::acc4 acc4;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, c = lane & 15;
  const int64_t r0 = (int64_t)blockIdx.y * RU;
  const int64_t c0 = ((int64_t)blockIdx.x * 4 + wave) * RU;
  if (c0 >= n) return;
  acc4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = zero4<T>();
#pragma unroll
  for (int pr = 0; pr < 2; ++pr) {
    const T* X = pr == 0 ? X1 : X2;
    const T* Y = pr == 0 ? Y1 : Y2;
    if (X == nullptr) continue;
    const T* xr[4];
    const T* yr[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      int64_t row = r0 + 16 * t + c;
      row = row < m ? row : m - 1;
      xr[t] = X + row * KP;
      int64_t col = c0 + 16 * t + c;
      col = col < n ? col : n - 1;
      yr[t] = Y + col * KP;
    }
    for (int kk = 0; kk < KP; kk += 4 * VEC) {
      V16<T> xa[4], yb[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        xa[t] = load16<T>(xr[t] + kk + VEC * g);
        yb[t] = load16<T>(yr[t] + kk + VEC * g);
      }
#pragma unroll
      for (int v = 0; v < VEC; ++v)
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[a][b] = mfma16(xa[a].v[v], yb[b].v[v], acc[a][b]);
    }
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = r0 + 16 * a + acc_row<T>(lane, r);
      if (row < m) {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int64_t col = c0 + 16 * b + c;
          if (col < n) D[row * ldd + col] += acc[a][b][r];
        }
      }
    }
}

template <typename T>
hipError_t mu_adjoint_rows(const T* X, const T* Xn, const T* N, const T* G, const T* gXn,
                           int64_t rows, int k, int KP, T eps, T* gN, T* gD, T* gX,
                           hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  switch (KP) {
#define CASE(K)                                                                               \
  case K:                                                                                     \
    mu_adjoint_rows_kernel<T, K><<<(unsigned)cdiv(rows, AdjSplit<K>::ROWS), 256, 0, st>>>(   \
        X, Xn, N, G, gXn, rows, k, eps, gN, gD, gX);                                          \
    break;
    CASE(16) CASE(32) CASE(48) CASE(64)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return NMF_LAUNCH_CHECK();
}

template <typename T>
hipError_t rowmm_add(const T* X, const T* M, int64_t rows, int k, int KP, T* Out,
                     hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  switch (KP) {
#define CASE(K)                                                                              \
  case K:                                                                                    \
    rowmm_add_kernel<T, K><<<(unsigned)cdiv(rows, AdjSplit<K>::ROWS), 256, 0, st>>>(X, M,     \
                                                                                  rows, k,   \
                                                                                  Out);      \
    break;
    CASE(16) CASE(32) CASE(48) CASE(64)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return NMF_LAUNCH_CHECK();
}

template <typename T>
hipError_t symmetrize(const T* G, int KP, T* M, hipStream_t st) {
  symmetrize_kernel<T><<<(unsigned)cdiv(KP * KP, 256), 256, 0, st>>>(G, KP, M);
  return NMF_LAUNCH_CHECK();
}

template <typename T>
hipError_t add_to(T* Y, const T* X, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  add_kernel<T><<<(unsigned)cdiv(n, 256), 256, 0, st>>>(Y, X, n);
  return NMF_LAUNCH_CHECK();
}

template <typename T>
hipError_t rank_update(T* D, int64_t ldd, int64_t m, int64_t n, const T* X1, const T* Y1,
                       const T* X2, const T* Y2, int KP, hipStream_t st) {
  if (m <= 0 || n <= 0) return hipSuccess;
  if (KP % (4 * Tr<T>::VEC) != 0) return hipErrorInvalidValue;
  dim3 grid((unsigned)cdiv(n, 4 * RU), (unsigned)cdiv(m, RU));
  rank_update_kernel<T><<<grid, 256, 0, st>>>(D, ldd, m, n, X1, Y1, X2, Y2, KP);
  return NMF_LAUNCH_CHECK();
}

#define INST(T)                                                                               \
  template hipError_t mu_adjoint_rows<T>(const T*, const T*, const T*, const T*, const T*,    \
                                         int64_t, int, int, T, T*, T*, T*, hipStream_t);      \
  template hipError_t rowmm_add<T>(const T*, const T*, int64_t, int, int, T*, hipStream_t);   \
  template hipError_t symmetrize<T>(const T*, int, T*, hipStream_t);                          \
  template hipError_t add_to<T>(T*, const T*, int64_t, hipStream_t);                          \
  template hipError_t rank_update<T>(T*, int64_t, int64_t, int64_t, const T*, const T*,       \
                                     const T*, const T*, int, hipStream_t);
INST(float)
INST(double)
#undef INST

}  // namespace nmfk
