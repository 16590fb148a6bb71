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

// One thread per row r (KP <= 64 values in registers; G read with uniform
// loads). Writes gN, gD (= dL/dD) and gX for the row; entries k..KP-1 are 0.
template <typename T, int KP>
__global__ __launch_bounds__(256) void mu_adjoint_rows_kernel(
    const T* __restrict__ X, const T* __restrict__ Xn, const T* __restrict__ N,
    const T* __restrict__ G, const T* __restrict__ gXn, int64_t rows, int k, T eps,
    T* __restrict__ gN, T* __restrict__ gD, T* __restrict__ gX) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  const T* xr = X + r * KP;
  T x[KP];
#pragma unroll
  for (int i = 0; i < KP; ++i) x[i] = xr[i];
  T dd[KP];  // dL/dD of this row
  constexpr int CH = 16;
#pragma unroll
  for (int i0 = 0; i0 < KP; i0 += CH) {
    T d[CH];
#pragma unroll
    for (int ii = 0; ii < CH; ++ii) d[ii] = T(0);
#pragma unroll
    for (int j = 0; j < KP; ++j)
#pragma unroll
      for (int ii = 0; ii < CH; ++ii) d[ii] = fma(x[j], G[j * KP + i0 + ii], d[ii]);
#pragma unroll
    for (int ii = 0; ii < CH; ++ii) {
      const int i = i0 + ii;
      const int64_t e = r * KP + i;
      if (i < k) {
        const T den = d[ii] + eps;
        const T g = gXn[e];
        gN[e] = g * x[i] / den;
        dd[i] = -g * Xn[e] / den;
        gX[e] = g * N[e] / den;  // direct term; (dL/dD) G is added below
      } else {
        gN[e] = T(0);
        dd[i] = T(0);
        gX[e] = T(0);
      }
    }
  }
#pragma unroll
  for (int i0 = 0; i0 < KP; i0 += CH) {
    T s[CH];
#pragma unroll
    for (int ii = 0; ii < CH; ++ii) s[ii] = T(0);
    // D_i = sum_j x_j G[j][i], so dL/dx_i picks up sum_j dd_j G[i][j]
#pragma unroll
    for (int j = 0; j < KP; ++j)
#pragma unroll
      for (int ii = 0; ii < CH; ++ii) s[ii] = fma(dd[j], G[(i0 + ii) * KP + j], s[ii]);
#pragma unroll
    for (int ii = 0; ii < CH; ++ii) {
      const int i = i0 + ii;
      const int64_t e = r * KP + i;
      gD[e] = dd[i];
      if (i < k) gX[e] += s[ii];
    }
  }
}

// Out[r] += X[r] M for rows x KP X and KP x KP M (one thread per row).
template <typename T, int KP>
__global__ __launch_bounds__(256) void rowmm_add_kernel(const T* __restrict__ X,
                                                        const T* __restrict__ M, int64_t rows,
                                                        int k, T* __restrict__ Out) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  T x[KP];
#pragma unroll
  for (int i = 0; i < KP; ++i) x[i] = X[r * KP + i];
  constexpr int CH = 16;
#pragma unroll
  for (int i0 = 0; i0 < KP; i0 += CH) {
    if (i0 < k) {
      T s[CH];
#pragma unroll
      for (int ii = 0; ii < CH; ++ii) s[ii] = T(0);
#pragma unroll
      for (int j = 0; j < KP; ++j)
#pragma unroll
        for (int ii = 0; ii < CH; ++ii) s[ii] = fma(x[j], M[j * KP + i0 + ii], s[ii]);
#pragma unroll
      for (int ii = 0; ii < CH; ++ii)
        if (i0 + ii < k) Out[r * KP + i0 + ii] += s[ii];
    }
  }
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
  const unsigned blocks = (unsigned)cdiv(rows, 256);
  switch (KP) {
#define CASE(K)                                                                               \
  case K:                                                                                     \
    mu_adjoint_rows_kernel<T, K><<<blocks, 256, 0, st>>>(X, Xn, N, G, gXn, rows, k, eps, gN, \
                                                          gD, gX);                            \
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
  const unsigned blocks = (unsigned)cdiv(rows, 256);
  switch (KP) {
#define CASE(K)                                                                 \
  case K: rowmm_add_kernel<T, K><<<blocks, 256, 0, st>>>(X, M, rows, k, Out); break;
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
