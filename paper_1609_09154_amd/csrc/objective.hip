// Relative error ||A - W H||_F / ||A||_F (Section 6.2), evaluated directly:
// a tile of W H^T... i.e. of W (Ht)^T, is formed on the matrix cores, the
// matching tile of A is read once, and squared differences are summed in
// double. Each workgroup writes one double; finish_relerr sums them in a
// fixed order, so the value is reproducible run to run.
#include "common.h"
#include "rowtile.h"
#include "kernels.h"

namespace nmfk {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block-wide sum of one double per thread (blockDim.x multiple of 64, <= 1024).
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double sh[16];
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += sh[i];
  return s;  // valid in thread 0
}

// Each wave: 64 rows x 64 columns of the residual; block = 4 waves stacked in
// columns (64 x 256).
constexpr int RT = 64;
template <typename T, typename TA>
__global__ __launch_bounds__(256) void residual_kernel(const TA* __restrict__ A, int64_t lda,
                                                       int64_t m, int64_t n,
                                                       const T* __restrict__ W,
                                                       const T* __restrict__ Ht, int KP,
                                                       double* __restrict__ partial) {
  constexpr int VEC = Tr<T>::VEC;
  typedef typename Tr<T>::acc4 acc4;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, c = lane & 15;
  const int64_t r0 = (int64_t)blockIdx.y * RT;
  const int64_t c0 = ((int64_t)blockIdx.x * 4 + wave) * RT;
  double local = 0.0;
  if (c0 < n) {
    acc4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = zero4<T>();
    const T* wr[4];
    const T* hr[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      int64_t row = r0 + 16 * t + c;
      row = row < m ? row : m - 1;
      wr[t] = W + row * KP;
      int64_t col = c0 + 16 * t + c;
      col = col < n ? col : n - 1;
      hr[t] = Ht + col * KP;
    }
    for (int kk = 0; kk < KP; kk += 4 * VEC) {
      V16<T> wa[4], hb[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        wa[t] = load16<T>(wr[t] + kk + VEC * g);
        hb[t] = load16<T>(hr[t] + kk + VEC * g);
      }
#pragma unroll
      for (int v = 0; v < VEC; ++v)
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[a][b] = mfma16(wa[a].v[v], hb[b].v[v], acc[a][b]);
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
            if (col < n) {
              const double d = to_double(A[row * lda + col]) - (double)acc[a][b][r];
              local += d * d;
            }
          }
        }
      }
  }
  const double s = block_sum(local);
  if (threadIdx.x == 0) partial[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = s;
}

template <typename T>
int64_t residual_partials(int64_t m, int64_t n) {
  return cdiv(n, 4 * RT) * cdiv(m, RT);
}

template <typename T, typename TA>
hipError_t residual_sq(const TA* A, int64_t lda, int64_t m, int64_t n, const T* W, const T* Ht,
                       int KP, double* partial, hipStream_t st) {
  dim3 grid((unsigned)cdiv(n, 4 * RT), (unsigned)cdiv(m, RT));
  residual_kernel<T, TA><<<grid, 256, 0, st>>>(A, lda, m, n, W, Ht, KP, partial);
  return NMF_LAUNCH_CHECK();
}

// ||A||^2: one block per 64 rows, double accumulation.
template <typename T>
__global__ __launch_bounds__(256) void sumsq_kernel(const T* __restrict__ A, int64_t lda,
                                                    int64_t m, int64_t n,
                                                    double* __restrict__ partial) {
  double local = 0.0;
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  for (int64_t r = r0; r < r0 + 64 && r < m; ++r)
    for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
      const double a = to_double(A[r * lda + j]);
      local += a * a;
    }
  const double s = block_sum(local);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// Projected gradient of 1/2 ||A - W H||_F^2 in one factor (Section 6.2's
// stationarity measure), on the row layout: for each row x with its product
// row p and the Gram G of the other factor, g = x G - p, and the projection
// keeps g_i where x_i > 0 and min(g_i, 0) where x_i = 0. Each block sums the
// squares of its rows in double: TPR threads per row (4; 16 for a double
// 128 x 128 Gram, to stay within LDS), RPT = KP / TPR entries each, with G
// and the block's rows staged in LDS.
template <typename T, int KP> struct PgSplit {
  static constexpr int TPR = (sizeof(T) == 8 && KP == 128) ? 16 : 4;
  static constexpr int ROWS = 256 / TPR;
};
template <typename T, int KP>
__global__ __launch_bounds__(256) void pgrad_sq_kernel(const T* __restrict__ X,
                                                       const T* __restrict__ P,
                                                       const T* __restrict__ G, int64_t rows,
                                                       int k, double* __restrict__ partial) {
  constexpr int PG_TPR = PgSplit<T, KP>::TPR, PG_ROWS = PgSplit<T, KP>::ROWS;
  constexpr int RPT = KP / PG_TPR;
  constexpr int VEC = Tr<T>::VEC;
  constexpr int XLD = KP + VEC;
  __shared__ __attribute__((aligned(16))) T Gs[KP * KP];
  __shared__ __attribute__((aligned(16))) T Xs[PG_ROWS * XLD];
  const int64_t rb = (int64_t)blockIdx.x * PG_ROWS;
  stage_square<T, KP, 256>(Gs, G, nullptr);
  stage_rows<T, KP, PG_ROWS, XLD, 256>(Xs, X, rb, rows);
  __syncthreads();
  const int lr = threadIdx.x / PG_TPR;
  const int64_t r = rb + lr;
  const int i0 = (threadIdx.x % PG_TPR) * RPT;
  const T* xs = &Xs[lr * XLD];
  double local = 0.0;
  if (r < rows) {
    T g[RPT];
#pragma unroll
    for (int ii = 0; ii < RPT; ++ii) g[ii] = T(0);
#pragma unroll 8
    for (int j = 0; j < KP; ++j) {
      const T xj = xs[j];
#pragma unroll
      for (int q = 0; q < RPT / VEC; ++q) {
        const V16<T> v = load16<T>(&Gs[j * KP + i0 + q * VEC]);
#pragma unroll
        for (int w = 0; w < VEC; ++w) g[q * VEC + w] = fma(xj, v.v[w], g[q * VEC + w]);
      }
    }
#pragma unroll
    for (int ii = 0; ii < RPT; ++ii) {
      const int i = i0 + ii;
      if (i < k) {
        const double gi = (double)g[ii] - (double)P[r * KP + i];
        const double pr = xs[i] > T(0) ? gi : (gi < 0.0 ? gi : 0.0);
        local += pr * pr;
      }
    }
  }
  const double s = block_sum(local);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// Upper bound on the blocks of any pgrad_sq launch (16 rows per block), and
// the exact count of one launch.
int64_t pgrad_partials(int64_t rows) { return cdiv(rows, 16); }
template <typename T>
int64_t pgrad_blocks(int64_t rows, int KP) {
  return cdiv(rows, (sizeof(T) == 8 && KP == 128) ? 16 : 64);
}
template int64_t pgrad_blocks<float>(int64_t, int);
template int64_t pgrad_blocks<double>(int64_t, int);

template <typename T>
hipError_t pgrad_sq(const T* X, const T* P, const T* G, int64_t rows, int k, int KP,
                    double* partial, hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  switch (KP) {
#define CASE(K)                                                                             \
  case K:                                                                                   \
    pgrad_sq_kernel<T, K><<<(unsigned)cdiv(rows, PgSplit<T, K>::ROWS), 256, 0, st>>>(      \
        X, P, G, rows, k, partial);                                                         \
    break;
    CASE(16) CASE(32) CASE(48) CASE(64) CASE(80) CASE(96) CASE(112) CASE(128)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return NMF_LAUNCH_CHECK();
}
template hipError_t pgrad_sq<float>(const float*, const float*, const float*, int64_t, int, int,
                                    double*, hipStream_t);
template hipError_t pgrad_sq<double>(const double*, const double*, const double*, int64_t, int,
                                     int, double*, hipStream_t);

template <typename T>
int64_t sumsq_partials(int64_t m, int64_t n) {
  (void)n;
  return cdiv(m, 64);
}

template <typename T>
hipError_t sumsq(const T* A, int64_t lda, int64_t m, int64_t n, double* partial,
                 hipStream_t st) {
  sumsq_kernel<T><<<(unsigned)cdiv(m, 64), 256, 0, st>>>(A, lda, m, n, partial);
  return NMF_LAUNCH_CHECK();
}

// One block of 256 threads; thread t sums partial[t], partial[t+256], ... in
// order, then a fixed tree.
template <typename T>
__global__ void finish_kernel(const double* __restrict__ partial, int64_t np,
                              const T* __restrict__ G1, const T* __restrict__ G2, int KP,
                              const double* __restrict__ ref_sq, double* __restrict__ out) {
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < np; i += blockDim.x) s += partial[i];
  if (G1 != nullptr)
    for (int e = threadIdx.x; e < KP * KP; e += blockDim.x) s += (double)G1[e] * (double)G2[e];
  const double tot = block_sum(s);
  if (threadIdx.x == 0) {
    if (ref_sq != nullptr) {
      const double v = tot > 0.0 ? tot : 0.0;
      *out = sqrt(v / *ref_sq);
    } else {
      *out = tot;
    }
  }
}

template <typename T>
hipError_t finish_relerr(const double* partial, int64_t np, const T* G1, const T* G2, int KP,
                         const double* ref_sq, double* out, hipStream_t st) {
  finish_kernel<T><<<1, 256, 0, st>>>(partial, np, G1, G2, KP, ref_sq, out);
  return NMF_LAUNCH_CHECK();
}

// Input scan: NaN, Inf or negative entries raise the flag.
template <typename T>
__global__ void check_dense_kernel(const T* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                                   int* __restrict__ flag) {
  const int64_t r0 = (int64_t)blockIdx.x * 16;
  int bad = 0;
  for (int64_t r = r0; r < r0 + 16 && r < m; ++r)
    for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
      const double a = to_double(A[r * lda + j]);
      if (!(a >= 0.0) || a == (double)INFINITY) bad = 1;
    }
  if (bad) atomicOr(flag, 1);
}

template <typename T>
hipError_t check_dense(const T* A, int64_t lda, int64_t m, int64_t n, int* flag,
                       hipStream_t st) {
  check_dense_kernel<T><<<(unsigned)cdiv(m, 16), 256, 0, st>>>(A, lda, m, n, flag);
  return NMF_LAUNCH_CHECK();
}

#define INST(T)                                                                               \
  template int64_t residual_partials<T>(int64_t, int64_t);                                    \
  template hipError_t residual_sq<T, T>(const T*, int64_t, int64_t, int64_t, const T*,        \
                                        const T*, int, double*, hipStream_t);                 \
  template int64_t sumsq_partials<T>(int64_t, int64_t);                                       \
  template hipError_t sumsq<T>(const T*, int64_t, int64_t, int64_t, double*, hipStream_t);    \
  template hipError_t finish_relerr<T>(const double*, int64_t, const T*, const T*, int,       \
                                       const double*, double*, hipStream_t);                  \
  template hipError_t check_dense<T>(const T*, int64_t, int64_t, int64_t, int*, hipStream_t);
INST(float)
INST(double)
#undef INST
#define INST_LP(TA)                                                                         \
  template hipError_t residual_sq<float, TA>(const TA*, int64_t, int64_t, int64_t,          \
                                             const float*, const float*, int, double*,       \
                                             hipStream_t);                                   \
  template int64_t sumsq_partials<TA>(int64_t, int64_t);                                    \
  template hipError_t sumsq<TA>(const TA*, int64_t, int64_t, int64_t, double*, hipStream_t); \
  template hipError_t check_dense<TA>(const TA*, int64_t, int64_t, int64_t, int*, hipStream_t);
INST_LP(uint16_t)
INST_LP(uint8_t)
#undef INST_LP

}  // namespace nmfk
