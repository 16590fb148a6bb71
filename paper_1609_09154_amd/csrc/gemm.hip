// Dense products of Algorithm 1 on the gfx950 matrix cores (MFMA 16x16x4,
// fp32 or fp64), for one GPU's whole problem:
//
//   NN:  D (M x N) = X (M x K) * Y (K x N)   X K-contiguous, Y N-contiguous
//        used for P = A H^T  (X = A, Y = H^T, K = n)
//   TN:  D (M x N) = X^T * Y, X (K x M), Y (K x N), both row-contiguous
//        used for R = A^T W  (X = A, Y = W, K = m)  and the Grams
//        W^T W, H H^T        (X = Y = W or H^T)
//
// N is the padded rank KP = 16 * NT (KP >= k, zero padded), so each wave
// owns MW 16-row tiles of the streamed side and all NT tiles of the rank
// side: every element of A is loaded into registers exactly once, by one
// lane, and feeds NT MFMAs. The rank-side operand (a few MB) is shared by
// all waves and read through the L2.
//
// The reduction index is a sum, so the K positions each lane supplies can be
// permuted freely as long as both operands agree. NN uses that to give each
// lane a 16-byte run of a row of A (VEC consecutive K values feed VEC
// successive MFMAs); TN uses the same freedom on the M side (VEC consecutive
// columns of a row of A feed VEC different output tiles).
//
// Large reductions can be split (grid.y) into slabs written to a workspace
// and summed in a fixed order by reduce_splits, so results are bitwise
// reproducible run to run.
#include "common.h"
#include "kernels.h"

namespace nmfk {

// ---------------------------------------------------------------------------
// NN kernel
// ---------------------------------------------------------------------------
template <typename T, int NT, int MW, bool VX>
__global__ __launch_bounds__(256) void gemm_nn_kernel(
    const T* __restrict__ X, int64_t ldx, const T* __restrict__ Y, int64_t ldy,
    T* __restrict__ D, int64_t ldd, int64_t dsplit, int64_t M, int64_t K,
    int64_t kchunk) {
  constexpr int VEC = Tr<T>::VEC;
  constexpr int KSTEP = 4 * VEC;
  typedef typename Tr<T>::acc4 acc4;
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4, c = lane & 15;
  const int64_t m0 = ((int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * (16 * MW);
  if (m0 >= M) return;
  const int64_t kbeg = (int64_t)blockIdx.y * kchunk;
  const int64_t kend = kbeg + kchunk < K ? kbeg + kchunk : K;

  const T* xr[MW];
#pragma unroll
  for (int mt = 0; mt < MW; ++mt) {
    int64_t row = m0 + 16 * mt + c;
    row = row < M ? row : M - 1;
    xr[mt] = X + row * ldx;
  }
  acc4 acc[MW][NT];
#pragma unroll
  for (int mt = 0; mt < MW; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = zero4<T>();

  V16<T> xa[MW], xb[MW];
  T ya[NT][VEC], yb[NT][VEC];

#define NN_LOAD(XV, YV, K0)                                                   \
  {                                                                           \
    const int64_t kk0 = (K0) + VEC * g;                                       \
    _Pragma("unroll") for (int mt = 0; mt < MW; ++mt) {                       \
      if constexpr (VX) {                                                     \
        XV[mt] = load16_stream<T>(xr[mt] + kk0);                              \
      } else {                                                                \
        _Pragma("unroll") for (int v = 0; v < VEC; ++v) XV[mt].v[v] = xr[mt][kk0 + v]; \
      }                                                                       \
    }                                                                         \
    _Pragma("unroll") for (int nt = 0; nt < NT; ++nt)                         \
      _Pragma("unroll") for (int v = 0; v < VEC; ++v)                         \
        YV[nt][v] = Y[(kk0 + v) * ldy + 16 * nt + c];                         \
  }
#define NN_COMPUTE(XV, YV)                                                    \
  {                                                                           \
    _Pragma("unroll") for (int v = 0; v < VEC; ++v)                           \
      _Pragma("unroll") for (int mt = 0; mt < MW; ++mt)                       \
        _Pragma("unroll") for (int nt = 0; nt < NT; ++nt)                     \
          acc[mt][nt] = mfma16(XV[mt].v[v], YV[nt][v], acc[mt][nt]);          \
  }

  const int64_t nsteps = (kend - kbeg) / KSTEP;
  if (nsteps > 0) {
    NN_LOAD(xa, ya, kbeg);
    int64_t s = 0;
    for (; s + 2 <= nsteps; s += 2) {
      NN_LOAD(xb, yb, kbeg + (s + 1) * KSTEP);
      NN_COMPUTE(xa, ya);
      if (s + 2 < nsteps) NN_LOAD(xa, ya, kbeg + (s + 2) * KSTEP);
      NN_COMPUTE(xb, yb);
    }
    if (s < nsteps) NN_COMPUTE(xa, ya);
  }
  const int64_t ktail = kbeg + nsteps * KSTEP;
  if (ktail < kend) {
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      const int64_t kk = ktail + VEC * g + v;
      const bool ok = kk < kend;
#pragma unroll
      for (int mt = 0; mt < MW; ++mt) xa[mt].v[v] = ok ? xr[mt][kk] : T(0);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) ya[nt][v] = ok ? Y[kk * ldy + 16 * nt + c] : T(0);
    }
    NN_COMPUTE(xa, ya);
  }
#undef NN_LOAD
#undef NN_COMPUTE

  T* Dp = D + (int64_t)blockIdx.y * dsplit;
#pragma unroll
  for (int mt = 0; mt < MW; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = m0 + 16 * mt + acc_row<T>(lane, r);
      if (row < M) {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) Dp[row * ldd + 16 * nt + c] = acc[mt][nt][r];
      }
    }
}

// ---------------------------------------------------------------------------
// TN kernel
// ---------------------------------------------------------------------------
// Column of X that lane column c feeds into M-tile t.  Vector path: tile t
// takes columns m0 + 16*VEC*(t/VEC) + VEC*c + t%VEC (one 16-byte load per
// lane covers VEC tiles).  Scalar path: m0 + 16 t + c.
template <typename T, bool VX>
__device__ __forceinline__ int64_t tn_col(int64_t m0, int t, int c) {
  constexpr int VEC = Tr<T>::VEC;
  if constexpr (VX) return m0 + 16 * VEC * (t / VEC) + VEC * c + (t % VEC);
  else return m0 + 16 * t + c;
}

template <typename T, int NT, int MW, bool VX, int U>
__global__ __launch_bounds__(256) void gemm_tn_kernel(
    const T* __restrict__ X, int64_t ldx, const T* __restrict__ Y, int64_t ldy,
    T* __restrict__ D, int64_t ldd, int64_t dsplit, int64_t M, int64_t K,
    int64_t kchunk) {
  constexpr int VEC = Tr<T>::VEC;
  constexpr int NQ = VX ? MW / VEC : MW;  // loads per row on the X side
  static_assert(!VX || MW % VEC == 0, "vector path needs MW % VEC == 0");
  typedef typename Tr<T>::acc4 acc4;
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4, c = lane & 15;
  const int64_t m0 = ((int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * (16 * MW);
  if (m0 >= M) return;
  const int64_t kbeg = (int64_t)blockIdx.y * kchunk;
  const int64_t kend = kbeg + kchunk < K ? kbeg + kchunk : K;
  // A wave whose columns run past M takes the guarded scalar path.
  const bool full = m0 + 16 * MW <= M;

  acc4 acc[MW][NT];
#pragma unroll
  for (int t = 0; t < MW; ++t)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[t][nt] = zero4<T>();

  // xs[u][t]: X value for tile t at row k0 + 4u + g; ys[u][nt]: Y value.
  T xa[U][MW], xb[U][MW];
  T ya[U][NT], yb[U][NT];

#define TN_LOAD(XS, YS, K0)                                                   \
  {                                                                           \
    _Pragma("unroll") for (int u = 0; u < U; ++u) {                           \
      const int64_t kk = (K0) + 4 * u + g;                                    \
      const T* xrow = X + kk * ldx;                                           \
      if constexpr (VX) {                                                     \
        _Pragma("unroll") for (int q = 0; q < NQ; ++q) {                      \
          V16<T> t16 = load16_stream<T>(xrow + m0 + 16 * VEC * q + VEC * c);  \
          _Pragma("unroll") for (int v = 0; v < VEC; ++v) XS[u][q * VEC + v] = t16.v[v]; \
        }                                                                     \
      } else {                                                                \
        _Pragma("unroll") for (int t = 0; t < MW; ++t) XS[u][t] = xrow[m0 + 16 * t + c]; \
      }                                                                       \
      _Pragma("unroll") for (int nt = 0; nt < NT; ++nt)                       \
        YS[u][nt] = Y[kk * ldy + 16 * nt + c];                                \
    }                                                                         \
  }
#define TN_COMPUTE(XS, YS)                                                    \
  {                                                                           \
    _Pragma("unroll") for (int u = 0; u < U; ++u)                             \
      _Pragma("unroll") for (int t = 0; t < MW; ++t)                          \
        _Pragma("unroll") for (int nt = 0; nt < NT; ++nt)                     \
          acc[t][nt] = mfma16(XS[u][t], YS[u][nt], acc[t][nt]);               \
  }

  constexpr int KSTEP = 4 * U;
  int64_t nsteps = (kend - kbeg) / KSTEP;
  if (!full) nsteps = 0;  // everything through the guarded tail loop below
  if (nsteps > 0) {
    TN_LOAD(xa, ya, kbeg);
    int64_t s = 0;
    for (; s + 2 <= nsteps; s += 2) {
      TN_LOAD(xb, yb, kbeg + (s + 1) * KSTEP);
      TN_COMPUTE(xa, ya);
      if (s + 2 < nsteps) TN_LOAD(xa, ya, kbeg + (s + 2) * KSTEP);
      TN_COMPUTE(xb, yb);
    }
    if (s < nsteps) TN_COMPUTE(xa, ya);
  }
  // Guarded remainder, 4 rows at a time (also the whole range for a ragged wave).
  for (int64_t k0 = kbeg + nsteps * KSTEP; k0 < kend; k0 += 4) {
    const int64_t kk = k0 + g;
    const bool okk = kk < kend;
    const int64_t kc = okk ? kk : kbeg;
#pragma unroll
    for (int t = 0; t < MW; ++t) {
      const int64_t col = tn_col<T, VX>(m0, t, c);
      xa[0][t] = (okk && col < M) ? X[kc * ldx + col] : T(0);
    }
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) ya[0][nt] = okk ? Y[kc * ldy + 16 * nt + c] : T(0);
#pragma unroll
    for (int t = 0; t < MW; ++t)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) acc[t][nt] = mfma16(xa[0][t], ya[0][nt], acc[t][nt]);
  }
#undef TN_LOAD
#undef TN_COMPUTE

  T* Dp = D + (int64_t)blockIdx.y * dsplit;
#pragma unroll
  for (int t = 0; t < MW; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int rho = acc_row<T>(lane, r);
      const int64_t row = tn_col<T, VX>(m0, t, rho);
      if (row < M) {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) Dp[row * ldd + 16 * nt + c] = acc[t][nt][r];
      }
    }
}

// out[i] = sum_s part[s * stride + i] in order s = 0, 1, ... (double sums).
template <typename T>
__global__ void reduce_splits_kernel(const T* __restrict__ part, int splits, int64_t stride,
                                     int64_t rows, int cols, int64_t ldo, T* __restrict__ out,
                                     int64_t ldp) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  const int64_t r = idx / cols, cc = idx - r * cols;
  double s = 0.0;
  for (int p = 0; p < splits; ++p) s += (double)part[p * stride + r * ldp + cc];
  out[r * ldo + cc] = (T)s;
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
template <typename T> static constexpr int mw_for(int NT) {
  return sizeof(T) == 4 ? 4 : (NT <= 4 ? 4 : 2);
}

template <typename T, int NT>
static hipError_t nn_dispatch(const GemmArgs<T>& a, bool vx, int64_t splits, int64_t kchunk,
                              T* D, int64_t ldd, int64_t dsplit, hipStream_t st) {
  constexpr int MW = mw_for<T>(NT);
  const int waves = 4;
  dim3 grid((unsigned)cdiv(a.M, 16 * MW * waves), (unsigned)splits);
  if (vx)
    gemm_nn_kernel<T, NT, MW, true><<<grid, 64 * waves, 0, st>>>(a.X, a.ldx, a.Y, a.ldy, D, ldd,
                                                                 dsplit, a.M, a.K, kchunk);
  else
    gemm_nn_kernel<T, NT, MW, false><<<grid, 64 * waves, 0, st>>>(a.X, a.ldx, a.Y, a.ldy, D, ldd,
                                                                  dsplit, a.M, a.K, kchunk);
  return NMF_LAUNCH_CHECK();
}

template <typename T, int NT, int MW>
static hipError_t tn_dispatch_mw(const GemmArgs<T>& a, bool vx, int waves, int64_t splits,
                                 int64_t kchunk, T* D, int64_t ldd, int64_t dsplit,
                                 hipStream_t st) {
  constexpr int U = 4;
  dim3 grid((unsigned)cdiv(a.M, 16 * MW * waves), (unsigned)splits);
  if constexpr (MW % Tr<T>::VEC == 0) {
    if (vx) {
      gemm_tn_kernel<T, NT, MW, true, U><<<grid, 64 * waves, 0, st>>>(
          a.X, a.ldx, a.Y, a.ldy, D, ldd, dsplit, a.M, a.K, kchunk);
      return NMF_LAUNCH_CHECK();
    }
  }
  gemm_tn_kernel<T, NT, MW, false, U><<<grid, 64 * waves, 0, st>>>(a.X, a.ldx, a.Y, a.ldy, D, ldd,
                                                                   dsplit, a.M, a.K, kchunk);
  return NMF_LAUNCH_CHECK();
}

template <typename T, int NT>
static hipError_t tn_dispatch(const GemmArgs<T>& a, bool vx, bool small_m, int64_t splits,
                              int64_t kchunk, T* D, int64_t ldd, int64_t dsplit, hipStream_t st) {
  if (small_m) {
    // Gram: the M side is the padded rank itself; one wave per 16*MW columns.
    constexpr int MW = NT <= 4 ? NT : 4;
    constexpr int MWd = (sizeof(T) == 8 && NT > 4) ? 2 : MW;
    return tn_dispatch_mw<T, NT, MWd>(a, vx, 1, splits, kchunk, D, ldd, dsplit, st);
  }
  constexpr int MW = mw_for<T>(NT);
  return tn_dispatch_mw<T, NT, MW>(a, vx, 4, splits, kchunk, D, ldd, dsplit, st);
}

static bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

template <typename T>
hipError_t gemm_run(GemmKind kind, const GemmArgs<T>& a, int64_t splits, T* part,
                    hipStream_t st) {
  constexpr int VEC = Tr<T>::VEC;
  const int NT = (int)(a.N / 16);
  if (NT < 1 || NT > 8 || a.N % 16 != 0) return hipErrorInvalidValue;
  if (splits < 1) splits = 1;
  const int64_t unit = kind == GemmKind::NN ? 4 * VEC : 16;
  int64_t kchunk = round_up(cdiv(a.K, splits), unit);
  splits = cdiv(a.K, kchunk);
  if (splits < 1) splits = 1;
  const bool vx = aligned16(a.X) && (a.ldx % VEC == 0);
  const bool small_m = kind == GemmKind::TN_GRAM;
  T* D = splits > 1 ? part : a.D;
  const int64_t ldd = splits > 1 ? a.N : a.ldd;
  const int64_t dsplit = a.M * a.N;
  hipError_t e = hipSuccess;
#define NT_CASE(n)                                                                        \
  case n:                                                                                 \
    e = kind == GemmKind::NN                                                              \
            ? nn_dispatch<T, n>(a, vx, splits, kchunk, D, ldd, dsplit, st)                \
            : tn_dispatch<T, n>(a, vx, small_m, splits, kchunk, D, ldd, dsplit, st);      \
    break;
  switch (NT) {
    NT_CASE(1) NT_CASE(2) NT_CASE(3) NT_CASE(4) NT_CASE(5) NT_CASE(6) NT_CASE(7) NT_CASE(8)
    default: return hipErrorInvalidValue;
  }
#undef NT_CASE
  if (e != hipSuccess || splits == 1) return e;
  const int64_t total = a.M * a.N;
  reduce_splits_kernel<T><<<(unsigned)cdiv(total, 256), 256, 0, st>>>(
      part, (int)splits, dsplit, a.M, (int)a.N, a.ldd, a.D, a.N);
  return NMF_LAUNCH_CHECK();
}

template hipError_t gemm_run<float>(GemmKind, const GemmArgs<float>&, int64_t, float*, hipStream_t);
template hipError_t gemm_run<double>(GemmKind, const GemmArgs<double>&, int64_t, double*, hipStream_t);

}  // namespace nmfk
