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
// Rank remainder (NR = 1): when k exceeds a multiple of 16 by at most 4
// (k = 50 = 3 * 16 + 2), the last four columns are computed with the 4x4x1
// MFMA instead of a fourth 16-wide tile. The same A-operand register is read
// as sixteen 4-row blocks (block b = lane / 4: lane group b / 4 fixes the K
// index, b % 4 the four rows), each multiplied by the remainder columns of
// its own K index; the four lane groups' blocks are summed at the end with
// two cross-lane adds. That costs 2 MFMA passes instead of 8 per step, and
// columns past 16 * NT + 4 are written as zeros.
//
// Large reductions can be split (grid.y) into slabs written to a workspace
// and summed in a fixed order by reduce_splits, so results are bitwise
// reproducible run to run.
#include "common.h"
#include "kernels.h"

namespace nmfk {

// ---------------------------------------------------------------------------
// Software pipeline over K steps. LOAD(buf, k0) issues the global loads of
// one step into a register buffer, COMPUTE(buf) runs its MFMAs. With three
// buffers the loads of step s+2 are in flight while step s computes.
// ---------------------------------------------------------------------------
// S-stage ring: buffer j % S holds step j; the loads of step s + S - 1 are
// issued before the MFMAs of step s. The steady-state loop body is unrolled S
// times so every buffer index is a compile-time constant and no branch sits
// between a load and its use.
#define NMF_PIPELINE(S, LOAD, COMPUTE, F, KBEG, NSTEPS, STEPK)                             \
  {                                                                                       \
    const int64_t n_ = (NSTEPS);                                                          \
    if (n_ < (S) - 1) {                                                                   \
      for (int64_t s_ = 0; s_ < n_; ++s_) {                                               \
        LOAD(F[0], (KBEG) + s_ * (STEPK));                                                \
        COMPUTE(F[0]);                                                                    \
      }                                                                                   \
    } else {                                                                              \
      _Pragma("unroll") for (int j_ = 0; j_ < (S) - 1; ++j_)                              \
        LOAD(F[j_], (KBEG) + j_ * (STEPK));                                               \
      int64_t s_ = 0;                                                                     \
      for (; s_ + 2 * (S) - 1 <= n_; s_ += (S)) {                                         \
        _Pragma("unroll") for (int j_ = 0; j_ < (S); ++j_) {                              \
          LOAD(F[(j_ + (S) - 1) % (S)], (KBEG) + (s_ + j_ + (S) - 1) * (STEPK));          \
          COMPUTE(F[j_]);                                                                 \
        }                                                                                 \
      }                                                                                   \
      _Pragma("unroll") for (int j_ = 0; j_ < 2 * (S) - 2; ++j_) {                        \
        if (s_ + j_ < n_) {                                                               \
          if (s_ + j_ + (S) - 1 < n_)                                                     \
            LOAD(F[(j_ + (S) - 1) % (S)], (KBEG) + (s_ + j_ + (S) - 1) * (STEPK));        \
          COMPUTE(F[j_ % (S)]);                                                           \
        }                                                                                 \
      }                                                                                   \
    }                                                                                     \
  }

// ---------------------------------------------------------------------------
// NN kernel. Y is either K x N (YT = false, ldy between K rows) or its
// transpose N x K (YT = true, ldy between N rows), which lets each lane fetch
// its VEC consecutive K values of a Y column with one 16-byte load.
// ---------------------------------------------------------------------------
template <typename T, int NT, int MW> struct FragNN {
  V16<T> x[MW];
  T y[NT][Tr<T>::VEC];
  T yr[Tr<T>::VEC];  // remainder columns (NR = 1)
};

template <typename T, int NT, int MW, bool VX, bool YT, int STAGES, int WPE, int NR = 0>
__global__ __launch_bounds__(256, WPE) void gemm_nn_kernel(
    const T* __restrict__ X, int64_t ldx, const T* __restrict__ Y, int64_t ldy,
    T* __restrict__ D, int64_t ldd, int64_t dsplit, int64_t M, int64_t K,
    int64_t kchunk, int ldd_cols_ = 16 * NT) {
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
  static_assert(NR == 0 || sizeof(T) == 4, "rank remainder tile is float only");
  acc4 acc[MW][NT];
  acc4 accr[MW];
  const int cr = 16 * NT + (lane & 3);  // remainder column fed by this lane
#pragma unroll
  for (int mt = 0; mt < MW; ++mt) {
    accr[mt] = zero4<T>();
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = zero4<T>();
  }

  FragNN<T, NT, MW> fr[STAGES];

#define NN_LOAD(F, K0)                                                        \
  {                                                                           \
    const int64_t kk0 = (K0) + VEC * g;                                       \
    _Pragma("unroll") for (int mt = 0; mt < MW; ++mt) {                       \
      if constexpr (VX) {                                                     \
        F.x[mt] = load16_stream<T>(xr[mt] + kk0);                             \
      } else {                                                                \
        _Pragma("unroll") for (int v = 0; v < VEC; ++v) F.x[mt].v[v] = xr[mt][kk0 + v]; \
      }                                                                       \
    }                                                                         \
    _Pragma("unroll") for (int nt = 0; nt < NT; ++nt) {                       \
      if constexpr (YT) {                                                     \
        const V16<T> t_ = load16<T>(Y + (int64_t)(16 * nt + c) * ldy + kk0);  \
        _Pragma("unroll") for (int v = 0; v < VEC; ++v) F.y[nt][v] = t_.v[v]; \
      } else {                                                                \
        _Pragma("unroll") for (int v = 0; v < VEC; ++v)                       \
          F.y[nt][v] = Y[(kk0 + v) * ldy + 16 * nt + c];                      \
      }                                                                       \
    }                                                                         \
    if constexpr (NR) {                                                       \
      if constexpr (YT) {                                                     \
        const V16<T> t_ = load16<T>(Y + (int64_t)cr * ldy + kk0);             \
        _Pragma("unroll") for (int v = 0; v < VEC; ++v) F.yr[v] = t_.v[v];    \
      } else {                                                                \
        _Pragma("unroll") for (int v = 0; v < VEC; ++v)                       \
          F.yr[v] = Y[(kk0 + v) * ldy + cr];                                  \
      }                                                                       \
    }                                                                         \
  }
#define NN_COMPUTE(F)                                                         \
  {                                                                           \
    _Pragma("unroll") for (int v = 0; v < VEC; ++v)                           \
      _Pragma("unroll") for (int mt = 0; mt < MW; ++mt) {                     \
        _Pragma("unroll") for (int nt = 0; nt < NT; ++nt)                     \
          acc[mt][nt] = mfma16(F.x[mt].v[v], F.y[nt][v], acc[mt][nt]);        \
        if constexpr (NR) accr[mt] = mfma4x4(F.x[mt].v[v], F.yr[v], accr[mt]); \
      }                                                                       \
  }

  const int64_t nsteps = (kend - kbeg) / KSTEP;
  NMF_PIPELINE(STAGES, NN_LOAD, NN_COMPUTE, fr, kbeg, nsteps, KSTEP)

  const int64_t ktail = kbeg + nsteps * KSTEP;
  if (ktail < kend) {
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      const int64_t kk = ktail + VEC * g + v;
      const bool ok = kk < kend;
#pragma unroll
      for (int mt = 0; mt < MW; ++mt) fr[0].x[mt].v[v] = ok ? xr[mt][kk] : T(0);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
        fr[0].y[nt][v] = ok ? (YT ? Y[(int64_t)(16 * nt + c) * ldy + kk] : Y[kk * ldy + 16 * nt + c])
                            : T(0);
      if constexpr (NR) fr[0].yr[v] = ok ? (YT ? Y[(int64_t)cr * ldy + kk] : Y[kk * ldy + cr]) : T(0);
    }
    NN_COMPUTE(fr[0]);
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
  if constexpr (NR) {
    // Sum the four lane groups (different K), then lanes 0..15 hold rows
    // m0 + 16 mt + 4 (lane / 4) + r of remainder column cr.
#pragma unroll
    for (int mt = 0; mt < MW; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        T v = accr[mt][r];
        v += __shfl_xor(v, 16, 64);
        v += __shfl_xor(v, 32, 64);
        const int64_t row = m0 + 16 * mt + 4 * (lane >> 2) + r;
        if (g == 0 && row < M) {
          Dp[row * ldd + cr] = v;
          for (int z = 16 * NT + 4 + (lane & 3); z < ldd_cols_; z += 4) Dp[row * ldd + z] = T(0);
        }
      }
  }
}

// ---------------------------------------------------------------------------
// TN kernel. One pipeline step covers 16 rows of X: lane group g supplies
// rows k0 + 4g + u to MFMA u (u = 0..3). Y is K x N (YT = false) or N x K
// (YT = true, so the four rows a lane needs are one 16-byte load).
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

template <typename T, int NT, int MW> struct FragTN {
  T x[4][MW];
  T y[4][NT];
  T yr[4];  // remainder columns (NR = 1)
};

template <typename T, int NT, int MW, bool VX, bool YT, int STAGES, int WPE, int NR = 0>
__global__ __launch_bounds__(256, WPE) void gemm_tn_kernel(
    const T* __restrict__ X, int64_t ldx, const T* __restrict__ Y, int64_t ldy,
    T* __restrict__ D, int64_t ldd, int64_t dsplit, int64_t M, int64_t K,
    int64_t kchunk, int ldd_cols_ = 16 * NT) {
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

  static_assert(NR == 0 || sizeof(T) == 4, "rank remainder tile is float only");
  acc4 acc[MW][NT];
  acc4 accr[MW];
  const int cr = 16 * NT + (lane & 3);  // remainder column fed by this lane
#pragma unroll
  for (int t = 0; t < MW; ++t) {
    accr[t] = zero4<T>();
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[t][nt] = zero4<T>();
  }

  FragTN<T, NT, MW> fr[STAGES];

#define TN_LOAD(F, K0)                                                        \
  {                                                                           \
    _Pragma("unroll") for (int u = 0; u < 4; ++u) {                           \
      const int64_t kk = (K0) + 4 * g + u;                                    \
      const T* xrow = X + kk * ldx;                                           \
      if constexpr (VX) {                                                     \
        _Pragma("unroll") for (int q = 0; q < NQ; ++q) {                      \
          V16<T> t16 = load16_stream<T>(xrow + m0 + 16 * VEC * q + VEC * c);  \
          _Pragma("unroll") for (int v = 0; v < VEC; ++v) F.x[u][q * VEC + v] = t16.v[v]; \
        }                                                                     \
      } else {                                                                \
        _Pragma("unroll") for (int t = 0; t < MW; ++t) F.x[u][t] = xrow[m0 + 16 * t + c]; \
      }                                                                       \
    }                                                                         \
    _Pragma("unroll") for (int nt = 0; nt < NT; ++nt) {                       \
      if constexpr (YT) {                                                     \
        const T* yrow = Y + (int64_t)(16 * nt + c) * ldy + (K0) + 4 * g;      \
        _Pragma("unroll") for (int h = 0; h < 4 / VEC; ++h) {                 \
          const V16<T> t_ = load16<T>(yrow + h * VEC);                        \
          _Pragma("unroll") for (int v = 0; v < VEC; ++v) F.y[h * VEC + v][nt] = t_.v[v]; \
        }                                                                     \
      } else {                                                                \
        _Pragma("unroll") for (int u = 0; u < 4; ++u)                         \
          F.y[u][nt] = Y[((K0) + 4 * g + u) * ldy + 16 * nt + c];             \
      }                                                                       \
    }                                                                         \
    if constexpr (NR) {                                                       \
      if constexpr (YT) {                                                     \
        const T* yrow = Y + (int64_t)cr * ldy + (K0) + 4 * g;                 \
        _Pragma("unroll") for (int h = 0; h < 4 / VEC; ++h) {                 \
          const V16<T> t_ = load16<T>(yrow + h * VEC);                        \
          _Pragma("unroll") for (int v = 0; v < VEC; ++v) F.yr[h * VEC + v] = t_.v[v]; \
        }                                                                     \
      } else {                                                                \
        _Pragma("unroll") for (int u = 0; u < 4; ++u)                         \
          F.yr[u] = Y[((K0) + 4 * g + u) * ldy + cr];                         \
      }                                                                       \
    }                                                                         \
  }
#define TN_COMPUTE(F)                                                         \
  {                                                                           \
    _Pragma("unroll") for (int u = 0; u < 4; ++u)                             \
      _Pragma("unroll") for (int t = 0; t < MW; ++t) {                        \
        _Pragma("unroll") for (int nt = 0; nt < NT; ++nt)                     \
          acc[t][nt] = mfma16(F.x[u][t], F.y[u][nt], acc[t][nt]);             \
        if constexpr (NR) accr[t] = mfma4x4(F.x[u][t], F.yr[u], accr[t]);     \
      }                                                                       \
  }

  constexpr int KSTEP = 16;
  int64_t nsteps = (kend - kbeg) / KSTEP;
  if (!full) nsteps = 0;  // everything through the guarded loop below
  NMF_PIPELINE(STAGES, TN_LOAD, TN_COMPUTE, fr, kbeg, nsteps, KSTEP)

  // Guarded remainder, 4 rows at a time (also the whole range for a ragged wave).
  for (int64_t k0 = kbeg + nsteps * KSTEP; k0 < kend; k0 += 4) {
    const int64_t kk = k0 + g;
    const bool okk = kk < kend;
    const int64_t kc = okk ? kk : kbeg;
#pragma unroll
    for (int t = 0; t < MW; ++t) {
      const int64_t col = tn_col<T, VX>(m0, t, c);
      fr[0].x[0][t] = (okk && col < M) ? X[kc * ldx + col] : T(0);
    }
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
      fr[0].y[0][nt] = okk ? (YT ? Y[(int64_t)(16 * nt + c) * ldy + kc] : Y[kc * ldy + 16 * nt + c])
                           : T(0);
    if constexpr (NR) fr[0].yr[0] = okk ? (YT ? Y[(int64_t)cr * ldy + kc] : Y[kc * ldy + cr]) : T(0);
#pragma unroll
    for (int t = 0; t < MW; ++t) {
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) acc[t][nt] = mfma16(fr[0].x[0][t], fr[0].y[0][nt], acc[t][nt]);
      if constexpr (NR) accr[t] = mfma4x4(fr[0].x[0][t], fr[0].yr[0], accr[t]);
    }
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
  if constexpr (NR) {
    // Block b's rows are tile columns 4 (b % 4) + i; sum the four lane groups.
#pragma unroll
    for (int t = 0; t < MW; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        T v = accr[t][r];
        v += __shfl_xor(v, 16, 64);
        v += __shfl_xor(v, 32, 64);
        const int64_t row = tn_col<T, VX>(m0, t, 4 * (lane >> 2) + r);
        if (g == 0 && row < M) {
          Dp[row * ldd + cr] = v;
          for (int z = 16 * NT + 4 + (lane & 3); z < ldd_cols_; z += 4) Dp[row * ldd + z] = T(0);
        }
      }
  }
}

// s += src[p * stride] for p = p0, p0 + step, ... < splits, added in that
// order in double. The loads go out RS_BATCH at a time before any is added,
// so a thread waits for one memory latency per batch rather than per slab.
constexpr int RS_BATCH = 8;
template <typename T>
__device__ __forceinline__ double ordered_sum(const T* __restrict__ src, int p0, int step,
                                              int splits, int64_t stride) {
  double s = 0.0;
  int p = p0;
  for (; p + (RS_BATCH - 1) * step < splits; p += RS_BATCH * step) {
    T v[RS_BATCH];
#pragma unroll
    for (int u = 0; u < RS_BATCH; ++u) v[u] = src[(int64_t)(p + u * step) * stride];
#pragma unroll
    for (int u = 0; u < RS_BATCH; ++u) s += (double)v[u];
  }
  for (; p < splits; p += step) s += (double)src[(int64_t)p * stride];
  return s;
}

// out[i] = sum_s part[s * stride + i] in order s = 0, 1, ... (double sums);
// outt (nullable) receives the transpose, outt[c * rows + r].
template <typename T>
__global__ void reduce_splits_kernel(const T* __restrict__ part, int splits, int64_t stride,
                                     int64_t rows, int cols, int64_t ldo, T* __restrict__ out,
                                     int64_t ldp, T* __restrict__ outt) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  const int64_t r = idx / cols, cc = idx - r * cols;
  const double s = ordered_sum<T>(part + r * ldp + cc, 0, 1, splits, stride);
  out[r * ldo + cc] = (T)s;
  if (outt) outt[cc * rows + r] = (T)s;
}

// Same sums for few outputs and many splits (the k x k Grams): RS_SUB
// threads per output each add every RS_SUB-th slab, then one thread adds the
// RS_SUB partial sums in order. The order is fixed, so results stay bitwise
// reproducible.
constexpr int RS_OUT = 16, RS_SUB = 16;
template <typename T>
__global__ __launch_bounds__(RS_OUT * RS_SUB) void reduce_splits_wide_kernel(
    const T* __restrict__ part, int splits, int64_t stride, int64_t rows, int cols, int64_t ldo,
    T* __restrict__ out, int64_t ldp, T* __restrict__ outt) {
  __shared__ double sh[RS_SUB][RS_OUT];
  const int o = threadIdx.x % RS_OUT, sub = threadIdx.x / RS_OUT;
  const int64_t idx = (int64_t)blockIdx.x * RS_OUT + o;
  const int64_t total = rows * cols;
  const int64_t r = idx / cols, cc = idx - r * cols;
  double s = 0.0;
  if (idx < total) s = ordered_sum<T>(part + r * ldp + cc, sub, RS_SUB, splits, stride);
  sh[sub][o] = s;
  __syncthreads();
  if (sub == 0 && idx < total) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < RS_SUB; ++q) t += sh[q][o];
    out[r * ldo + cc] = (T)t;
    if (outt) outt[cc * rows + r] = (T)t;
  }
}

template <typename T>
hipError_t reduce_splits(const T* part, int splits, int64_t dsplit, int64_t M, int N,
                         int64_t ldd, T* D, int64_t ldp, hipStream_t st, T* Dt) {
  const int64_t total = M * N;
  if (total < 65536 && splits > 16)
    reduce_splits_wide_kernel<T><<<(unsigned)cdiv(total, RS_OUT), RS_OUT * RS_SUB, 0, st>>>(
        part, splits, dsplit, M, N, ldd, D, ldp, Dt);
  else
    reduce_splits_kernel<T><<<(unsigned)cdiv(total, 256), 256, 0, st>>>(part, splits, dsplit, M,
                                                                         N, ldd, D, ldp, Dt);
  return NMF_LAUNCH_CHECK();
}
template hipError_t reduce_splits<float>(const float*, int, int64_t, int64_t, int, int64_t, float*,
                                         int64_t, hipStream_t, float*);
template hipError_t reduce_splits<double>(const double*, int, int64_t, int64_t, int, int64_t,
                                          double*, int64_t, hipStream_t, double*);

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
// Launch shapes, chosen by a timing sweep at m = n = 65536, k = 50 on MI355X:
// for float and ranks up to 64 one wave per SIMD (accumulators in AGPRs) with
// a deep register pipeline is fastest; the TN kernel then takes 128 columns
// of A per wave. Larger ranks and double use two waves per SIMD.
struct Shape { int mw, stages, wpe; };
template <typename T> static constexpr Shape nn_shape(int NT) {
  return sizeof(T) == 4 ? (NT <= 4 ? Shape{4, 6, 1} : Shape{4, 3, 1})
                        : Shape{NT <= 4 ? 4 : 2, 2, 2};
}
template <typename T> static constexpr Shape tn_shape(int NT) {
  return sizeof(T) == 4 ? (NT <= 4 ? Shape{8, 4, 1} : Shape{4, 3, 1})
                        : Shape{NT <= 4 ? 4 : 2, 2, 2};
}
// A float TN product at ranks up to 64 whose streamed operand has under 2^28
// elements (8192 x 4096 at k = 64 in the unrolled-gradient layers) has too
// few 128-column waves to keep a pipeline per SIMD busy; there two waves per
// SIMD of 64 columns each, with a shallower pipeline, took 5% less time per
// product.
constexpr Shape TN_SMALL = {4, 3, 2};
template <typename T> static bool tn_small(int NT, int64_t M, int64_t K) {
  return sizeof(T) == 4 && NT <= 4 && M * K < ((int64_t)1 << 28);
}
constexpr int WAVES = 4;  // waves per workgroup of the product kernels

// Split the reduction until the grid has about one workgroup per CU, keeping
// every split at least 256 long. A small product (under 2^26 multiply-adds,
// such as a 2000 x 1000 matrix at k = 10) may split down to slabs of 64: its
// few output rows would otherwise leave most of the chip idle while each
// wavefront walks a long reduction, and at that size the partials cost
// little. No split is longer than MAX_SPLIT_LEN: the matrix cores add a
// split's products into one float32 accumulator, one rounding per four
// terms, and over 32768 terms (65536^2 at k = 50 with two splits) that
// rounding moved a HALS trajectory by 1.1e-5 relative at its second
// iteration, against 2.4e-7 with splits of 8192 (whose partials are summed in
// double) at 2.6% more time per product. Those extra splits are taken only
// while the partials stay under 2^28 elements (out_elems per split).
constexpr int64_t MAX_SPLIT_LEN = 8192;
static int64_t auto_splits(int64_t wgs, int64_t K, int64_t macs, int64_t out_elems) {
  const int64_t minlen = macs < ((int64_t)1 << 26) ? 64 : 256;
  int64_t s = 1;
  while (wgs * s < 256 && K / (2 * s) >= minlen && s < MAX_PRODUCT_SPLITS) s *= 2;
  while (K > s * MAX_SPLIT_LEN && s < MAX_PRODUCT_SPLITS &&
         2 * s * out_elems <= ((int64_t)1 << 28))
    s *= 2;
  return s;
}

template <typename T, int NT, int NR, bool VX, bool YT>
static void nn_launch(const GemmArgs<T>& a, dim3 grid, int64_t kchunk, T* D, int64_t ldd,
                      int64_t dsplit, hipStream_t st) {
  constexpr Shape sh = nn_shape<T>(NT + NR);
  gemm_nn_kernel<T, NT, sh.mw, VX, YT, sh.stages, sh.wpe, NR><<<grid, 64 * WAVES, 0, st>>>(
      a.X, a.ldx, a.Y, a.ldy, D, ldd, dsplit, a.M, a.K, kchunk, (int)a.N);
}

template <typename T, int NT, int NR>
static hipError_t nn_dispatch(const GemmArgs<T>& a, bool vx, int64_t splits, int64_t kchunk,
                              T* D, int64_t ldd, int64_t dsplit, hipStream_t st) {
  constexpr Shape sh = nn_shape<T>(NT + NR);
  dim3 grid((unsigned)cdiv(a.M, 16 * sh.mw * WAVES), (unsigned)splits);
  if (vx) {
    if (a.yt) nn_launch<T, NT, NR, true, true>(a, grid, kchunk, D, ldd, dsplit, st);
    else nn_launch<T, NT, NR, true, false>(a, grid, kchunk, D, ldd, dsplit, st);
  } else {
    if (a.yt) nn_launch<T, NT, NR, false, true>(a, grid, kchunk, D, ldd, dsplit, st);
    else nn_launch<T, NT, NR, false, false>(a, grid, kchunk, D, ldd, dsplit, st);
  }
  return NMF_LAUNCH_CHECK();
}

template <typename T, int NT, int NR, int MW, int S, int WPE, bool YT>
static hipError_t tn_launch(const GemmArgs<T>& a, bool vx, int waves, int64_t splits,
                            int64_t kchunk, T* D, int64_t ldd, int64_t dsplit, hipStream_t st) {
  dim3 grid((unsigned)cdiv(a.M, 16 * MW * waves), (unsigned)splits);
  if constexpr (MW % Tr<T>::VEC == 0) {
    if (vx) {
      gemm_tn_kernel<T, NT, MW, true, YT, S, WPE, NR><<<grid, 64 * waves, 0, st>>>(
          a.X, a.ldx, a.Y, a.ldy, D, ldd, dsplit, a.M, a.K, kchunk, (int)a.N);
      return NMF_LAUNCH_CHECK();
    }
  }
  gemm_tn_kernel<T, NT, MW, false, YT, S, WPE, NR><<<grid, 64 * waves, 0, st>>>(
      a.X, a.ldx, a.Y, a.ldy, D, ldd, dsplit, a.M, a.K, kchunk, (int)a.N);
  return NMF_LAUNCH_CHECK();
}

template <typename T, int NT, int NR>
static hipError_t tn_dispatch(const GemmArgs<T>& a, bool vx, bool small_m, int64_t splits,
                              int64_t kchunk, T* D, int64_t ldd, int64_t dsplit, hipStream_t st) {
  if constexpr (NR == 0) {
    if (small_m) {
      // Gram: the M side is the padded rank itself; one wave per 16*MW columns.
      constexpr int MW = NT <= 4 ? NT : 4;
      constexpr int MWd = (sizeof(T) == 8 && NT > 4) ? 2 : MW;
      return tn_launch<T, NT, 0, MWd, 2, 2, false>(a, vx, 1, splits, kchunk, D, ldd, dsplit, st);
    }
  }
  if constexpr (sizeof(T) == 4 && NT + NR <= 4) {
    if (tn_small<T>(NT + NR, a.M, a.K)) {
      constexpr Shape sh = TN_SMALL;
      if (a.yt)
        return tn_launch<T, NT, NR, sh.mw, sh.stages, sh.wpe, true>(a, vx, WAVES, splits, kchunk,
                                                                    D, ldd, dsplit, st);
      return tn_launch<T, NT, NR, sh.mw, sh.stages, sh.wpe, false>(a, vx, WAVES, splits, kchunk,
                                                                   D, ldd, dsplit, st);
    }
  }
  constexpr Shape sh = tn_shape<T>(NT + NR);
  if (a.yt)
    return tn_launch<T, NT, NR, sh.mw, sh.stages, sh.wpe, true>(a, vx, WAVES, splits, kchunk, D,
                                                                ldd, dsplit, st);
  return tn_launch<T, NT, NR, sh.mw, sh.stages, sh.wpe, false>(a, vx, WAVES, splits, kchunk, D,
                                                               ldd, dsplit, st);
}

template <typename T>
static int64_t rows_per_wg(GemmKind kind, int NT, int64_t M, int64_t K) {
  const Shape s = kind == GemmKind::NN ? nn_shape<T>(NT)
                  : tn_small<T>(NT, M, K) ? TN_SMALL
                                          : tn_shape<T>(NT);
  return 16 * s.mw * WAVES;
}

template <typename T>
int64_t gemm_auto_splits(GemmKind kind, int64_t M, int64_t N, int64_t K) {
  if (kind == GemmKind::TN_GRAM) return 0;
  return auto_splits(cdiv(M, rows_per_wg<T>(kind, (int)(N / 16), M, K)), K, M * N * K, M * N);
}

static bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

template <typename T>
hipError_t gemm_run(GemmKind kind, const GemmArgs<T>& a_in, int64_t splits, T* part,
                    hipStream_t st, int* nsplit) {
  constexpr int VEC = Tr<T>::VEC;
  GemmArgs<T> a = a_in;
  const int NT = (int)(a.N / 16);
  if (NT < 1 || NT > 8 || a.N % 16 != 0) return hipErrorInvalidValue;
  if (splits < 1) splits = kind == GemmKind::TN_GRAM ? 1 : gemm_auto_splits<T>(kind, a.M, a.N, a.K);
  const int64_t unit = kind == GemmKind::NN ? 4 * VEC : 16;
  int64_t kchunk = round_up(cdiv(a.K, splits), unit);
  splits = cdiv(a.K, kchunk);
  if (splits < 1) splits = 1;
  const bool vx = aligned16(a.X) && (a.ldx % VEC == 0);
  // A transposed Y is only read with 16-byte loads; otherwise use it as given.
  if (a.yt && !(aligned16(a.Y) && a.ldy % VEC == 0)) return hipErrorInvalidValue;
  const bool small_m = kind == GemmKind::TN_GRAM;
  if (small_m) a.yt = false;
  // a transposed copy is written by the reduction, so a Gram that wants one
  // goes through it even unsplit
  if (a.Dt && !small_m) return hipErrorInvalidValue;
  const bool reduce = splits > 1 || a.Dt;
  T* D = reduce ? part : a.D;
  const int64_t ldd = reduce ? a.N : a.ldd;
  const int64_t dsplit = a.M * a.N;
  // Rank remainder: float, not a Gram, and the valid columns end 1..4 past a
  // multiple of 16 (the rest of the padded tile is zero).
  const int nvalid = a.nvalid > 0 ? a.nvalid : (int)a.N;
  const bool rem = sizeof(T) == 4 && !small_m && nvalid > 16 && nvalid % 16 >= 1 &&
                   nvalid % 16 <= 4;
  const int NTf = rem ? nvalid / 16 : NT;
  hipError_t e = hipSuccess;
#define NT_CASE(n)                                                                        \
  case n:                                                                                 \
    if (rem) {                                                                            \
      if constexpr (sizeof(T) == 4)                                                       \
        e = kind == GemmKind::NN                                                          \
                ? nn_dispatch<T, n, 1>(a, vx, splits, kchunk, D, ldd, dsplit, st)         \
                : tn_dispatch<T, n, 1>(a, vx, small_m, splits, kchunk, D, ldd, dsplit, st); \
    } else {                                                                              \
      e = kind == GemmKind::NN                                                            \
              ? nn_dispatch<T, n, 0>(a, vx, splits, kchunk, D, ldd, dsplit, st)           \
              : tn_dispatch<T, n, 0>(a, vx, small_m, splits, kchunk, D, ldd, dsplit, st); \
    }                                                                                     \
    break;
  switch (NTf) {
    NT_CASE(1) NT_CASE(2) NT_CASE(3) NT_CASE(4) NT_CASE(5) NT_CASE(6) NT_CASE(7) NT_CASE(8)
    default: return hipErrorInvalidValue;
  }
#undef NT_CASE
  if (nsplit) *nsplit = (int)splits;
  if (e != hipSuccess || !reduce || nsplit) return e;
  return reduce_splits<T>(part, (int)splits, dsplit, a.M, (int)a.N, a.ldd, a.D, a.N, st, a.Dt);
}

template int64_t gemm_auto_splits<float>(GemmKind, int64_t, int64_t, int64_t);
template int64_t gemm_auto_splits<double>(GemmKind, int64_t, int64_t, int64_t);
template hipError_t gemm_run<float>(GemmKind, const GemmArgs<float>&, int64_t, float*, hipStream_t,
                                    int*);
template hipError_t gemm_run<double>(GemmKind, const GemmArgs<double>&, int64_t, double*,
                                     hipStream_t, int*);

}  // namespace nmfk
