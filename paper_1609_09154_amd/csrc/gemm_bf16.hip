// BF16 products for dense A stored in bfloat16: P = A H^T and R = A^T W of
// Algorithm 1 on the gfx950 BF16 matrix cores with float accumulation; the
// factors stay float and are rounded to bfloat16 (round to nearest even) into
// a packed, transposed copy before each product.
//
// Both products are computed as D (M x N, float) = X (M x K) Y (N x K)^T with
// X and Y bfloat16 and K contiguous in both: X is A (or its transposed copy)
// and Y is the packed factor (k x K). That is the native operand layout of
// v_mfma_f32_16x16x32_bf16 (lane l supplies row l % 16, eight consecutive K
// values starting at 8 (l / 16), for both operands), so the matrix is
// streamed with 16-byte loads straight into MFMA operands.
//
// At rank k the product does k flops per byte of A, far below the BF16 ridge
// of the chip, so the kernel is built to keep HBM busy: A is read once with
// non-temporal loads, several K steps deep; the factor slice of each K step
// (N rows x 64 values) is loaded once per workgroup into LDS and shared by its
// four waves.
#include "common.h"
#include "kernels.h"

namespace nmfk {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mfma_bf16(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x8 as_bf16x8(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }

// bfloat16 bits of x, rounded to nearest even (NaN stays a quiet NaN).
__device__ __forceinline__ uint16_t to_bf16_rne(float x) {
  const unsigned u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

constexpr int BK = 64;         // K values per step (two MFMAs per tile)
constexpr int BWAVES = 4;      // waves per workgroup
constexpr int YLD = BK + 8;    // LDS row pitch of the factor slice (bf16 units)

// Lane (g = l / 16, c = l % 16) of a wave reads, for each of its row tiles,
// the 32 bytes X[row][k0 + 16 g .. k0 + 16 g + 15]: elements 0..7 feed the
// first MFMA of the step and 8..15 the second. The same K permutation is
// applied to the factor operand, so the sum is unchanged.
template <int MT> struct XFrag { u32x4 v[MT][2]; };

// NT 16-column tiles (N = 16 NT), MT 16-row tiles per wave, STAGES K steps
// of X in registers (STAGES - 1 in flight while one is multiplied), WPE
// waves per SIMD to leave room for (the register budget follows from it).
template <int NT, int MT, int STAGES, int WPE>
__global__ __launch_bounds__(64 * BWAVES, WPE) void gemm_bf16_nt_kernel(
    const uint16_t* __restrict__ X, int64_t ldx, const uint16_t* __restrict__ Y, int64_t ldy,
    float* __restrict__ D, int64_t ldd, int64_t dsplit, int64_t M, int64_t K, int64_t kchunk) {
  constexpr int NR = 16 * NT;               // factor rows (the padded rank)
  constexpr int YCH = BK / 8;               // 16-byte chunks per factor row per step
  constexpr int YRP = 256 / YCH;            // factor rows staged per pass
  constexpr int YPASS = (NR + YRP - 1) / YRP;
  // LDS rows NR..YPASS*YRP-1 take the copies of the last pass past the
  // factor's end (their global row is clamped): no branch in the staging.
  __shared__ __attribute__((aligned(16))) uint16_t Ys[2][YPASS * YRP * YLD];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, c = lane & 15;
  const int64_t m0 = (int64_t)blockIdx.x * (16 * MT * BWAVES) + wave * 16 * MT;
  const int64_t kbeg = (int64_t)blockIdx.y * kchunk;
  const int64_t kend = kbeg + kchunk < K ? kbeg + kchunk : K;
  D += (int64_t)blockIdx.y * dsplit;

  const uint16_t* xr[MT];
#pragma unroll
  for (int t = 0; t < MT; ++t) {
    int64_t row = m0 + 16 * t + c;
    row = row < M ? row : M - 1;
    xr[t] = X + row * ldx + 16 * g;
  }
  // factor staging: thread tid copies chunk (tid % YCH) of rows tid / YCH + 32 p
  const int ych = tid % YCH, yrow0 = tid / YCH;

  f32x4 acc[MT][NT];
#pragma unroll
  for (int t = 0; t < MT; ++t)
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[t][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  const int64_t nfull = (kend - kbeg) / BK;
  XFrag<MT> xf[STAGES];
  u32x4 yv[2][YPASS];  // factor slices of the next two steps, in registers

  auto load_x = [&](XFrag<MT>& f, int64_t k0) {
#pragma unroll
    for (int t = 0; t < MT; ++t) {
      f.v[t][0] = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(xr[t] + k0));
      f.v[t][1] = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(xr[t] + k0 + 8));
    }
  };
  auto load_y = [&](u32x4 (&v)[YPASS], int64_t k0) {
#pragma unroll
    for (int p = 0; p < YPASS; ++p) {
      const int r = yrow0 + p * YRP;
      const int rg = r < NR ? r : NR - 1;
      v[p] = *reinterpret_cast<const u32x4*>(Y + (int64_t)rg * ldy + k0 + 8 * ych);
    }
  };
  auto store_y = [&](const u32x4 (&v)[YPASS], int buf) {
#pragma unroll
    for (int p = 0; p < YPASS; ++p) {
      const int r = yrow0 + p * YRP;
      *reinterpret_cast<u32x4*>(&Ys[buf][r * YLD + 8 * ych]) = v[p];
    }
  };
  auto compute = [&](const XFrag<MT>& f, int buf) {
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      const uint16_t* yp = &Ys[buf][(16 * j + c) * YLD + 16 * g];
      const bf16x8 b0 = as_bf16x8(*reinterpret_cast<const u32x4*>(yp));
      const bf16x8 b1 = as_bf16x8(*reinterpret_cast<const u32x4*>(yp + 8));
#pragma unroll
      for (int t = 0; t < MT; ++t) {
        acc[t][j] = mfma_bf16(as_bf16x8(f.v[t][0]), b0, acc[t][j]);
        acc[t][j] = mfma_bf16(as_bf16x8(f.v[t][1]), b1, acc[t][j]);
      }
    }
  };

  // Memory loads complete in issue order as far as the wait counter is
  // concerned, so each step issues the factor slice it will need two steps
  // later before the matrix rows it will need STAGES - 1 steps later: the
  // slice written to LDS at the end of a step was issued a full step earlier,
  // ahead of the newest row loads, and waiting for it leaves those in flight.
  static_assert(STAGES % 2 == 0, "the unrolled ring also indexes the two factor slices");
  if (nfull > 0) {
    load_y(yv[0], kbeg);
#pragma unroll
    for (int s = 0; s < STAGES - 1; ++s)
      if (s < nfull) load_x(xf[s], kbeg + s * BK);
    if (nfull > 1) load_y(yv[1], kbeg + BK);
    store_y(yv[0], 0);
    __syncthreads();
    // Steady state: every prefetch is in range, so the unrolled body has no
    // branch between a load and its use and the wait counts stay exact.
    // STAGES is even, so ring and buffer indices are constants.
    constexpr int AHEAD = STAGES - 1 > 2 ? STAGES - 1 : 2;
    int64_t s = 0;
    for (; s + STAGES + AHEAD <= nfull; s += STAGES) {
#pragma unroll
      for (int u = 0; u < STAGES; ++u) {
        const int64_t st = s + u;
        load_y(yv[u & 1], kbeg + (st + 2) * BK);
        load_x(xf[(u + STAGES - 1) % STAGES], kbeg + (st + STAGES - 1) * BK);
        // keep the prefetches ahead of this step's matrix-core work
        __builtin_amdgcn_sched_barrier(0);
        compute(xf[u], u & 1);
        store_y(yv[(u + 1) & 1], (u + 1) & 1);
        __syncthreads();
      }
    }
    // Drain: the last steps, with the loads past the end skipped.
    for (; s < nfull; s += STAGES) {
#pragma unroll
      for (int u = 0; u < STAGES; ++u) {
        const int64_t st = s + u;
        if (st < nfull) {
          if (st + 2 < nfull) load_y(yv[u & 1], kbeg + (st + 2) * BK);
          const int64_t pre = st + STAGES - 1;
          if (pre < nfull) load_x(xf[(u + STAGES - 1) % STAGES], kbeg + pre * BK);
          compute(xf[u], u & 1);
          if (st + 1 < nfull) store_y(yv[(u + 1) & 1], (u + 1) & 1);
          __syncthreads();
        }
      }
    }
  }
  // K tail (fewer than BK values left): element loads, zero beyond kend
  const int64_t kt = kbeg + nfull * BK;
  if (kt < kend) {
    XFrag<MT> f;
#pragma unroll
    for (int t = 0; t < MT; ++t)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        unsigned w[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          // xr[t] already points at K offset 16 g of its row
          const int64_t kk = kt + 16 * g + 8 * h + 2 * q;
          const unsigned lo = kk < kend ? xr[t][kt + 8 * h + 2 * q] : 0u;
          const unsigned hi = kk + 1 < kend ? xr[t][kt + 8 * h + 2 * q + 1] : 0u;
          w[q] = lo | (hi << 16);
        }
        f.v[t][h] = u32x4{w[0], w[1], w[2], w[3]};
      }
    for (int e = tid; e < NR * BK; e += 64 * BWAVES) {
      const int r = e / BK, kk = e % BK;
      Ys[0][r * YLD + kk] = (kt + kk < kend) ? Y[(int64_t)r * ldy + kt + kk] : (uint16_t)0;
    }
    __syncthreads();
    compute(f, 0);
  }
  // store: element r of tile (t, j) is row 4 g + r, column c
#pragma unroll
  for (int t = 0; t < MT; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = m0 + 16 * t + 4 * g + r;
      if (row < M) {
#pragma unroll
        for (int j = 0; j < NT; ++j) D[row * ldd + 16 * j + c] = acc[t][j][r];
      }
    }
}

// Ft (KP x rows, row pitch ldt) = bfloat16(F^T) for F rows x KP float.
__global__ __launch_bounds__(256) void pack_bf16_t_kernel(const float* __restrict__ F,
                                                         int64_t rows, int KP,
                                                         uint16_t* __restrict__ Ft, int64_t ldt) {
  __shared__ float tile[32][33];
  const int64_t r0 = (int64_t)blockIdx.x * 32;
  const int c0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int i = ty; i < 32; i += 8) {
    const int64_t r = r0 + i;
    const int cc = c0 + tx;
    tile[i][tx] = (r < rows && cc < KP) ? F[r * KP + cc] : 0.f;
  }
  __syncthreads();
  for (int i = ty; i < 32; i += 8) {
    const int cc = c0 + i;
    const int64_t r = r0 + tx;
    if (cc < KP && r < rows) Ft[(int64_t)cc * ldt + r] = to_bf16_rne(tile[tx][i]);
  }
}

hipError_t pack_bf16_t(const float* F, int64_t rows, int KP, uint16_t* Ft, int64_t ldt,
                       hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  dim3 grid((unsigned)cdiv(rows, 32), (unsigned)cdiv(KP, 32));
  pack_bf16_t_kernel<<<grid, 256, 0, st>>>(F, rows, KP, Ft, ldt);
  return NMF_LAUNCH_CHECK();
}

constexpr int B_MT = 4, B_STAGES = 4, B_WPE = 1;  // launch shape (timing sweep at 131072 x 65536, k = 100)
constexpr int BROWS = 16 * B_MT * BWAVES;

int64_t gemm_bf16_splits(int64_t M, int64_t K) {
  const int64_t blocks = cdiv(M, BROWS);
  int64_t s = 1;
  while (blocks * s < 256 && K / (2 * s) >= 16 * BK && s < 16) s *= 2;
  return s;
}

hipError_t gemm_bf16_nt(const uint16_t* X, int64_t ldx, const uint16_t* Y, int64_t ldy, float* D,
                        int64_t ldd, int64_t M, int N, int64_t K, float* part, hipStream_t st) {
  if (M <= 0) return hipSuccess;
  if (N % 16 != 0 || N > 128 || ldx % 8 != 0 || ldy % 8 != 0) return hipErrorInvalidValue;
  const int64_t splits = gemm_bf16_splits(M, K);
  const int64_t kchunk = round_up(cdiv(K, splits), BK);
  const int64_t nsplit = cdiv(K, kchunk);
  float* out = nsplit > 1 ? part : D;
  const int64_t ldo = nsplit > 1 ? N : ldd;
  const int64_t dsplit = (int64_t)M * N;
  dim3 grid((unsigned)cdiv(M, BROWS), (unsigned)nsplit);
  const int NT = N / 16;
#define CASE(J)                                                                            \
  case J:                                                                                  \
    gemm_bf16_nt_kernel<J, B_MT, B_STAGES, B_WPE><<<grid, 64 * BWAVES, 0, st>>>(          \
        X, ldx, Y, ldy, out, ldo, dsplit, M, K, kchunk);                                   \
    break;
  switch (NT) {
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
    default: return hipErrorInvalidValue;
  }
#undef CASE
  hipError_t e = NMF_LAUNCH_CHECK();
  if (e != hipSuccess || nsplit == 1) return e;
  return reduce_splits<float>(part, (int)nsplit, dsplit, M, N, ldd, D, N, st);
}

}  // namespace nmfk
