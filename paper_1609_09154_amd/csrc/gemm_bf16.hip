// Reduced-precision products for dense A: P = A H^T and R = A^T W of
// Algorithm 1 on the gfx950 matrix cores with float accumulation, for A
// stored in bfloat16 or in FP8 E4M3. The factors stay float; before each
// product the factor operand is packed, transposed, into the same format
// (round to nearest even): bfloat16 directly; FP8 after dividing each rank
// column by the smallest power of two that brings its largest entry to at
// most 448 (the E4M3 maximum), the power being multiplied back into that
// output column.
//
// Both products are computed as D (M x N, float) = X (M x K) Y (N x K)^T with
// X and Y in the reduced format and K contiguous in both: X is A (or its
// transposed copy) and Y is the packed factor. Each K step covers 128 bytes of
// a row; lane (g = l / 16, c = l % 16) of a wave reads bytes 32 g .. 32 g + 31
// of that step of row c of each of its row tiles, with two 16-byte loads. For
// FP8 those 32 values are the operand of v_mfma_scale_f32_16x16x128_f8f6f4
// (lane l: row l % 16, K values 32 (l / 16) .. + 31). For bfloat16 they feed
// two v_mfma_f32_16x16x32_bf16 (lane l: row l % 16, eight K values from
// 8 (l / 16)): values 0..7 the first, 8..15 the second; the factor operand
// gets the same K permutation, so the sum is unchanged.
//
// At rank k the product does k (bfloat16) or 2k (FP8) flops per byte of A,
// far below the ridge of either format, so the kernel is built to keep HBM
// busy: A is read once with non-temporal loads, several K steps deep; the
// factor slice of each K step (N rows x 128 bytes) is loaded once per
// workgroup into LDS and shared by its four waves.
#include "common.h"
#include "kernels.h"

namespace nmfk {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ bf16x8 as_bf16x8(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }

__device__ __forceinline__ i32x8 join32(u32x4 a, u32x4 b) {
  return __builtin_bit_cast(i32x8, __builtin_shufflevector(a, b, 0, 1, 2, 3, 4, 5, 6, 7));
}

// bfloat16 bits of x, rounded to nearest even (NaN stays a quiet NaN).
__device__ __forceinline__ uint16_t to_bf16_rne(float x) {
  const unsigned u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// FP8 E4M3 bits of x (sign, 4 exponent bits with bias 7, 3 fraction bits;
// largest finite 448, no infinities), rounded to nearest even and saturating
// at 448. |x| is rounded to a multiple of its binade's spacing (2^(e-3) for
// 2^e <= |x| < 2^(e+1), e >= -6, and 2^-9 below 2^-6); the scalings by powers
// of two are exact, so the only rounding is the one to an integer.
__device__ __forceinline__ uint8_t to_fp8_e4m3_rne(float x) {
  const unsigned sgn = (__float_as_uint(x) >> 24) & 0x80u;
  const float a = fabsf(x);
  if (!(a == a)) return 0x7f;
  if (a >= 448.f) return (uint8_t)(sgn | 0x7eu);
  int e = (int)((__float_as_uint(a) >> 23) & 0xffu) - 127;
  e = e < -6 ? -6 : e;
  const float q = rintf(ldexpf(a, 3 - e));     // multiples of 2^(e-3)
  if (q == 0.f) return (uint8_t)sgn;
  if (e == -6 && q < 8.f) return (uint8_t)(sgn | (unsigned)q);  // subnormal: q 2^-9
  // q in [8, 16]: 16 carries into the next binade
  const int qi = (int)q;
  const int ee = qi == 16 ? e + 1 : e;
  const int f = qi == 16 ? 0 : qi - 8;
  return (uint8_t)(sgn | ((unsigned)(ee + 7) << 3) | (unsigned)f);
}

constexpr int SB = 128;        // bytes of each row per K step
constexpr int BWAVES = 4;      // waves per workgroup

template <int MT> struct XFrag { u32x4 v[MT][2]; };

// TE: stored element (uint16_t bfloat16 bits or uint8_t FP8 E4M3 bits).
// NT 16-column tiles (N = 16 NT), MT 16-row tiles per wave, STAGES K steps of
// X in registers (STAGES - 1 in flight while one is multiplied), WPE waves per
// SIMD to leave room for. FP8 outputs: column j is multiplied by colscale[j].
template <typename TE, int NT, int MT, int STAGES, int WPE>
__global__ __launch_bounds__(64 * BWAVES, WPE) void gemm_lp_nt_kernel(
    const TE* __restrict__ X, int64_t ldx, const TE* __restrict__ Y, int64_t ldy,
    const float* __restrict__ colscale, float* __restrict__ D, int64_t ldd, int64_t dsplit,
    int64_t M, int64_t K, int64_t kchunk) {
  constexpr bool FP8 = sizeof(TE) == 1;
  constexpr int BK = SB / (int)sizeof(TE);    // K values per step
  constexpr int LE = 32 / (int)sizeof(TE);    // K values per lane per step
  constexpr int VE = 16 / (int)sizeof(TE);    // K values per 16-byte load
  constexpr int YLD = BK + VE;                // LDS row pitch (16 bytes of padding)
  constexpr int NR = 16 * NT;                 // factor rows (the padded rank)
  constexpr int YCH = SB / 16;                // 16-byte chunks per factor row per step
  constexpr int YRP = 256 / YCH;              // factor rows staged per pass
  constexpr int YPASS = (NR + YRP - 1) / YRP;
  // LDS rows NR..YPASS*YRP-1 take the copies of the last pass past the
  // factor's end (their global row is clamped): no branch in the staging.
  __shared__ __attribute__((aligned(16))) TE Ys[2][YPASS * YRP * YLD];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, c = lane & 15;
  const int64_t m0 = (int64_t)blockIdx.x * (16 * MT * BWAVES) + wave * 16 * MT;
  const int64_t kbeg = (int64_t)blockIdx.y * kchunk;
  const int64_t kend = kbeg + kchunk < K ? kbeg + kchunk : K;
  D += (int64_t)blockIdx.y * dsplit;

  const TE* xr[MT];
#pragma unroll
  for (int t = 0; t < MT; ++t) {
    int64_t row = m0 + 16 * t + c;
    row = row < M ? row : M - 1;
    xr[t] = X + row * ldx + LE * g;
  }
  // factor staging: thread tid copies chunk (tid % YCH) of rows tid / YCH + YRP p
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
      f.v[t][1] = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(xr[t] + k0 + VE));
    }
  };
  auto load_y = [&](u32x4 (&v)[YPASS], int64_t k0) {
#pragma unroll
    for (int p = 0; p < YPASS; ++p) {
      const int r = yrow0 + p * YRP;
      const int rg = r < NR ? r : NR - 1;
      v[p] = *reinterpret_cast<const u32x4*>(Y + (int64_t)rg * ldy + k0 + VE * ych);
    }
  };
  auto store_y = [&](const u32x4 (&v)[YPASS], int buf) {
#pragma unroll
    for (int p = 0; p < YPASS; ++p) {
      const int r = yrow0 + p * YRP;
      *reinterpret_cast<u32x4*>(&Ys[buf][r * YLD + VE * ych]) = v[p];
    }
  };
  auto compute = [&](const XFrag<MT>& f, int buf) {
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      const TE* yp = &Ys[buf][(16 * j + c) * YLD + LE * g];
      const u32x4 b0 = *reinterpret_cast<const u32x4*>(yp);
      const u32x4 b1 = *reinterpret_cast<const u32x4*>(yp + VE);
#pragma unroll
      for (int t = 0; t < MT; ++t) {
        if constexpr (FP8) {
          // operand formats 0 (E4M3) and no block scales: a plain FP8 product
          acc[t][j] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(
              join32(f.v[t][0], f.v[t][1]), join32(b0, b1), acc[t][j], 0, 0, 0, 0, 0, 0);
        } else {
          acc[t][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(f.v[t][0]),
                                                              as_bf16x8(b0), acc[t][j], 0, 0, 0);
          acc[t][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(f.v[t][1]),
                                                              as_bf16x8(b1), acc[t][j], 0, 0, 0);
        }
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
    for (int t = 0; t < MT; ++t) {
      TE e[LE];
#pragma unroll
      for (int q = 0; q < LE; ++q) {
        // xr[t] already points at K offset LE g of its row
        e[q] = kt + LE * g + q < kend ? xr[t][kt + q] : (TE)0;
      }
      u32x4 w[2];
      __builtin_memcpy(w, e, sizeof(w));
      f.v[t][0] = w[0];
      f.v[t][1] = w[1];
    }
    for (int e = tid; e < NR * BK; e += 64 * BWAVES) {
      const int r = e / BK, kk = e % BK;
      Ys[0][r * YLD + kk] = (kt + kk < kend) ? Y[(int64_t)r * ldy + kt + kk] : (TE)0;
    }
    __syncthreads();
    compute(f, 0);
  }
  // store: element r of tile (t, j) is row 4 g + r, column c
  float cs[NT];
#pragma unroll
  for (int j = 0; j < NT; ++j) cs[j] = FP8 ? colscale[16 * j + c] : 1.f;
#pragma unroll
  for (int t = 0; t < MT; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = m0 + 16 * t + 4 * g + r;
      if (row < M) {
#pragma unroll
        for (int j = 0; j < NT; ++j)
          D[row * ldd + 16 * j + c] = FP8 ? acc[t][j][r] * cs[j] : acc[t][j][r];
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

// FP8 packing, pass 1: maxbits[j] = bits of max_r |F[r][j]| (non-negative
// floats order like their bit patterns), KP a multiple of 4 up to 128;
// maxbits starts at 0. Thread (ty, c) of a block reads 16-byte chunks c of
// rows ty, ty + R, ... of the block's slices (R = 256 / (KP / 4) rows per
// pass, four passes in flight), the block reduces its maxima in LDS and
// raises each column's word once.
__global__ __launch_bounds__(256) void colmax_kernel(const float* __restrict__ F, int64_t rows,
                                                     int KP, unsigned* __restrict__ maxbits) {
  __shared__ unsigned part[256 * 4];
  const int q = KP / 4;           // float4 chunks per row
  const int R = 256 / q;          // rows per pass
  const int tid = threadIdx.x;
  const int c = tid % q, ty = tid / q;
  unsigned mx[4] = {0u, 0u, 0u, 0u};
  if (ty < R) {
    const int64_t stride = (int64_t)gridDim.x * R;
    for (int64_t r0 = (int64_t)blockIdx.x * R + ty; r0 < rows; r0 += 4 * stride) {
      f32x4 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t r = r0 + u * stride;
        v[u] = r < rows ? *reinterpret_cast<const f32x4*>(F + r * KP + 4 * c)
                        : f32x4{0.f, 0.f, 0.f, 0.f};
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int e = 0; e < 4; ++e) mx[e] = max(mx[e], __float_as_uint(fabsf(v[u][e])));
    }
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) part[tid * 4 + e] = mx[e];
  __syncthreads();
  if (tid < KP) {
    // column tid is element tid % 4 of chunk tid / 4, held by threads ty q + tid / 4
    unsigned m = 0;
    for (int t = 0; t < R; ++t) m = max(m, part[(t * q + tid / 4) * 4 + tid % 4]);
    if (m) atomicMax(&maxbits[tid], m);
  }
}

__global__ void zero_u32_kernel(unsigned* __restrict__ p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// Exponent p of the column scale 2^p: the smallest integer with
// 448 2^p >= mx (0 for mx = 0). With mx = f 2^E, f in [0.5, 1), and
// 448 = 0.875 2^9: p = E - 9 if f <= 0.875, else E - 8. No rounding.
__device__ __forceinline__ int fp8_col_exp(unsigned maxbits) {
  const float mx = __uint_as_float(maxbits);
  if (!(mx > 0.f)) return 0;
  int E;
  const float f = frexpf(mx, &E);
  return f <= 0.875f ? E - 9 : E - 8;
}

// Pass 2: Ft (KP x rows, pitch ldt) = FP8(F^T / 2^p_j), colscale[j] = 2^p_j.
__global__ __launch_bounds__(256) void pack_fp8_t_kernel(const float* __restrict__ F,
                                                        int64_t rows, int KP,
                                                        const unsigned* __restrict__ maxbits,
                                                        uint8_t* __restrict__ Ft, int64_t ldt,
                                                        float* __restrict__ colscale) {
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
    if (cc < KP && r < rows)
      Ft[(int64_t)cc * ldt + r] = to_fp8_e4m3_rne(ldexpf(tile[tx][i], -fp8_col_exp(maxbits[cc])));
  }
  if (blockIdx.x == 0 && blockIdx.y == 0)
    for (int j = threadIdx.x; j < KP; j += blockDim.x)
      colscale[j] = ldexpf(1.f, fp8_col_exp(maxbits[j]));
}

hipError_t pack_bf16_t(const float* F, int64_t rows, int KP, uint16_t* Ft, int64_t ldt,
                       hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  dim3 grid((unsigned)cdiv(rows, 32), (unsigned)cdiv(KP, 32));
  pack_bf16_t_kernel<<<grid, 256, 0, st>>>(F, rows, KP, Ft, ldt);
  return NMF_LAUNCH_CHECK();
}

hipError_t pack_fp8_t(const float* F, int64_t rows, int KP, uint8_t* Ft, int64_t ldt,
                      float* colscale, unsigned* maxbits, hipStream_t st) {
  if (KP < 4 || KP > 128 || KP % 4 != 0) return hipErrorInvalidValue;
  zero_u32_kernel<<<1, 128, 0, st>>>(maxbits, KP);
  if (rows > 0) {
    const int R = 256 / (KP / 4);
    const int64_t want = cdiv(rows, 4 * R), blocks = want < 1024 ? want : 1024;
    colmax_kernel<<<(unsigned)blocks, 256, 0, st>>>(F, rows, KP, maxbits);
    dim3 grid((unsigned)cdiv(rows, 32), (unsigned)cdiv(KP, 32));
    pack_fp8_t_kernel<<<grid, 256, 0, st>>>(F, rows, KP, maxbits, Ft, ldt, colscale);
  }
  return NMF_LAUNCH_CHECK();
}

constexpr int B_MT = 4, B_STAGES = 4, B_WPE = 1;  // launch shape (timing sweep at 131072 x 65536, k = 100)
constexpr int BROWS = 16 * B_MT * BWAVES;

int64_t gemm_lp_splits(int64_t M, int64_t K) {
  const int64_t blocks = cdiv(M, BROWS);
  int64_t s = 1;
  while (blocks * s < 256 && K / (2 * s) >= 1024 && s < 16) s *= 2;
  return s;
}

template <typename TE>
static hipError_t gemm_lp_nt(const TE* X, int64_t ldx, const TE* Y, int64_t ldy,
                             const float* colscale, float* D, int64_t ldd, int64_t M, int N,
                             int64_t K, float* part, hipStream_t st) {
  constexpr int VE = 16 / (int)sizeof(TE);
  constexpr int BK = SB / (int)sizeof(TE);
  if (M <= 0) return hipSuccess;
  if (N % 16 != 0 || N < 16 || N > 128 || ldx % VE != 0 || ldy % VE != 0)
    return hipErrorInvalidValue;
  const int64_t splits = gemm_lp_splits(M, K);
  const int64_t kchunk = round_up(cdiv(K, splits), BK);
  const int64_t nsplit = cdiv(K, kchunk);
  float* out = nsplit > 1 ? part : D;
  const int64_t ldo = nsplit > 1 ? N : ldd;
  const int64_t dsplit = (int64_t)M * N;
  dim3 grid((unsigned)cdiv(M, BROWS), (unsigned)nsplit);
  const int NT = N / 16;
#define CASE(J)                                                                            \
  case J:                                                                                  \
    gemm_lp_nt_kernel<TE, J, B_MT, B_STAGES, B_WPE><<<grid, 64 * BWAVES, 0, st>>>(         \
        X, ldx, Y, ldy, colscale, out, ldo, dsplit, M, K, kchunk);                         \
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

hipError_t gemm_bf16_nt(const uint16_t* X, int64_t ldx, const uint16_t* Y, int64_t ldy, float* D,
                        int64_t ldd, int64_t M, int N, int64_t K, float* part, hipStream_t st) {
  return gemm_lp_nt<uint16_t>(X, ldx, Y, ldy, nullptr, D, ldd, M, N, K, part, st);
}

hipError_t gemm_fp8_nt(const uint8_t* X, int64_t ldx, const uint8_t* Y, int64_t ldy,
                       const float* colscale, float* D, int64_t ldd, int64_t M, int N, int64_t K,
                       float* part, hipStream_t st) {
  if (!colscale) return hipErrorInvalidValue;
  return gemm_lp_nt<uint8_t>(X, ldx, Y, ldy, colscale, D, ldd, M, N, K, part, st);
}

}  // namespace nmfk
