// Shared device helpers for the gfx950 NMF kernels: element traits, the
// 16x16x4 MFMA wrappers and the launch helpers used by every kernel file.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nmf.h"

namespace nmfk {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// Per-type traits. VEC is the number of elements in one 16-byte load.
template <typename T> struct Tr;
template <> struct Tr<float> {
  static constexpr int VEC = 4;
  typedef f32x4 acc4;   // 16x16 MFMA accumulator fragment (4 per lane)
};
template <> struct Tr<double> {
  static constexpr int VEC = 2;
  typedef f64x4 acc4;
};

// D(16x16) += A(16x4) B(4x16).  Operand lane layout (both types): lane l
// supplies A[l % 16][l / 16] and B[l / 16][l % 16].
__device__ __forceinline__ f32x4 mfma16(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mfma16(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// 16 independent 4x4 blocks, k = 1: block b = l / 4 takes A_b[i] from lane
// 4b + i and B_b[j] from lane 4b + j; lane 4b + j holds D_b[r][j] in element r.
__device__ __forceinline__ f32x4 mfma4x4(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 0, 0, 0);
}

// Row of the 16x16 output held by lane `lane` in accumulator element `r`.
// f32: lane l holds rows 4*(l/16) + r; f64: rows 4*r + l/16. Column is l % 16.
template <typename T> __device__ __forceinline__ int acc_row(int lane, int r);
template <> __device__ __forceinline__ int acc_row<float>(int lane, int r) {
  return 4 * (lane >> 4) + r;
}
template <> __device__ __forceinline__ int acc_row<double>(int lane, int r) {
  return 4 * r + (lane >> 4);
}

template <typename T> __device__ __forceinline__ typename Tr<T>::acc4 zero4() {
  typename Tr<T>::acc4 z;
  z[0] = 0; z[1] = 0; z[2] = 0; z[3] = 0;
  return z;
}

// 16-byte vector of T.
template <typename T> struct V16 { T v[Tr<T>::VEC]; };

template <typename T>
__device__ __forceinline__ V16<T> load16(const T* p) {
  V16<T> r;
  if constexpr (sizeof(T) == 4) {
    float4 t = *reinterpret_cast<const float4*>(p);
    r.v[0] = t.x; r.v[1] = t.y; r.v[2] = t.z; r.v[3] = t.w;
  } else {
    double2 t = *reinterpret_cast<const double2*>(p);
    r.v[0] = t.x; r.v[1] = t.y;
  }
  return r;
}

// Non-temporal 16-byte load for data streamed exactly once (the large A).
template <typename T>
__device__ __forceinline__ V16<T> load16_stream(const T* p) {
  V16<T> r;
  if constexpr (sizeof(T) == 4) {
    f32x4 t = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(p));
    r.v[0] = t[0]; r.v[1] = t[1]; r.v[2] = t[2]; r.v[3] = t[3];
  } else {
    typedef double f64x2 __attribute__((ext_vector_type(2)));
    f64x2 t = __builtin_nontemporal_load(reinterpret_cast<const f64x2*>(p));
    r.v[0] = t[0]; r.v[1] = t[1];
  }
  return r;
}

// bfloat16 and FP8 E4M3 values are carried as their bits (uint16_t, uint8_t)
// outside the matrix-core operands. to_double widens any stored element type.
__device__ __forceinline__ float bf16_bits_to_float(uint16_t b) {
  return __uint_as_float((unsigned)b << 16);
}
// E4M3: exponent field e (bias 7), fraction f: (8 + f) 2^(e - 10) for e > 0,
// f 2^-9 for e = 0; all ones (S.1111.111) is NaN.
__device__ __forceinline__ float fp8_e4m3_bits_to_float(uint8_t b) {
  const int e = (b >> 3) & 15, f = b & 7;
  float v = e ? ldexpf((float)(8 + f), e - 10) : ldexpf((float)f, -9);
  if (e == 15 && f == 7) v = __builtin_nanf("");
  return (b & 0x80) ? -v : v;
}
__device__ __forceinline__ double to_double(float x) { return (double)x; }
__device__ __forceinline__ double to_double(double x) { return x; }
__device__ __forceinline__ double to_double(uint16_t x) { return (double)bf16_bits_to_float(x); }
__device__ __forceinline__ double to_double(uint8_t x) { return (double)fp8_e4m3_bits_to_float(x); }

// Sum over groups of G consecutive lanes (G = 2, 4, 8 or 16, a group inside
// one 16-lane row) with DPP lane permutations: quad_perm [1,0,3,2] and
// [2,3,0,1] (partners at xor 1 and xor 2), row_half_mirror (lane i with
// 7 - i of its 8) and row_mirror (lane i with 15 - i). Each step adds a value
// that is the same on both partners, so every lane of a group ends with the
// same bits. Every lane of the wave must take part.
template <int CTRL> __device__ __forceinline__ float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
template <int CTRL> __device__ __forceinline__ double dpp_move(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
template <int G, typename T> __device__ __forceinline__ T group_sum(T v) {
  static_assert(G == 1 || G == 2 || G == 4 || G == 8 || G == 16, "group of 1..16 lanes");
  if constexpr (G >= 2) v = v + dpp_move<0xB1>(v);
  if constexpr (G >= 4) v = v + dpp_move<0x4E>(v);
  if constexpr (G >= 8) v = v + dpp_move<0x141>(v);
  if constexpr (G >= 16) v = v + dpp_move<0x140>(v);
  return v;
}

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
__host__ __device__ inline int64_t round_up(int64_t a, int64_t b) { return cdiv(a, b) * b; }

}  // namespace nmfk

// Host-side launch status helper: every launcher returns hipError_t.
#define NMF_LAUNCH_CHECK() hipGetLastError()
