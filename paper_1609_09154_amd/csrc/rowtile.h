// Transposed store of a block of factor rows, shared by the row kernels that
// hand their output to a dense product: the products read the rank-side
// factor as KP x rows (each rank column's rows contiguous, 16-byte loads
// along the reduction index), and a row kernel that already holds its block
// of rows in LDS writes that copy directly instead of a separate transpose.
#pragma once

#include "common.h"
#include "kernels.h"

namespace nmfk {

template <typename T>
__device__ __forceinline__ void store16(T* p, const V16<T>& r) {
  if constexpr (sizeof(T) == 4)
    *reinterpret_cast<float4*>(p) = make_float4(r.v[0], r.v[1], r.v[2], r.v[3]);
  else
    *reinterpret_cast<double2*>(p) = make_double2(r.v[0], r.v[1]);
}

// Staging from global memory to LDS for the row kernels (NTHR threads per
// block). Each thread issues all of its 16-byte loads (load) before its first
// LDS write (store), so a block waits for one memory latency rather than one
// per element; a kernel can issue other independent loads between the two.
//
// A KP x KP matrix (pitch KP in LDS): dst[e] = G[e] (+ G2[e] when G2 is set),
// or its transpose (store_t: dst[j * KP + i] = G[i * KP + j]; the loads stay
// row-contiguous, the LDS writes scatter).
template <typename T, int KP, int NTHR> struct SquareStage {
  static constexpr int VEC = Tr<T>::VEC, NV = KP * KP / VEC, PER = (NV + NTHR - 1) / NTHR;
  V16<T> v[PER];
  __device__ __forceinline__ static int slot(int u) { return u * NTHR + (int)threadIdx.x; }
  __device__ __forceinline__ void load(const T* __restrict__ G, const T* __restrict__ G2) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int ic = slot(u) < NV ? slot(u) : NV - 1;
      v[u] = load16<T>(G + ic * VEC);
      if (G2) {
        const V16<T> w = load16<T>(G2 + ic * VEC);
#pragma unroll
        for (int q = 0; q < VEC; ++q) v[u].v[q] += w.v[q];
      }
    }
  }
  // The sum of n KP x KP slabs at G + q * stride, added in slab order in
  // double and rounded to T: the same bits as the ordered sum of those slabs
  // as a separate pass (reduce_splits).
  __device__ __forceinline__ void load_sum(const T* __restrict__ G, int n, int64_t stride);
  __device__ __forceinline__ void store(T* dst) const {
#pragma unroll
    for (int u = 0; u < PER; ++u)
      if (slot(u) < NV) {
#pragma unroll
        for (int q = 0; q < VEC; ++q) dst[slot(u) * VEC + q] = v[u].v[q];
      }
  }
  __device__ __forceinline__ void store_t(T* dst) const {
#pragma unroll
    for (int u = 0; u < PER; ++u)
      if (slot(u) < NV) {
        const int i = slot(u) * VEC / KP, j0 = slot(u) * VEC % KP;
#pragma unroll
        for (int q = 0; q < VEC; ++q) dst[(j0 + q) * KP + i] = v[u].v[q];
      }
  }
};

// The block's ROWS rows of a rows x KP factor: dst[q * LD + j] =
// X[(rb + q) * KP + j] (zero past the end; rows >= 1).
template <typename T, int KP, int ROWS, int LD, int NTHR> struct RowStage {
  static constexpr int VEC = Tr<T>::VEC, CPR = KP / VEC, NV = ROWS * CPR;
  static constexpr int PER = (NV + NTHR - 1) / NTHR;
  static_assert(LD % VEC == 0, "16-byte aligned LDS rows");
  V16<T> v[PER];
  __device__ __forceinline__ static int slot(int u) { return u * NTHR + (int)threadIdx.x; }
  __device__ __forceinline__ void load(const T* __restrict__ X, int64_t rb, int64_t rows) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int ic = slot(u) < NV ? slot(u) : NV - 1;
      int64_t row = rb + ic / CPR;
      row = row < rows ? row : rows - 1;
      v[u] = load16<T>(X + row * KP + (ic % CPR) * VEC);
    }
  }
  __device__ __forceinline__ void store(T* dst, int64_t rb, int64_t rows) const {
#pragma unroll
    for (int u = 0; u < PER; ++u)
      if (slot(u) < NV) {
        const int q = slot(u) / CPR, c = slot(u) % CPR;
        const bool in = rb + q < rows;
#pragma unroll
        for (int e = 0; e < VEC; ++e) dst[q * LD + c * VEC + e] = in ? v[u].v[e] : T(0);
      }
  }
};

template <typename T, int KP, int NTHR>
__device__ __forceinline__ void stage_square(T* dst, const T* __restrict__ G,
                                             const T* __restrict__ G2) {
  SquareStage<T, KP, NTHR> st;
  st.load(G, G2);
  st.store(dst);
}

template <typename T, int KP, int NTHR>
__device__ __forceinline__ void stage_square_t(T* dst, const T* __restrict__ G) {
  SquareStage<T, KP, NTHR> st;
  st.load(G, nullptr);
  st.store_t(dst);
}

template <typename T, int KP, int ROWS, int LD, int NTHR>
__device__ __forceinline__ void stage_rows(T* dst, const T* __restrict__ X, int64_t rb,
                                           int64_t rows) {
  RowStage<T, KP, ROWS, LD, NTHR> st;
  st.load(X, rb, rows);
  st.store(dst, rb, rows);
}

// acc[e] += the RPT entries at p[e] of each slab q < n at p + q stride,
// added in slab order in double (16-byte runs when RPT is a multiple of VEC
// and p is 16-byte aligned, else element by element). The slabs are fetched
// eight at a time so that their loads are in flight together rather than one
// memory latency per slab.
template <typename T, int RPT>
__device__ __forceinline__ void slab_sum(const T* p, int n, int64_t stride, double (&acc)[RPT]) {
  constexpr int VEC = Tr<T>::VEC, G = 8;
  if constexpr (RPT % VEC == 0) {
    constexpr int NV = RPT / VEC;
    int q = 0;
    for (; q + G <= n; q += G) {
      V16<T> v[G][NV];
#pragma unroll
      for (int u = 0; u < G; ++u)
#pragma unroll
        for (int h = 0; h < NV; ++h) v[u][h] = load16<T>(p + (q + u) * stride + h * VEC);
#pragma unroll
      for (int u = 0; u < G; ++u)
#pragma unroll
        for (int h = 0; h < NV; ++h)
#pragma unroll
          for (int w = 0; w < VEC; ++w) acc[h * VEC + w] += (double)v[u][h].v[w];
    }
    for (; q < n; ++q) {
#pragma unroll
      for (int h = 0; h < NV; ++h) {
        const V16<T> v = load16<T>(p + q * stride + h * VEC);
#pragma unroll
        for (int w = 0; w < VEC; ++w) acc[h * VEC + w] += (double)v.v[w];
      }
    }
  } else {
    int q = 0;
    for (; q + G <= n; q += G) {
      T v[G][RPT];
#pragma unroll
      for (int u = 0; u < G; ++u)
#pragma unroll
        for (int e = 0; e < RPT; ++e) v[u][e] = p[(q + u) * stride + e];
#pragma unroll
      for (int u = 0; u < G; ++u)
#pragma unroll
        for (int e = 0; e < RPT; ++e) acc[e] += (double)v[u][e];
    }
    for (; q < n; ++q)
#pragma unroll
      for (int e = 0; e < RPT; ++e) acc[e] += (double)p[q * stride + e];
  }
}

template <typename T, int KP, int NTHR>
__device__ __forceinline__ void SquareStage<T, KP, NTHR>::load_sum(const T* __restrict__ G, int n,
                                                                   int64_t stride) {
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int ic = slot(u) < NV ? slot(u) : NV - 1;
    double acc[VEC];
#pragma unroll
    for (int q = 0; q < VEC; ++q) acc[q] = 0.0;
    slab_sum<T, VEC>(G + ic * VEC, n, stride, acc);
#pragma unroll
    for (int q = 0; q < VEC; ++q) v[u].v[q] = (T)acc[q];
  }
}

// slab[a][b] = sum_q Xs[q][a] Ds[q][b] over a block's ROWS staged rows (LDS,
// pitch LD): the block's share of the Gram product X^T D, on the matrix
// cores. The block's waves take the 16 x 16 output tiles in turn; each tile
// runs down the rows four at a time (lane l: row k0 + l / 16, column l % 16
// of both operands). Rows past the end are zero in both.
template <typename T, int KP, int ROWS, int LD>
__device__ __forceinline__ void block_gram_partial(const T* Xs, const T* Ds, T* __restrict__ slab) {
  constexpr int NTL = KP / 16, TILES = NTL * NTL;
  typedef typename Tr<T>::acc4 acc4;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nwaves = blockDim.x >> 6;
  for (int t = wave; t < TILES; t += nwaves) {
    const int a0 = (t / NTL) * 16, b0 = (t % NTL) * 16;
    acc4 acc = zero4<T>();
#pragma unroll 8
    for (int k0 = 0; k0 < ROWS; k0 += 4) {
      const int q = k0 + (lane >> 4);
      acc = mfma16(Xs[q * LD + a0 + (lane & 15)], Ds[q * LD + b0 + (lane & 15)], acc);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
      slab[(a0 + acc_row<T>(lane, r)) * KP + b0 + (lane & 15)] = acc[r];
  }
}

// Writes rows [rb, rb + ROWS) of a rows x KP block held in LDS as
// tile[q * LD + i] (q = row - rb) to out[i * rows + row]. Column i's rows of
// the block go out as whole 16-byte runs when rows is a multiple of VEC (out
// is then 16-byte aligned at every run); rows past the end are skipped. Uses
// every thread of the block; the caller synchronises before (tile written)
// and nothing after.
template <typename T, int KP, int ROWS, int LD>
__device__ __forceinline__ void store_rows_transposed(const T* tile, int64_t rb, int64_t rows,
                                                      T* __restrict__ out) {
  constexpr int VEC = Tr<T>::VEC;
  static_assert(ROWS % VEC == 0, "whole vectors per column");
  constexpr int RV = ROWS / VEC;
  const bool vec = rows % VEC == 0;
  for (int e = threadIdx.x; e < KP * RV; e += blockDim.x) {
    const int i = e / RV, q0 = (e % RV) * VEC;
    const int64_t r0 = rb + q0;
    if (r0 >= rows) continue;
    T* dst = out + (int64_t)i * rows + r0;
    if (vec) {
      if constexpr (sizeof(T) == 4) {
        *reinterpret_cast<float4*>(dst) =
            make_float4(tile[q0 * LD + i], tile[(q0 + 1) * LD + i], tile[(q0 + 2) * LD + i],
                        tile[(q0 + 3) * LD + i]);
      } else {
        *reinterpret_cast<double2*>(dst) = make_double2(tile[q0 * LD + i], tile[(q0 + 1) * LD + i]);
      }
    } else {
#pragma unroll
      for (int v = 0; v < VEC; ++v)
        if (r0 + v < rows) dst[v] = tile[(q0 + v) * LD + i];
    }
  }
}

}  // namespace nmfk
