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
// accumulates dL/dA, and the small row-times-matrix update; and the pieces of
// the HALS adjoint (reverse column sweep, Gram gradient, normalisation).
#include "common.h"
#include "grid.h"
#include "rowtile.h"
#include "kernels.h"

namespace nmfk {

// Rows are split over TPR threads (a power of two, whole rows per wave) of
// RPT outputs each; 256 threads cover 256 / TPR rows; G is staged in LDS.
template <int KP> struct AdjSplit {
  static constexpr int TPR = KP == 48 ? 4 : KP / 8;
  static constexpr int RPT = KP / TPR;
  static constexpr int ROWS = 256 / TPR;
};

// Local adjoint of Xn = X * N / (X G + eps) for the rows of one block. The
// gradient reaching Xn is gXn, plus (PRE) Y + Xn (M + M^T): what the next
// half-step's product (Y) and Gram (M) pass back to Xn, added here rather
// than in kernels of their own. Writes gN (and, if gNt is set, its
// transpose), gD (= dL/dD) and gX; entries k..KP-1 are 0. G, (PRE) M + M^T
// (from M and its transpose Mtr), the block's rows of X and (PRE) of Xn live
// in LDS; the Xn rows' buffer then holds dL/dD and the X rows' buffer gN for
// the transposed store. With Gslab set, the block also writes its share of
// dL/dG = X^T (dL/dD) to slab blockIdx.x (KP x KP) of Gslab, for an ordered
// sum over the blocks.
// Both G-products run in the same form: one value of the row broadcast from
// LDS times 16-byte runs of a matrix row, d_i = sum_j x_j G[j][i] from G
// and (dL/dx)_i = sum_j dd_j G[i][j] from G^T (Gtr, the Gram's transposed
// copy, staged as well where the LDS budget allows, GT; otherwise row i of G
// against the row's dd).
template <typename T, int KP, bool PRE>
__global__ __launch_bounds__(256) void mu_adjoint_rows_kernel(
    const T* __restrict__ X, const T* __restrict__ Xn, const T* __restrict__ N,
    const T* __restrict__ G, const T* __restrict__ Gtr, const T* __restrict__ gXn, Split<T> Y,
    const T* __restrict__ M, const T* __restrict__ Mtr, int64_t rows, int k, T eps,
    T* __restrict__ gN, T* __restrict__ gNt, T* __restrict__ gD, T* __restrict__ gX,
    T* __restrict__ Gslab) {
  constexpr int TPR = AdjSplit<KP>::TPR, RPT = AdjSplit<KP>::RPT, ROWS = AdjSplit<KP>::ROWS;
  constexpr int VEC = Tr<T>::VEC;
  constexpr int DLD = KP + VEC;
  constexpr bool GT = sizeof(T) == 4 || KP <= 32;
  __shared__ __attribute__((aligned(16))) T Gs[KP * KP];
  __shared__ __attribute__((aligned(16))) T Gt[GT ? KP * KP : VEC];
  __shared__ __attribute__((aligned(16))) T Ms[PRE ? KP * KP : VEC];
  __shared__ __attribute__((aligned(16))) T Xs[ROWS * DLD];
  __shared__ __attribute__((aligned(16))) T Ds[ROWS * DLD];
  __shared__ __attribute__((aligned(16))) T GNs[ROWS * DLD];
  const int64_t rb = (int64_t)blockIdx.x * ROWS;
  const int lr = threadIdx.x / TPR;
  const int64_t r = rb + lr;
  const bool live = r < rows;
  const int i0 = (threadIdx.x % TPR) * RPT;
  // The staging loads, then Y's slabs (independent of them, summed in slab
  // order in double and rounded once), all in flight together; then the LDS
  // writes.
  SquareStage<T, KP, 256> gst, gtst, mst;
  RowStage<T, KP, ROWS, DLD, 256> xst, xnst;
  gst.load(G, nullptr);
  if constexpr (GT) gtst.load(Gtr, nullptr);
  if constexpr (PRE) {
    if (M) mst.load(M, Mtr);
    xnst.load(Xn, rb, rows);
  }
  xst.load(X, rb, rows);
  // the row's entries of gXn, N and (not PRE) Xn: 16-byte runs, issued with
  // the staging loads (rows past the end read the last row and store nothing)
  constexpr int NV = RPT / VEC;
  const int64_t rowc = live ? r : rows - 1;
  V16<T> gxv[NV], nv[NV], xnv[NV];
#pragma unroll
  for (int h = 0; h < NV; ++h) {
    gxv[h] = load16<T>(gXn + rowc * KP + i0 + h * VEC);
    nv[h] = load16<T>(N + rowc * KP + i0 + h * VEC);
    if constexpr (!PRE) xnv[h] = load16<T>(Xn + rowc * KP + i0 + h * VEC);
  }
  double ys[RPT];
#pragma unroll
  for (int ii = 0; ii < RPT; ++ii) ys[ii] = 0.0;
  if (PRE && live && Y.p) slab_sum<T, RPT>(Y.p + r * KP + i0, Y.n, Y.stride, ys);
  gst.store(Gs);
  if constexpr (GT) gtst.store(Gt);
  if constexpr (PRE) {
    if (M) {
      mst.store(Ms);
    } else {
      for (int e = threadIdx.x; e < KP * KP; e += 256) Ms[e] = T(0);
    }
    xnst.store(Ds, rb, rows);
  }
  xst.store(Xs, rb, rows);
  __syncthreads();
  const T* xs = &Xs[lr * DLD];
  const T* xns = &Ds[lr * DLD];
  // d = x G (the denominators) and, PRE, p = xn (M + M^T)
  T d[RPT], p[RPT];
#pragma unroll
  for (int ii = 0; ii < RPT; ++ii) d[ii] = p[ii] = T(0);
#pragma unroll 8
  for (int j = 0; j < KP; ++j) {
    const T xj = xs[j];
    T xnj = T(0);
    if constexpr (PRE) xnj = xns[j];
#pragma unroll
    for (int q = 0; q < RPT / VEC; ++q) {
      const V16<T> v = load16<T>(&Gs[j * KP + i0 + q * VEC]);
#pragma unroll
      for (int w = 0; w < VEC; ++w) d[q * VEC + w] = fma(xj, v.v[w], d[q * VEC + w]);
      if constexpr (PRE) {
        const V16<T> mv = load16<T>(&Ms[j * KP + i0 + q * VEC]);
#pragma unroll
        for (int w = 0; w < VEC; ++w) p[q * VEC + w] = fma(xnj, mv.v[w], p[q * VEC + w]);
      }
    }
  }
  if constexpr (PRE) {
    if (Y.p) {
#pragma unroll
      for (int ii = 0; ii < RPT; ++ii) p[ii] += (T)ys[ii];
    }
  }
  T gn[RPT], dd[RPT], gx[RPT];
#pragma unroll
  for (int ii = 0; ii < RPT; ++ii) {
    const int i = i0 + ii;
    gn[ii] = dd[ii] = gx[ii] = T(0);
    if (live && i < k) {
      T g = gxv[ii / VEC].v[ii % VEC];
      if constexpr (PRE) g += p[ii];
      const T xn = PRE ? xns[i] : xnv[ii / VEC].v[ii % VEC];
      const T den = d[ii] + eps;
      gn[ii] = g * xs[i] / den;
      dd[ii] = -g * xn / den;
      gx[ii] = g * nv[ii / VEC].v[ii % VEC] / den;  // direct term; (dL/dD) G^T is added below
    }
  }
  if (live) {
#pragma unroll
    for (int ii = 0; ii < RPT; ++ii) {
      gN[r * KP + i0 + ii] = gn[ii];
      gD[r * KP + i0 + ii] = dd[ii];
    }
  }
  __syncthreads();  // the staged rows of Xn are no longer read
#pragma unroll
  for (int ii = 0; ii < RPT; ++ii) {
    Ds[lr * DLD + i0 + ii] = dd[ii];
    GNs[lr * DLD + i0 + ii] = gn[ii];
  }
  __syncthreads();
  if (Gslab) block_gram_partial<T, KP, ROWS, DLD>(Xs, Ds, Gslab + (int64_t)blockIdx.x * KP * KP);
  if (live) {
    // D_i = sum_j x_j G[j][i], so dL/dx_i picks up sum_j dd_j G[i][j]
    if constexpr (GT) {
      T acc[RPT];
#pragma unroll
      for (int ii = 0; ii < RPT; ++ii) acc[ii] = T(0);
      const T* dds = &Ds[lr * DLD];
#pragma unroll 8
      for (int j = 0; j < KP; ++j) {
        const T dj = dds[j];
#pragma unroll
        for (int q = 0; q < RPT / VEC; ++q) {
          const V16<T> v = load16<T>(&Gt[j * KP + i0 + q * VEC]);
#pragma unroll
          for (int w = 0; w < VEC; ++w) acc[q * VEC + w] = fma(dj, v.v[w], acc[q * VEC + w]);
        }
      }
#pragma unroll
      for (int ii = 0; ii < RPT; ++ii)
        gX[r * KP + i0 + ii] = i0 + ii < k ? gx[ii] + acc[ii] : T(0);
    } else {
#pragma unroll
      for (int ii = 0; ii < RPT; ++ii) {
        const int i = i0 + ii;
        T acc = gx[ii];
        if (i < k) {
#pragma unroll 4
          for (int q = 0; q < KP / VEC; ++q) {
            const V16<T> gv = load16<T>(&Gs[i * KP + q * VEC]);
            const V16<T> dv = load16<T>(&Ds[lr * DLD + q * VEC]);
#pragma unroll
            for (int w = 0; w < VEC; ++w) acc = fma(dv.v[w], gv.v[w], acc);
          }
        }
        gX[r * KP + i] = acc;
      }
    }
  }
  if (gNt) store_rows_transposed<T, KP, ROWS, DLD>(GNs, rb, rows, gNt);
}

// Out[r] = (Out[r] + Y[r]) + X[r] M for rows x KP X and KP x KP M, columns
// < k; Y (nullable) arrives as a product's slabs, summed in slab order in
// double.
template <typename T, int KP>
__global__ __launch_bounds__(256) void rowmm_add_kernel(const T* __restrict__ X,
                                                        const T* __restrict__ M, Split<T> Y,
                                                        int64_t rows, int k, T* __restrict__ Out) {
  constexpr int TPR = AdjSplit<KP>::TPR, RPT = AdjSplit<KP>::RPT, ROWS = AdjSplit<KP>::ROWS;
  constexpr int VEC = Tr<T>::VEC;
  constexpr int XLD = KP + VEC;
  __shared__ __attribute__((aligned(16))) T Ms[KP * KP];
  __shared__ __attribute__((aligned(16))) T Xs[ROWS * XLD];
  const int64_t rb = (int64_t)blockIdx.x * ROWS;
  const int lr = threadIdx.x / TPR;
  const int64_t r = rb + lr;
  const bool live = r < rows;
  const int i0 = (threadIdx.x % TPR) * RPT;
  SquareStage<T, KP, 256> mst;
  RowStage<T, KP, ROWS, XLD, 256> xst;
  mst.load(M, nullptr);
  xst.load(X, rb, rows);
  double ys[RPT];
#pragma unroll
  for (int ii = 0; ii < RPT; ++ii) ys[ii] = 0.0;
  if (live && Y.p) slab_sum<T, RPT>(Y.p + r * KP + i0, Y.n, Y.stride, ys);
  mst.store(Ms);
  xst.store(Xs, rb, rows);
  __syncthreads();
  if (!live) return;
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
    if (i0 + ii < k) {
      T o = Out[r * KP + i0 + ii];
      if (Y.p) o += (T)ys[ii];
      Out[r * KP + i0 + ii] = o + s[ii];
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
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride)
    Y[e] += X[e];
}

// D (m x n, ld ldd) = beta D + sum_{t < L} (X1_t Y1_t^T + X2_t Y2_t^T) with
// X*_t m x KP and Y*_t n x KP (row layout, KP contiguous, slab t at offset
// t m KP or t n KP): the whole reduction of one checkpoint segment, 2 L KP
// long, in one pass over D. Each wave forms a 64 x 64 tile on the matrix
// cores (16 x 16 x 4 tiles, the reduction index permuted so every operand
// load is 16 bytes; the loads of step s + 1 are in flight while step s
// computes) and adds it to D; a workgroup is 64 rows x 256 columns. The
// tile goes to D through LDS, 16 rows at a time, so that each row of D is
// read and written as whole 16-byte runs across consecutive lanes (vec: n,
// ldd and D allow it; otherwise element by element).
constexpr int RU = 64;
template <typename T>
__global__ __launch_bounds__(256, 2) void rank_update_kernel(T* __restrict__ D, int64_t ldd,
                                                          int64_t m, int64_t n,
                                                          const T* __restrict__ X1,
                                                          const T* __restrict__ Y1,
                                                          const T* __restrict__ X2,
                                                          const T* __restrict__ Y2, int KP,
                                                          int L, int beta, int vec) {
  constexpr int VEC = Tr<T>::VEC;
  constexpr int KSTEP = 4 * VEC;        // reduction entries per step
  constexpr int LD = RU + VEC;          // LDS row pitch of a staged slab
  constexpr int LPR = RU / VEC;         // lanes per row when draining (16 or 32)
  constexpr int RPP = 64 / LPR;         // rows per pass (4 or 2)
  typedef typename Tr<T>::acc4 acc4;
  __shared__ __attribute__((aligned(16))) T slab[4][16 * LD];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, c = lane & 15;
  const int64_t r0 = (int64_t)blockIdx.y * RU;
  const int64_t c0 = ((int64_t)blockIdx.x * 4 + wave) * RU;
  if (c0 >= n) return;
  // float: the wave's tile of D is loaded at the start, in the layout of the
  // drain below, so that its latency hides behind the matrix-core work
  constexpr bool PREFETCH = sizeof(T) == 4;
  constexpr int NP = 16 / RPP;
  V16<T> dpre[PREFETCH ? 4 : 1][PREFETCH ? NP : 1];
  if constexpr (PREFETCH) {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        const int64_t row = r0 + 16 * a + p * RPP + lane / LPR;
        const int64_t col = c0 + (lane % LPR) * VEC;
        if (beta && vec && row < m && col < n) {
          dpre[a][p] = load16<T>(D + row * ldd + col);
        } else {
#pragma unroll
          for (int v = 0; v < VEC; ++v) dpre[a][p].v[v] = T(0);
        }
      }
  }
  acc4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = zero4<T>();
  // Offsets of the lane's rows of X and of Y within a slab (clamped at the
  // ends; the extra products land outside D and are not stored).
  int64_t xo[4], yo[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int64_t row = r0 + 16 * t + c, col = c0 + 16 * t + c;
    xo[t] = (row < m ? row : m - 1) * KP + VEC * g;
    yo[t] = (col < n ? col : n - 1) * KP + VEC * g;
  }
  // Step s covers entries kk .. kk + KSTEP - 1 of pair p = s / SPP of the
  // reduction: pair 2t is (X1_t, Y1_t), pair 2t + 1 is (X2_t, Y2_t).
  const int SPP = KP / KSTEP;
  const int npair = X2 ? 2 * L : L;
  const int64_t nsteps = (int64_t)npair * SPP;
  V16<T> xa[2][4], yb[2][4];
  auto load = [&](V16<T>(&xv)[4], V16<T>(&yv)[4], int64_t s) {
    const int p = (int)(s / SPP), kk = (int)(s % SPP) * KSTEP;
    const int t = X2 ? p >> 1 : p;
    const bool second = X2 && (p & 1);
    const T* Xb = (second ? X2 : X1) + (int64_t)t * m * KP + kk;
    const T* Yb = (second ? Y2 : Y1) + (int64_t)t * n * KP + kk;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      xv[q] = load16<T>(Xb + xo[q]);
      yv[q] = load16<T>(Yb + yo[q]);
    }
  };
  auto compute = [&](const V16<T>(&xv)[4], const V16<T>(&yv)[4]) {
#pragma unroll
    for (int v = 0; v < VEC; ++v)
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = mfma16(xv[a].v[v], yv[b].v[v], acc[a][b]);
  };
  if (nsteps > 0) load(xa[0], yb[0], 0);
  for (int64_t s = 0; s < nsteps; s += 2) {
    if (s + 1 < nsteps) load(xa[1], yb[1], s + 1);
    compute(xa[0], yb[0]);
    if (s + 2 < nsteps) load(xa[0], yb[0], s + 2);
    if (s + 1 < nsteps) compute(xa[1], yb[1]);
  }
  T* sw = slab[wave];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int b = 0; b < 4; ++b) sw[acc_row<T>(lane, r) * LD + 16 * b + c] = acc[a][b][r];
    // LDS operations of one wave complete in order: the reads below see the
    // writes above, and the next slab's writes follow these reads.
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int p = 0; p < 16 / RPP; ++p) {
      const int rl = p * RPP + lane / LPR;
      const int cl = (lane % LPR) * VEC;
      const int64_t row = r0 + 16 * a + rl, col = c0 + cl;
      if (row < m && col < n) {
        T* dp = D + row * ldd + col;
        const T* sp = &sw[rl * LD + cl];
        if (vec) {
          V16<T> dv;
          if constexpr (PREFETCH) {
            dv = dpre[a][p];
          } else if (beta) {
            dv = load16<T>(dp);
          } else {
#pragma unroll
            for (int v = 0; v < VEC; ++v) dv.v[v] = T(0);
          }
#pragma unroll
          for (int v = 0; v < VEC; ++v) dv.v[v] += sp[v];
          if constexpr (sizeof(T) == 4) {
            *reinterpret_cast<float4*>(dp) = make_float4(dv.v[0], dv.v[1], dv.v[2], dv.v[3]);
          } else {
            *reinterpret_cast<double2*>(dp) = make_double2(dv.v[0], dv.v[1]);
          }
        } else {
#pragma unroll
          for (int v = 0; v < VEC; ++v)
            if (col + v < n) dp[v] = (beta ? dp[v] : T(0)) + sp[v];
        }
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// --- HALS (Section 4.2, Eq. (5)) -------------------------------------------
// Column i of a HALS sweep on a row x sets x_i' = max(0, (p_i - sum_{j != i}
// x_j G_ji) / G_ii) (skipped when G_ii = 0), i = 0..k-1 in order with the
// newest values. Its reverse, for i = k-1..0, with g the gradient with
// respect to the row's values at that point and M = [x_i' > 0]:
//     delta_i = M g_i / G_ii   (= dL/dp_i)
//     g_j -= G_ji delta_i for j != i,   g_i = 0
// (x_i' does not depend on the old x_i). What is left in g is dL/dx (old).
// dL/dG is formed by the driver from the deltas: the value of x_j that
// column i saw is the new one for j <= i and the old one for j > i, so
//     dL/dG[j][i] = -(X_new^T Delta)[j][i] for j <= i, -(X_old^T Delta)[j][i]
//     otherwise.
// A group of TPR lanes per row (as in the forward sweep): lane `sub` owns
// entries sub*R .. sub*R + R - 1 of g, of the mask and of the deltas. At step
// i the owner of entry i forms delta_i, a group sum (the other lanes add 0)
// hands it to every lane, and each lane updates its own entries of g with
// column i of G (staged in LDS, column-contiguous). Rows past the end run on
// a clamped copy of the last row and store nothing.
template <int KP> struct HalsAdjGroup {
  static constexpr int TPR = KP == 16 ? 4 : (KP == 32 ? 8 : 16);
  static constexpr int R = KP / TPR;
  static constexpr int ROWS = 256 / TPR;
};

// With Xold and Tslab set, the block also writes its shares of the two
// Gram products of the sweep's Gram gradient, Xnew^T Delta and Xold^T Delta,
// to slab blockIdx.x of Tslab and of Tslab + nblocks KP^2 (KP x KP each), for
// ordered sums over the blocks.
template <typename T, int KP>
__global__ __launch_bounds__(256) void hals_adjoint_rows_kernel(
    const T* __restrict__ Xnew, const T* __restrict__ G, const T* __restrict__ gXnew,
    int64_t rows, int k, T* __restrict__ gXold, T* __restrict__ Delta, T* __restrict__ Dt,
    const T* __restrict__ Xold, T* __restrict__ Tslab) {
  constexpr int TPR = HalsAdjGroup<KP>::TPR, R = HalsAdjGroup<KP>::R;
  constexpr int ROWS = HalsAdjGroup<KP>::ROWS;
  constexpr int VEC = Tr<T>::VEC;
  constexpr int DLD = KP + VEC;
  __shared__ __attribute__((aligned(16))) T Gs[KP * KP];
  __shared__ __attribute__((aligned(16))) T Ds[ROWS * DLD];
  __shared__ __attribute__((aligned(16))) T XNs[ROWS * DLD];
  __shared__ __attribute__((aligned(16))) T XOs[ROWS * DLD];
  const bool grams = Tslab != nullptr;  // uniform over the block
  const int sub = threadIdx.x % TPR;
  const int64_t rb = (int64_t)blockIdx.x * ROWS;
  const int64_t r = rb + threadIdx.x / TPR;
  const int64_t rr = r < rows ? r : rows - 1;
  // G's loads, the block's rows of Xnew and Xold (for the Gram shares) and
  // the row's values, in flight together
  SquareStage<T, KP, 256> gst;
  RowStage<T, KP, ROWS, DLD, 256> xnst, xost;
  gst.load(G, nullptr);
  if (grams) {
    xnst.load(Xnew, rb, rows);
    xost.load(Xold, rb, rows);
  }
  T g[R], d[R];
  unsigned mask = 0;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    g[q] = gXnew[rr * KP + sub * R + q];
    mask |= (Xnew[rr * KP + sub * R + q] > T(0) ? 1u : 0u) << q;
    d[q] = T(0);
  }
  gst.store_t(Gs);
  if (grams) {
    xnst.store(XNs, rb, rows);
    xost.store(XOs, rb, rows);
  }
  __syncthreads();
#pragma unroll
  for (int i = KP - 1; i >= 0; --i) {
    if (i < k) {
      const T gii = Gs[i * KP + i];
      if (gii > T(0)) {
        const bool own = sub == i / R;
        const T mine = (own && ((mask >> (i % R)) & 1u)) ? g[i % R] / gii : T(0);
        const T di = group_sum<TPR>(mine);
        const T* gc = &Gs[i * KP + sub * R];
#pragma unroll
        for (int q = 0; q < R; ++q) g[q] = fma(-gc[q], di, g[q]);
        if (own) {
          g[i % R] = T(0);
          d[i % R] = di;
        }
      }
    }
  }
  if (r < rows) {
#pragma unroll
    for (int q = 0; q < R; ++q) {
      gXold[r * KP + sub * R + q] = g[q];
      Delta[r * KP + sub * R + q] = d[q];
    }
  }
  if (Dt == nullptr && !grams) return;  // uniform over the block
#pragma unroll
  for (int q = 0; q < R; ++q) Ds[(threadIdx.x / TPR) * DLD + sub * R + q] = d[q];
  __syncthreads();
  if (grams) {
    // rows past the end are zero in XNs and XOs, so their deltas add nothing
    const int64_t slab = (int64_t)KP * KP;
    block_gram_partial<T, KP, ROWS, DLD>(XNs, Ds, Tslab + blockIdx.x * slab);
    block_gram_partial<T, KP, ROWS, DLD>(XOs, Ds, Tslab + (gridDim.x + blockIdx.x) * slab);
  }
  // Delta transposed (Dt[i * rows + r]), the layout the next product reads
  if (Dt) store_rows_transposed<T, KP, ROWS, DLD>(Ds, rb, rows, Dt);
}

// M = S + S^T with S[a][b] = -(a <= b ? T1[a][b] : T2[a][b]) (KP x KP): the
// symmetric Gram gradient of a HALS sweep from T1 = X_new^T Delta and
// T2 = X_old^T Delta, each given as nb per-block slabs (T1's at slabs, T2's
// after them). GG_SUB threads per output add every GG_SUB-th slab, then one
// thread adds their partial sums in order (a fixed order: reproducible bit for
// bit), rounds T1 and T2 to T and combines them.
constexpr int GG_OUT = 16, GG_SUB = 16;
template <typename T>
__global__ __launch_bounds__(GG_OUT * GG_SUB) void hals_gram_grad_kernel(
    const T* __restrict__ slabs, int nb, int KP, T* __restrict__ M) {
  __shared__ double sh[2][GG_SUB][GG_OUT];
  const int o = threadIdx.x % GG_OUT, sub = threadIdx.x / GG_OUT;
  const int e = blockIdx.x * GG_OUT + o;
  const bool in = e < KP * KP;
  const int a = in ? e / KP : 0, b = in ? e % KP : 0;
  const int64_t sl = (int64_t)KP * KP;
  const T* pab = slabs + (a <= b ? 0 : nb * sl) + a * KP + b;
  const T* pba = slabs + (b <= a ? 0 : nb * sl) + b * KP + a;
  double s1 = 0.0, s2 = 0.0;
  if (in) {
    // eight slabs' loads in flight at a time, added in slab order
    constexpr int NB = 8;
    int p = sub;
    for (; p + (NB - 1) * GG_SUB < nb; p += NB * GG_SUB) {
      T va[NB], vb[NB];
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        va[u] = pab[(int64_t)(p + u * GG_SUB) * sl];
        vb[u] = pba[(int64_t)(p + u * GG_SUB) * sl];
      }
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        s1 += (double)va[u];
        s2 += (double)vb[u];
      }
    }
    for (; p < nb; p += GG_SUB) {
      s1 += (double)pab[(int64_t)p * sl];
      s2 += (double)pba[(int64_t)p * sl];
    }
  }
  sh[0][sub][o] = s1;
  sh[1][sub][o] = s2;
  __syncthreads();
  if (sub == 0 && in) {
    double t1 = 0.0, t2 = 0.0;
#pragma unroll
    for (int q = 0; q < GG_SUB; ++q) {
      t1 += sh[0][q][o];
      t2 += sh[1][q][o];
    }
    M[e] = -((T)t1 + (T)t2);
  }
}

// Column dot products out[c] = sum_r X[r][c] Y[r][c] (rows x KP, KP <= 128)
// in double, for two pairs (X, Y) at once: each block sums a slice of one
// pair's rows per column (256 / KP row lanes, combined in LDS), and a second
// kernel adds the block partials of each column in a fixed tree.
constexpr int COLDOT_BLOCKS = 256;
template <typename T>
__global__ __launch_bounds__(256) void coldot_partials_kernel(const T* __restrict__ X1,
                                                              const T* __restrict__ Y1,
                                                              int64_t rows1, int nb1,
                                                              const T* __restrict__ X2,
                                                              const T* __restrict__ Y2,
                                                              int64_t rows2, int KP,
                                                              double* __restrict__ part) {
  __shared__ double sh[256];
  // blocks [0, nb1) take the first pair, the rest the second, each pair
  // striding over its rows with its own block count
  const bool two = (int)blockIdx.x >= nb1;
  const T* X = two ? X2 : X1;
  const T* Y = two ? Y2 : Y1;
  const int64_t rows = two ? rows2 : rows1;
  const int b = two ? (int)blockIdx.x - nb1 : (int)blockIdx.x;
  const int nb = two ? (int)gridDim.x - nb1 : nb1;
  const int lanes = 256 / KP;
  const int c = threadIdx.x % KP, lr = threadIdx.x / KP;
  double acc = 0.0;
  if (lr < lanes)
    for (int64_t r = (int64_t)b * lanes + lr; r < rows; r += (int64_t)nb * lanes)
      acc += (double)X[r * KP + c] * (double)Y[r * KP + c];
  sh[threadIdx.x] = acc;
  __syncthreads();
  if ((int)threadIdx.x < KP) {
    double t = 0.0;
    for (int q = 0; q < lanes; ++q) t += sh[q * KP + threadIdx.x];
    part[((two ? COLDOT_BLOCKS : 0) + (int64_t)b) * KP + threadIdx.x] = t;
  }
}

// One block per column of both pairs (column c of the second pair is block
// KP + c): the block partials (at most COLDOT_BLOCKS) are added pairwise in
// a fixed tree in LDS.
__global__ __launch_bounds__(COLDOT_BLOCKS) void coldot_finish_kernel(
    const double* __restrict__ part, int nb1, int nb2, int KP, double* __restrict__ out) {
  __shared__ double sh[COLDOT_BLOCKS];
  const bool two = (int)blockIdx.x >= KP;
  const int c = two ? (int)blockIdx.x - KP : (int)blockIdx.x, t = threadIdx.x;
  const int nblocks = two ? nb2 : nb1;
  const double* p = part + (two ? (int64_t)COLDOT_BLOCKS * KP : 0);
  sh[t] = t < nblocks ? p[(int64_t)t * KP + c] : 0.0;
  __syncthreads();
  for (int h = COLDOT_BLOCKS / 2; h > 0; h >>= 1) {
    if (t < h) sh[t] += sh[t + h];
    __syncthreads();
  }
  if (t == 0) out[blockIdx.x] = sh[0];
}

// Adjoint of the HALS normalisation Wn = W' diag(1/s), Hc = diag(s) H
// (s_c = ||w_c'||; columns with s_c = 0 or c >= k pass unchanged):
//     ds_c = -<gWn_c, Wn_c> / s_c + <gHc_c, H_c>
//     gW'_c = gWn_c / s_c + ds_c Wn_c,   gH_c = s_c gHc_c
// on the row layout (H as H^T, n x KP). dots holds <gWn_c, Wn_c> in [0, KP)
// and <gHc_c, H_c> in [KP, 2 KP). Rows 0..m-1 of the grid write gWp, rows
// m..m+n-1 write gHt.
template <typename T>
__global__ void hals_norm_adjoint_kernel(const T* __restrict__ gWn, const T* __restrict__ Wn,
                                         int64_t m, const T* __restrict__ gHc, int64_t n,
                                         const T* __restrict__ norms,
                                         const double* __restrict__ dots, int k, int KP,
                                         T* __restrict__ gWp, T* __restrict__ gHt) {
  const int64_t total = (m + n) * KP, stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int64_t r = e / KP;
    const int c = (int)(e - r * KP);
    const T s = norms[c];
    const bool scaled = c < k && s > T(0);
    if (r < m) {
      const int64_t q = r * KP + c;
      if (scaled) {
        const double ds = -dots[c] / (double)s + dots[KP + c];
        gWp[q] = (T)((double)gWn[q] / (double)s + ds * (double)Wn[q]);
      } else {
        gWp[q] = gWn[q];
      }
    } else {
      const int64_t q = (r - m) * KP + c;
      gHt[q] = scaled ? s * gHc[q] : gHc[q];
    }
  }
}

template <typename T>
int64_t mu_adjoint_blocks(int64_t rows, int KP) {
  switch (KP) {
    case 16: return cdiv(rows, AdjSplit<16>::ROWS);
    case 32: return cdiv(rows, AdjSplit<32>::ROWS);
    case 48: return cdiv(rows, AdjSplit<48>::ROWS);
    case 64: return cdiv(rows, AdjSplit<64>::ROWS);
    default: return 0;
  }
}

template <typename T>
hipError_t mu_adjoint_rows(const T* X, const T* Xn, const T* N, const T* G, const T* Gt,
                           const T* gXn, Split<T> Y, const T* M, const T* Mt, int64_t rows, int k,
                           int KP, T eps, T* gN, T* gNt, T* gD, T* gX, T* Gslab,
                           hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  if ((Y.p && Y.n < 1) || !Gt || (M && !Mt)) return hipErrorInvalidValue;
  const bool pre = Y.p != nullptr || M != nullptr;
  switch (KP) {
#define CASE(K)                                                                               \
  case K:                                                                                     \
    if (pre)                                                                                  \
      mu_adjoint_rows_kernel<T, K, true><<<(unsigned)cdiv(rows, AdjSplit<K>::ROWS), 256, 0,    \
                                           st>>>(X, Xn, N, G, Gt, gXn, Y, M, Mt, rows, k, eps, \
                                                 gN, gNt, gD, gX, Gslab);                      \
    else                                                                                      \
      mu_adjoint_rows_kernel<T, K, false><<<(unsigned)cdiv(rows, AdjSplit<K>::ROWS), 256, 0,   \
                                            st>>>(X, Xn, N, G, Gt, gXn, Y, M, Mt, rows, k,     \
                                                  eps, gN, gNt, gD, gX, Gslab);                \
    break;
    CASE(16) CASE(32) CASE(48) CASE(64)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return NMF_LAUNCH_CHECK();
}

template <typename T>
hipError_t rowmm_add(const T* X, const T* M, int64_t rows, int k, int KP, T* Out,
                     hipStream_t st, Split<T> Y) {
  if (rows <= 0) return hipSuccess;
  if (Y.p && Y.n < 1) return hipErrorInvalidValue;
  switch (KP) {
#define CASE(K)                                                                              \
  case K:                                                                                    \
    rowmm_add_kernel<T, K><<<(unsigned)cdiv(rows, AdjSplit<K>::ROWS), 256, 0, st>>>(X, M, Y,  \
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
  add_kernel<T><<<capped_grid(cdiv(n, 256)), 256, 0, st>>>(Y, X, n);
  return NMF_LAUNCH_CHECK();
}

template <typename T>
hipError_t rank_update(T* D, int64_t ldd, int64_t m, int64_t n, const T* X1, const T* Y1,
                       const T* X2, const T* Y2, int KP, int L, int beta, hipStream_t st) {
  if (m <= 0 || n <= 0) return hipSuccess;
  if (KP % (4 * Tr<T>::VEC) != 0 || L < 0 || (beta != 0 && beta != 1))
    return hipErrorInvalidValue;
  constexpr int VEC = Tr<T>::VEC;
  const int vec = n % VEC == 0 && ldd % VEC == 0 && (uintptr_t)D % 16 == 0;
  dim3 grid((unsigned)cdiv(n, 4 * RU), (unsigned)cdiv(m, RU));
  rank_update_kernel<T><<<grid, 256, 0, st>>>(D, ldd, m, n, X1, Y1, X2, Y2, KP, L, beta, vec);
  return NMF_LAUNCH_CHECK();
}

template <typename T>
int64_t hals_adjoint_blocks(int64_t rows, int KP) {
  switch (KP) {
    case 16: return cdiv(rows, HalsAdjGroup<16>::ROWS);
    case 32: return cdiv(rows, HalsAdjGroup<32>::ROWS);
    case 48: return cdiv(rows, HalsAdjGroup<48>::ROWS);
    case 64: return cdiv(rows, HalsAdjGroup<64>::ROWS);
    default: return 0;
  }
}

template <typename T>
hipError_t hals_adjoint_rows(const T* Xnew, const T* G, const T* gXnew, int64_t rows, int k,
                             int KP, T* gXold, T* Delta, T* Dt, const T* Xold, T* Tslab,
                             hipStream_t st) {
  if (Tslab && !Xold) return hipErrorInvalidValue;
  if (rows <= 0) return hipSuccess;
  switch (KP) {
#define CASE(K)                                                                               \
  case K:                                                                                     \
    hals_adjoint_rows_kernel<T, K><<<(unsigned)cdiv(rows, HalsAdjGroup<K>::ROWS), 256, 0,      \
                                     st>>>(Xnew, G, gXnew, rows, k, gXold, Delta, Dt, Xold,   \
                                           Tslab);                                            \
    break;
    CASE(16) CASE(32) CASE(48) CASE(64)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return NMF_LAUNCH_CHECK();
}

template <typename T>
hipError_t hals_gram_grad(const T* slabs, int nb, int KP, T* M, hipStream_t st) {
  if (nb < 1) return hipErrorInvalidValue;
  hals_gram_grad_kernel<T><<<(unsigned)cdiv(KP * KP, GG_OUT), GG_OUT * GG_SUB, 0, st>>>(
      slabs, nb, KP, M);
  return NMF_LAUNCH_CHECK();
}

int64_t coldot_partials(int KP) { return 2 * (int64_t)COLDOT_BLOCKS * KP; }

template <typename T>
hipError_t coldot2(const T* X1, const T* Y1, int64_t rows1, const T* X2, const T* Y2,
                   int64_t rows2, int KP, double* part, double* out, hipStream_t st) {
  if (KP < 1 || KP > 128) return hipErrorInvalidValue;
  const int lanes = 256 / KP;
  auto blocks_for = [&](int64_t rows) {
    const int64_t b = cdiv(rows > 0 ? rows : 1, lanes);
    return (int)(b < COLDOT_BLOCKS ? b : COLDOT_BLOCKS);
  };
  const int nb1 = blocks_for(rows1), nb2 = blocks_for(rows2);
  coldot_partials_kernel<T><<<(unsigned)(nb1 + nb2), 256, 0, st>>>(X1, Y1, rows1, nb1, X2, Y2,
                                                                    rows2, KP, part);
  hipError_t e = NMF_LAUNCH_CHECK();
  if (e != hipSuccess) return e;
  coldot_finish_kernel<<<(unsigned)(2 * KP), COLDOT_BLOCKS, 0, st>>>(part, nb1, nb2, KP, out);
  return NMF_LAUNCH_CHECK();
}

template <typename T>
hipError_t hals_norm_adjoint(const T* gWn, const T* Wn, int64_t m, const T* gHc, int64_t n,
                             const T* norms, const double* dots, int k, int KP, T* gWp, T* gHt,
                             hipStream_t st) {
  const int64_t total = (m + n) * KP;
  if (total == 0) return hipSuccess;
  hals_norm_adjoint_kernel<T><<<capped_grid(cdiv(total, 256)), 256, 0, st>>>(
      gWn, Wn, m, gHc, n, norms, dots, k, KP, gWp, gHt);
  return NMF_LAUNCH_CHECK();
}

#define INST(T)                                                                               \
  template hipError_t hals_adjoint_rows<T>(const T*, const T*, const T*, int64_t, int, int,   \
                                           T*, T*, T*, const T*, T*, hipStream_t);            \
  template int64_t hals_adjoint_blocks<T>(int64_t, int);                                      \
  template hipError_t hals_gram_grad<T>(const T*, int, int, T*, hipStream_t);                 \
  template hipError_t coldot2<T>(const T*, const T*, int64_t, const T*, const T*, int64_t,    \
                                 int, double*, double*, hipStream_t);                         \
  template hipError_t hals_norm_adjoint<T>(const T*, const T*, int64_t, const T*, int64_t,    \
                                           const T*, const double*, int, int, T*, T*,         \
                                           hipStream_t);                                      \
  template hipError_t mu_adjoint_rows<T>(const T*, const T*, const T*, const T*, const T*,    \
                                         const T*, Split<T>, const T*, const T*, int64_t, int, \
                                         int, T, T*, T*, T*, T*, T*, hipStream_t);             \
  template int64_t mu_adjoint_blocks<T>(int64_t, int);                                        \
  template hipError_t rowmm_add<T>(const T*, const T*, int64_t, int, int, T*, hipStream_t,    \
                                   Split<T>);                                                \
  template hipError_t symmetrize<T>(const T*, int, T*, hipStream_t);                          \
  template hipError_t add_to<T>(T*, const T*, int64_t, hipStream_t);                          \
  template hipError_t rank_update<T>(T*, int64_t, int64_t, int64_t, const T*, const T*,       \
                                     const T*, const T*, int, int, int, hipStream_t);
INST(float)
INST(double)
#undef INST

}  // namespace nmfk
