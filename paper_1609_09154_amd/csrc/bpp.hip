// Batched nonnegative least squares by block principal pivoting (Section 4.3,
// Eqs. (6)-(7)): for every row p of P solve
//     min_{x >= 0} 1/2 x^T G x - p^T x,    y = G x - p,
// until x_F >= 0 and y off F >= 0 (F the passive set). All right-hand sides
// share G (the Gram of the fixed factor), so one launch covers all of them:
// four right-hand sides per wavefront, one per 16-lane row, index j held by
// lane j % 16 of its row in slot j / 16 (k <= 64), the passive set a 64-bit
// mask and the infeasible set read from ballots.
//
// The exchange rule is Kim and Park's (the method the paper cites): swap all
// of V while |V| keeps falling, at most three times without progress, then
// only the largest index of V. Factorisation, solves and sign tests run in
// double for every storage type: with float arithmetic, rounding noise on
// entries whose exact value is zero flips their sign from one pivot to the
// next and the pivoting can cycle. A non-positive pivot sets status |= 1;
// reaching the pivot cap sets status |= 2.
#include <utility>

#include "common.h"
#include "kernels.h"


// ===========================================================================
// Compact solver. The passive-set system only involves the |F| indices of F,
// and the KKT conditions give an equivalent system on the active set A:
//     y = G x - p,  x_A = 0,  y_F = 0   =>   x = G^-1 (p + y),
//     (G^-1)_AA y_A = -(G^-1 p)_A,       x_F = (G^-1 p)_F + (G^-1)_FA y_A.
// With k <= 64 one of |F|, |A| is at most 32, so each solve eliminates at
// most 32 pivots. The solved set S (F, or A) is listed in increasing index
// order; lane i of a right-hand side's row holds rows i and i + 16 of
// [M_SS | rhs_S] in double registers, and Gauss-Jordan elimination takes each
// pivot row from its lane with a row broadcast (DPP row_newbcast, one move
// per double, no LDS and no waits). The other half of the KKT pair follows
// from the solution by one product with G (passive form: y off F) or G^-1
// (active form: x_F). Each right-hand side starts from the support of the
// incoming X (warm start); the solution is unique, so the start only changes
// how many exchanges are needed. The four right-hand sides of a wavefront
// eliminate together at the size of the largest of their systems.
// ===========================================================================
namespace nmfk {

constexpr int BPP_WAVES = 4;   // wavefronts per workgroup
constexpr int BPP_RPW = 4;     // right-hand sides per wavefront (one per 16-lane row)
constexpr int CNF = 32;        // largest eliminated set

// v from lane q (any lane of the wavefront), through two scalar reads
__device__ __forceinline__ double rdl(double v, int q) {
  const unsigned long long b = __double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_readlane((unsigned)(b & 0xffffffffu), q);
  const unsigned hi = __builtin_amdgcn_readlane((unsigned)(b >> 32), q);
  return __longlong_as_double(((unsigned long long)hi << 32) | lo);
}

// v from lane L of this lane's 16-lane row (DPP row_newbcast: one v_mov_b64_dpp)
template <int L> __device__ __forceinline__ double row_bcast(double v) {
  return __builtin_amdgcn_update_dpp(0.0, v, 0x150 + L, 0xf, 0xf, true);
}

// Bits of this row's right-hand side from per-slot predicates: index
// 16 s + i of row g is bit 16 g + i of the ballot of slot s.
template <int JS>
__device__ __forceinline__ uint64_t row_bits(const bool (&pr)[JS], int g) {
  uint64_t m = 0;
#pragma unroll
  for (int s = 0; s < JS; ++s) m |= ((__ballot(pr[s]) >> (16 * g)) & 0xFFFFull) << (16 * s);
  return m;
}

// LDS written by some lanes of a wavefront and read by others of the same
// wavefront: keep the accesses in program order.
__device__ __forceinline__ void wave_lds_order() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

// 1 / v for v > 0: the hardware estimate refined by two Newton steps
// (r <- r + r (1 - v r)), within an ulp or two of the quotient.
__device__ __forceinline__ double recip(double v) {
  double r = __builtin_amdgcn_rcp(v);
  r = fma(r, fma(-v, r, 1.0), r);
  r = fma(r, fma(-v, r, 1.0), r);
  return r;
}

// One Gauss-Jordan step on pivot Q of every row's system: the pivot row
// comes from lane Q % 16, slot Q / 16, and its pivot is recorded in pvl[Q]
// (the row's own pivots; their signs are tested after the elimination). The
// pivot row's entry in column Q is cleared, so it takes no multiple of
// itself (column Q is not read again). Systems smaller than NS are padded
// with zero rows and columns: the zero pivots of their extra steps are
// raised to 1e-300, which leaves every multiplier of a zero column zero.
// a[rs][c] is row i + 16 rs, column c.
template <int NS, int Q>
__device__ __forceinline__ void gj_step(double (&a)[2][CNF], double (&b)[2], double* pvl, int nsm,
                                        int i) {
  constexpr int RS = NS > 16 ? 2 : 1;
  constexpr int QS = Q >> 4, QL = Q & 15;
  if (Q >= nsm) return;
  // the lane index is re-read per step, so the compiler keeps no lane
  // masks for all steps at once
  int li = i;
  asm volatile("" : "+v"(li));
  const double pr0 = row_bcast<QL>(a[QS][Q]);
  pvl[Q] = pr0;
  if (li == QL) a[QS][Q] = 0.0;
  const double rinv = recip(fmax(pr0, 1e-300));
  double f[RS];
#pragma unroll
  for (int rs = 0; rs < RS; ++rs) f[rs] = a[rs][Q] * rinv;
  const double pb = row_bcast<QL>(b[QS]);
#pragma unroll
  for (int rs = 0; rs < RS; ++rs) b[rs] = fma(-f[rs], pb, b[rs]);
#pragma unroll
  for (int c = Q + 1; c < NS; ++c) {
    const double pr = row_bcast<QL>(a[QS][c]);
#pragma unroll
    for (int rs = 0; rs < RS; ++rs) a[rs][c] = fma(-f[rs], pr, a[rs][c]);
  }
}

template <int NS, int... Q>
__device__ __forceinline__ void gj_steps(std::integer_sequence<int, Q...>, double (&a)[2][CNF],
                                         double (&b)[2], double* pvl, int nsm, int i) {
  (gj_step<NS, Q>(a, b, pvl, nsm, i), ...);
}

// acc[s] += M[16 s + i][f] * x_T for the solution entry x_T of position T
// (held by lane T % 16, slot T / 16) at index f. M is G (LDS, leading
// dimension KP + 1) or G^-1 (ACTIVE, leading dimension KP).
template <int T, bool ACTIVE, int KP>
__device__ __forceinline__ void product_step(const double* __restrict__ Gs,
                                             const double* __restrict__ Ginv, const int (&fi)[CNF],
                                             const double (&xs)[2], int nsm, int i,
                                             double (&acc)[KP / 16]) {
  constexpr int LD = ACTIVE ? KP : KP + 1;
  if (T >= nsm) return;
  const double v = row_bcast<T & 15>(xs[T >> 4]);
  const double* m = (ACTIVE ? Ginv : Gs) + i * LD + fi[T];
#pragma unroll
  for (int s = 0; s < KP / 16; ++s) acc[s] = fma(m[16 * s * LD], v, acc[s]);
}

template <bool ACTIVE, int KP, int... T>
__device__ __forceinline__ void product_steps(std::integer_sequence<int, T...>,
                                              const double* __restrict__ Gs,
                                              const double* __restrict__ Ginv,
                                              const int (&fi)[CNF], const double (&xs)[2], int nsm,
                                              int i, double (&acc)[KP / 16]) {
  (product_step<T, ACTIVE, KP>(Gs, Ginv, fi, xs, nsm, i, acc), ...);
}

// Loads each row's system on its solved set (listed in il, right-hand side
// in rl by index), eliminates, stores the solution by index in sl, and adds
// the product of the same matrix's columns on the solved set with the
// solution to acc (one entry per index of the row). The matrix comes from G
// in LDS (passive form) or from G^-1 (ACTIVE); a row with ns = 0 takes no
// part. Positions of il past a row's ns hold the index KP, whose row and
// column of the LDS copy of G are zero, so the passive loads need no
// masking; every load address is in range, so the loads are branch-free. A
// non-positive pivot of a row's own system sets bad.
template <int NS, bool ACTIVE, int KP>
__device__ __forceinline__ void solve_rows(const double* __restrict__ Gs,
                                           const double* __restrict__ Ginv, const int* il,
                                           const double* rl, double* sl, double* pvl, int ns,
                                           int nsm, int i, bool& bad, double (&acc)[KP / 16]) {
  constexpr int RS = NS > 16 ? 2 : 1;
  constexpr int LD = KP + 1;
  double a[2][CNF], b[2];
  int li = i;
  asm volatile("" : "+v"(li));
  int ri[RS];
#pragma unroll
  for (int rs = 0; rs < RS; ++rs) {
    ri[rs] = il[li + 16 * rs];
    b[rs] = rl[ri[rs]];   // rl[KP] is zero
  }
  if (ACTIVE) {
    bool rv[RS];
#pragma unroll
    for (int rs = 0; rs < RS; ++rs) {
      rv[rs] = ri[rs] < KP;
      ri[rs] = min(ri[rs], KP - 1);
    }
#pragma unroll
    for (int c = 0; c < NS; ++c) {
      const int cc = il[c];
#pragma unroll
      for (int rs = 0; rs < RS; ++rs) {
        const double v = Ginv[ri[rs] * KP + min(cc, KP - 1)];
        a[rs][c] = (rv[rs] && cc < KP) ? v : 0.0;
      }
    }
  } else {
#pragma unroll
    for (int c = 0; c < NS; ++c) {
      const int cc = il[c];
#pragma unroll
      for (int rs = 0; rs < RS; ++rs) a[rs][c] = Gs[ri[rs] * LD + cc];
    }
  }
  gj_steps<NS>(std::make_integer_sequence<int, NS>{}, a, b, pvl, nsm, li);
  double xs[2] = {0.0, 0.0};
  bool lbad = false;
#pragma unroll
  for (int rs = 0; rs < RS; ++rs) {
    if (li + 16 * rs < ns) {
      const double dq = pvl[li + 16 * rs];
      if (!(dq > 0.0)) lbad = true;
      xs[rs] = b[rs] / dq;
      sl[ri[rs]] = xs[rs];
    }
  }
  // a bad pivot in any lane of the row marks the whole row
  if ((__ballot(lbad) >> (16 * (__lane_id() >> 4))) & 0xFFFFull) bad = true;
  // positions past ns hold the index KP; their x_T is 0
  int fi[CNF];
#pragma unroll
  for (int t = 0; t < NS; ++t) fi[t] = ACTIVE ? min(il[t], KP - 1) : il[t];
  product_steps<ACTIVE, KP>(std::make_integer_sequence<int, NS>{}, Gs, Ginv, fi, xs, nsm, li, acc);
}

// The size an elimination of at most nsm unknowns runs at (solve_pass).
__device__ __forceinline__ int bpp_size_class(int nsm, int KP) {
  if (nsm <= 8) return 8;
  if (nsm <= 12) return 12;
  if (nsm <= 16 || KP <= 16) return 16;
  return (nsm + 1) & ~1;   // 18, 20, ..., 32
}

// One elimination pass over the rows with ns > 0 at the size class of the
// largest of them.
template <bool ACTIVE, int KP>
__device__ __forceinline__ void solve_pass(const double* __restrict__ Gs,
                                           const double* __restrict__ Ginv, const int* il,
                                           const double* rl, double* sl, double* pvl, int ns,
                                           int i, bool& bad, double (&acc)[KP / 16]) {
  const int nsm = max(max(__builtin_amdgcn_readlane(ns, 0), __builtin_amdgcn_readlane(ns, 16)),
                      max(__builtin_amdgcn_readlane(ns, 32), __builtin_amdgcn_readlane(ns, 48)));
  if (nsm == 0) return;
#define NMF_BPP_CLASS(C) solve_rows<C, ACTIVE, KP>(Gs, Ginv, il, rl, sl, pvl, ns, nsm, i, bad, acc)
  if (nsm <= 8) NMF_BPP_CLASS(8);
  else if (nsm <= 12) NMF_BPP_CLASS(12);
  else if (nsm <= 16 || KP <= 16) NMF_BPP_CLASS(16);
  else if (nsm <= 18) NMF_BPP_CLASS(18);
  else if (nsm <= 20) NMF_BPP_CLASS(20);
  else if (nsm <= 22) NMF_BPP_CLASS(22);
  else if (nsm <= 24) NMF_BPP_CLASS(24);
  else if (nsm <= 26) NMF_BPP_CLASS(26);
  else if (nsm <= 28) NMF_BPP_CLASS(28);
  else if (nsm <= 30) NMF_BPP_CLASS(30);
  else NMF_BPP_CLASS(32);
#undef NMF_BPP_CLASS
}


// Ginv (KP x KP, double) = inverse of G restricted to the indices i < k with
// G_ii > 0 (zero rows and columns elsewhere); *ok = 0 when a pivot of that
// block is not positive (the block is not numerically positive definite).
// An index with G_ii = 0 belongs to a zero column of the fixed factor: its
// right-hand side entry is exactly 0 too, so it stays active with
// x_i = y_i = 0.
//
// One wavefront, in-place Gauss-Jordan in double: lane r holds row r of M
// (G on the live indices, the identity elsewhere) and ends with row r of
// M^-1. The step on pivot q subtracts f_r times the raw pivot row from every
// row r, with f_r = M_rq / M_qq off the pivot row and 1 - 1 / M_qq on it
// (which scales the pivot row by 1 / M_qq), then sets column q to the
// inverse's column (-f_r, and 1 / M_qq on the pivot row). Pivot rows are
// read with readlane; steps of indices outside the live set are identity
// steps and are skipped.
template <int Q, int KP>
__device__ __forceinline__ void ginv_step(double (&a)[KP], int lane, uint64_t live, int k,
                                          bool& good) {
  if (Q >= k || !((live >> Q) & 1ull)) return;
  const double pv = rdl(a[Q], Q);
  if (!(pv > 0.0)) good = false;
  const double s = pv > 0.0 ? 1.0 / pv : 1.0;
  const bool me = lane == Q;
  const double f = me ? 1.0 - s : a[Q] * s;
#pragma unroll
  for (int c = 0; c < KP; ++c)
    if (c != Q) a[c] = fma(-f, rdl(a[c], Q), a[c]);
  a[Q] = me ? s : -f;
}

template <int KP, int... Q>
__device__ __forceinline__ void ginv_steps(std::integer_sequence<int, Q...>, double (&a)[KP],
                                           int lane, uint64_t live, int k, bool& good) {
  (ginv_step<Q, KP>(a, lane, live, k, good), ...);
}

template <typename TS, int KP>
__global__ __launch_bounds__(64) void gram_inverse_kernel(const TS* __restrict__ G, int k,
                                                          double* __restrict__ Ginv,
                                                          int* __restrict__ ok) {
  const int lane = threadIdx.x;
  const bool mine = lane < k && G[lane * KP + lane] > TS(0);
  const uint64_t live = __ballot(mine);
  double a[KP];
#pragma unroll
  for (int c = 0; c < KP; ++c) {
    const bool lc = (live >> c) & 1ull;
    a[c] = (mine && lc) ? (double)G[lane * KP + c] : (lane == c ? 1.0 : 0.0);
  }
  bool good = true;
  ginv_steps<KP>(std::make_integer_sequence<int, KP>{}, a, lane, live, k, good);
  if (lane < KP) {
#pragma unroll
    for (int c = 0; c < KP; ++c)
      Ginv[lane * KP + c] = (mine && ((live >> c) & 1ull)) ? a[c] : 0.0;
  }
  if (lane == 0) *ok = good ? 1 : 0;
}

template <typename TS, int KP>
__global__ __launch_bounds__(64 * BPP_WAVES, 2) void bpp_quad_kernel(
    TS* __restrict__ X, const TS* __restrict__ P, const TS* __restrict__ G,
    const double* __restrict__ Ginv, const int* __restrict__ ginv_ok, int64_t rows, int k,
    int max_pivots, int warm, int* __restrict__ status, unsigned long long* __restrict__ pivots) {
  static_assert(KP % 16 == 0 && KP <= 64, "16-lane rows over at most 64 indices");
  constexpr int JS = KP / 16;   // index slots per lane
  constexpr int LD = KP + 1;
  // G in double with a zero row and column at index KP (the padding index)
  __shared__ double Gs[(KP + 1) * LD];
  __shared__ double rhs_l[BPP_WAVES][BPP_RPW][KP + 1];   // right-hand side of the solved system
  __shared__ double sol_l[BPP_WAVES][BPP_RPW][KP];   // its solution, by index
  __shared__ double p_l[BPP_WAVES][BPP_RPW][KP];     // the right-hand side p
  __shared__ double cp_l[BPP_WAVES][BPP_RPW][KP];    // G^-1 p (active form)
  __shared__ int idx_l[BPP_WAVES][BPP_RPW][CNF];     // the solved set, increasing
  __shared__ double piv_l[BPP_WAVES][BPP_RPW][CNF];  // pivots of the last elimination
  // per right-hand-side row of a wavefront: eliminations, their algorithmic
  // flops, sizes, wavefront-maximum sizes and size classes (BPP_T_* order)
  __shared__ unsigned long long tally_l[BPP_WAVES][BPP_RPW][BPP_TALLIES];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, g = lane >> 4, i = lane & 15;
  {
    // all of a thread's loads of G issued before its first LDS write (one
    // memory latency, not one per element); the padding row and column are 0
    constexpr int NG = (KP + 1) * LD, PER = (NG + 64 * BPP_WAVES - 1) / (64 * BPP_WAVES);
    TS gv[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = u * 64 * BPP_WAVES + (int)threadIdx.x;
      const int r = e / LD, c = e % LD;
      gv[u] = G[(e < NG && r < KP && c < KP) ? r * KP + c : 0];
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = u * 64 * BPP_WAVES + (int)threadIdx.x;
      const int r = e / LD, c = e % LD;
      if (e < NG) Gs[e] = (r < KP && c < KP) ? (double)gv[u] : 0.0;
    }
  }
  for (int e = threadIdx.x; e < BPP_WAVES * BPP_RPW * CNF; e += blockDim.x)
    (&idx_l[0][0][0])[e] = KP;
  for (int e = threadIdx.x; e < BPP_WAVES * BPP_RPW; e += blockDim.x)
    (&rhs_l[0][0][0])[e * (KP + 1) + KP] = 0.0;
  for (int e = threadIdx.x; e < BPP_WAVES * BPP_RPW * BPP_TALLIES; e += blockDim.x)
    (&tally_l[0][0][0])[e] = 0ull;
  __syncthreads();
  double* rl = rhs_l[wv][g];
  double* sl = sol_l[wv][g];
  int* il = idx_l[wv][g];
  double* pl = p_l[wv][g];
  double* cpl = cp_l[wv][g];
  double* pvl = piv_l[wv][g];
  // live: index in range with a nonzero Gram diagonal (see gram_inverse_kernel)
  bool act[JS];
#pragma unroll
  for (int s = 0; s < JS; ++s) {
    const int j = 16 * s + i;
    act[s] = j < k && Gs[j * LD + j] > 0.0;
  }
  const uint64_t all = row_bits<JS>(act, 0);   // the same for every row
  const bool have_ginv = k > CNF && *ginv_ok != 0;
  unsigned long long my_pivots = 0;
  int my_status = 0;

  // Each 16-lane row works through its own sequence of right-hand sides
  // (r, r + stride, ...): a row that finishes one starts the next in the
  // same round, so the four rows of a wavefront stay busy until their
  // sequences run out.
  const int64_t stride = (int64_t)gridDim.x * BPP_WAVES * BPP_RPW;
  int64_t r = ((int64_t)blockIdx.x * BPP_WAVES + wv) * BPP_RPW + g - stride;
  double x[JS], y[JS];
  // the next right-hand side's entries of P and warm-start signs, loaded
  // while the current one is solved
  TS pnext[JS];
  unsigned wnext = 0;   // bit s: warm-start sign of slot s
  bool have_next = false;
  uint64_t F = 0;
  bool live = true, done = true, have_cp = false, bad = false, first = false, from_warm = false;
  int budget = 3, best = k + 1, npiv = 0;
  for (;;) {
    bool solve = false;
    while (live && !solve) {
      if (done) {
        // store the finished right-hand side and start the next one
        if (r >= 0) {
          if (bad) my_status |= 1;
          my_pivots += (unsigned long long)npiv;
#pragma unroll
          for (int s = 0; s < JS; ++s) {
            const int j = 16 * s + i;
            X[r * KP + j] = (j < k) ? (TS)(x[s] > 0.0 ? x[s] : 0.0) : TS(0);
          }
        }
        r += stride;
        live = r < rows;
        if (!live) break;
        const int64_t ro = r * KP;
        if (!have_next) {
          wnext = 0;
#pragma unroll
          for (int s = 0; s < JS; ++s) {
            const int j = 16 * s + i;
            pnext[s] = j < k ? P[ro + j] : TS(0);
            wnext |= (warm && X[ro + j] > TS(0) ? 1u : 0u) << s;
          }
        }
        bool wpos[JS];
#pragma unroll
        for (int s = 0; s < JS; ++s) {
          const int j = 16 * s + i;
          const double pj = (double)pnext[s];
          pl[j] = pj;
          x[s] = 0.0;
          y[s] = -pj;
          wpos[s] = act[s] && ((wnext >> s) & 1u);
        }
        // this row's next right-hand side (it is the only reader and writer
        // of its rows of X and P)
        const int64_t rn = r + stride;
        have_next = rn < rows;
        if (have_next) {
          wnext = 0;
#pragma unroll
          for (int s = 0; s < JS; ++s) {
            const int j = 16 * s + i;
            pnext[s] = j < k ? P[rn * KP + j] : TS(0);
            wnext |= (warm && X[rn * KP + j] > TS(0) ? 1u : 0u) << s;
          }
        }
        F = row_bits<JS>(wpos, g) & all;
        done = false;
        have_cp = false;
        bad = false;
        first = F != 0;   // the warm-start set is solved before any test
        from_warm = first;
        budget = 3;
        best = k + 1;
        npiv = 0;
      }
      if (!first) {
        bool inf[JS];
#pragma unroll
        for (int s = 0; s < JS; ++s) {
          const bool inF = (F >> (16 * s + i)) & 1ull;
          inf[s] = act[s] && (inF ? (x[s] < 0.0) : (y[s] < 0.0));
        }
        const uint64_t V = row_bits<JS>(inf, g);
        if (V == 0) {
          done = true;
          continue;
        }
        if (npiv >= max_pivots) {
          my_status |= 2;
          done = true;
          continue;
        }
        const int nv = __popcll(V);
        uint64_t E;
        if (nv < best) { best = nv; budget = 3; E = V; }
        else if (budget >= 1) { --budget; E = V; }
        else { E = 1ull << (63 - __clzll(V)); }
        F ^= E;
      }
      first = false;
      ++npiv;
      if (F == 0) {
        // x = 0 solves the empty passive set
#pragma unroll
        for (int s = 0; s < JS; ++s) { x[s] = 0.0; y[s] = -pl[16 * s + i]; }
        continue;
      }
      if (__popcll(F) > CNF && !have_ginv) {   // G^-1 unavailable (G singular)
        bad = true;
        done = true;
        continue;
      }
      solve = true;
    }
    if (__ballot(live) == 0) break;
    const int nf = __popcll(F);
    const bool passive = nf <= CNF;
    if (solve && !passive && !have_cp) {
      // cp = G^-1 p, once per right-hand side
#pragma unroll
      for (int s = 0; s < JS; ++s) {
        const int jr = act[s] ? 16 * s + i : 0;
        double acc = 0.0;
        for (int l = 0; l < k; ++l) acc = fma(Ginv[jr * KP + l], pl[l], acc);
        cpl[16 * s + i] = act[s] ? acc : 0.0;
      }
      have_cp = true;
      if (i == 0) tally_l[wv][g][BPP_T_FLOPS] += 2ull * k * k;
    }
    const uint64_t S = passive ? F : (all & ~F);
    const int ns = solve ? __popcll(S) : 0;   // 0 in the active form when F holds every index
    if (__ballot(solve) == 0) continue;
    if (solve && ns > 0) {
      // the system size this row's elimination runs at: the largest of its
      // form in the wavefront, then that size's class
      const int nf_p = passive ? ns : 0, nf_a = passive ? 0 : ns;
      const int mp = max(max(__builtin_amdgcn_readlane(nf_p, 0), __builtin_amdgcn_readlane(nf_p, 16)),
                         max(__builtin_amdgcn_readlane(nf_p, 32), __builtin_amdgcn_readlane(nf_p, 48)));
      const int ma = max(max(__builtin_amdgcn_readlane(nf_a, 0), __builtin_amdgcn_readlane(nf_a, 16)),
                         max(__builtin_amdgcn_readlane(nf_a, 32), __builtin_amdgcn_readlane(nf_a, 48)));
      if (i == 0) {
        const unsigned long long n3 = (unsigned long long)ns;
        const int mx = passive ? mp : ma;
        unsigned long long* t = tally_l[wv][g];
        t[BPP_T_SOLVES] += 1ull;
        t[BPP_T_FLOPS] += n3 * n3 * n3 - n3 + 2ull * k * n3;
        t[BPP_T_SIZE] += n3;
        t[BPP_T_SIZE_MAX] += (unsigned long long)mx;
        t[BPP_T_SIZE_CLASS] += (unsigned long long)bpp_size_class(mx, KP);
      }
    }
    if (solve) {
      // the solved set in increasing order, then the padding index KP
#pragma unroll
      for (int s = 0; s < JS; ++s) {
        const int j = 16 * s + i;
        if ((S >> j) & 1ull) il[__popcll(S & ((1ull << j) - 1ull))] = j;
        rl[j] = passive ? pl[j] : cpl[j];
      }
      if (i >= ns) il[i] = KP;
      if (i + 16 >= ns) il[i + 16] = KP;
    }
    wave_lds_order();
    bool sbad = false;
    // the other half of the KKT pair comes with the solve: one product with
    // G (passive form) or G^-1 over the solved set
    double acc[JS];
#pragma unroll
    for (int s = 0; s < JS; ++s) acc[s] = 0.0;
    solve_pass<false, KP>(Gs, Ginv, il, rl, sl, pvl, passive ? ns : 0, i, sbad, acc);
    if (KP > CNF) solve_pass<true, KP>(Gs, Ginv, il, rl, sl, pvl, passive ? 0 : ns, i, sbad, acc);
    wave_lds_order();
    if (!solve) continue;
    if (sbad) {
      if (npiv == 1 && from_warm) {
        // The warm-start set was not positive definite: start over from F = {}.
        F = 0;
#pragma unroll
        for (int s = 0; s < JS; ++s) { x[s] = 0.0; y[s] = -pl[16 * s + i]; }
      } else {
        bad = true;
        done = true;
      }
      continue;
    }
#pragma unroll
    for (int s = 0; s < JS; ++s) {
      const int j = 16 * s + i;
      const bool inF = (F >> j) & 1ull, inS = (S >> j) & 1ull;
      if (passive) {
        x[s] = inF ? sl[j] : 0.0;
        y[s] = (inF || !act[s]) ? 0.0 : acc[s] - pl[j];
      } else {
        // (G^-1)_AA z = (G^-1 p)_A gives z = -y_A; x_F = (G^-1 p)_F - (G^-1)_FA z
        y[s] = inS ? -sl[j] : 0.0;
        x[s] = inF ? cpl[j] - acc[s] : 0.0;
      }
    }
  }
  if (i == 0) {
    tally_l[wv][g][BPP_T_PIVOTS] = my_pivots;
    if (my_status) atomicOr(status, my_status);
  }
  wave_lds_order();
  // one set of atomics per wavefront: lane c adds tally c of its four rows
  if (lane < BPP_TALLIES) {
    const unsigned long long v = tally_l[wv][0][lane] + tally_l[wv][1][lane] +
                                 tally_l[wv][2][lane] + tally_l[wv][3][lane];
    if (v) atomicAdd(pivots + lane, v);
  }
}

template <typename T>
hipError_t bpp_rows_compact(T* X, const T* P, const T* G, int64_t rows, int k, int KP,
                            int max_pivots, int warm, double* Ginv, int* ginv_ok, int* status,
                            unsigned long long* pivots, hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  const int64_t maxb = 256 * 16;
  const unsigned blocks = (unsigned)std::min<int64_t>(maxb, cdiv(rows, BPP_WAVES * BPP_RPW));
#define CASE(K)                                                                          \
  case K:                                                                                \
    if (k > CNF) gram_inverse_kernel<T, K><<<1, 64, 0, st>>>(G, k, Ginv, ginv_ok);            \
    bpp_quad_kernel<T, K><<<blocks, 64 * BPP_WAVES, 0, st>>>(                         \
        X, P, G, Ginv, ginv_ok, rows, k, max_pivots, warm, status, pivots);              \
    break;
  switch (KP) {
    CASE(16) CASE(32) CASE(48) CASE(64)
    default: return hipErrorInvalidValue;
  }
#undef CASE
  return NMF_LAUNCH_CHECK();
}

template hipError_t bpp_rows_compact<float>(float*, const float*, const float*, int64_t, int, int,
                                            int, int, double*, int*, int*, unsigned long long*,
                                            hipStream_t);
template hipError_t bpp_rows_compact<double>(double*, const double*, const double*, int64_t, int,
                                             int, int, int, double*, int*, int*,
                                             unsigned long long*, hipStream_t);

}  // namespace nmfk
