// C ABI of the NMF library: argument checks, workspace, and the AU-NMF
// iteration driver (Algorithm 1) that sequences the kernels of gemm.hip,
// update.hip, bpp.hip, sparse.hip and objective.hip on one HIP stream.
//
// Internal layout ("row layout"): the factor updated in each half-step is
// stored with one row per right-hand side, padded to KP columns:
//   W  (m x KP)  rows of W;        P = A H^T   (m x KP),  Q = H H^T (KP x KP)
//   Ht (n x KP)  rows of H^T;      R = A^T W   (n x KP),  S = W^T W (KP x KP)
// so the W step (Q, P -> W) and the H step (S, R -> Ht) run the same kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"
#include "kernels.h"
#include "nmf.h"

using nmfk::cdiv;
using nmfk::round_up;

struct nmf_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  void* at = nullptr;    // transposed copy of a dense A (see nmf_opts.transpose_a)
  size_t at_bytes = 0;
  void* scratch = nullptr;  // this device's address of the fixed scratch array (below)
  hipEvent_t switch_event = nullptr;  // orders a new stream after the old (nmf_set_stream)
};

// Fixed device scratch of the allocation-free update (nmf_update_noalloc).
// Every GPU the library runs on holds its own copy until the process ends.
// In host code the name is only a host-side stand-in: kernels and copies are
// given the per-device address that hipGetSymbolAddress returns, never the
// name itself.
static __device__ __align__(256) unsigned char scratch[NMF_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};
bool g_scratch_done[kMaxDevices] = {};

// The scratch array's address on `device` (which must be current), looked
// up once per device; null when the lookup failed (*err says why).
void* scratch_address(int device, hipError_t* err) {
  *err = hipSuccess;
  if (device < 0 || device >= kMaxDevices) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_done[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_scratch_err[device] = e;
    g_scratch_ptr[device] = e == hipSuccess ? p : nullptr;
    if (e != hipSuccess) (void)hipGetLastError();
    g_scratch_done[device] = true;
  }
  *err = g_scratch_err[device];
  return g_scratch_ptr[device];
}

__global__ void zero_words_kernel(uint32_t* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

}  // namespace

namespace {

nmf_status fail(nmf_ctx* c, nmf_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

nmf_status hip_fail(nmf_ctx* c, hipError_t e, const char* where) {
  std::string msg = std::string(where) + ": " + hipGetErrorString(e);
  if (c) c->err = msg;
  return e == hipErrorOutOfMemory ? NMF_ENOMEM : NMF_EDEVICE;
}

#define HIP_TRY(expr)                                  \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, #expr); \
  } while (0)

// Bump allocator over the context workspace (256-byte aligned slices).
struct Carve {
  size_t off = 0;
  template <typename P> size_t take(size_t count) {
    const size_t at = off;
    off = round_up(off + count * sizeof(P), 256);
    return at;
  }
};

nmf_status ensure_ws(nmf_ctx* ctx, size_t bytes) {
  if (bytes <= ctx->ws_bytes) return NMF_OK;
  if (ctx->ws) {
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    HIP_TRY(hipFree(ctx->ws));
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
  }
  const size_t want = round_up(bytes, (size_t)1 << 20);
  hipError_t e = hipMalloc(&ctx->ws, want);
  if (e != hipSuccess) {
    ctx->ws = nullptr;
    (void)hipGetLastError();
    return fail(ctx, NMF_ENOMEM, "workspace allocation of " + std::to_string(want) + " bytes failed");
  }
  ctx->ws_bytes = want;
  return NMF_OK;
}

template <typename P> P* at(nmf_ctx* ctx, size_t off) {
  return reinterpret_cast<P*>(reinterpret_cast<char*>(ctx->ws) + off);
}

int kp_dense(int k) { return (int)round_up(k, 16); }
int kp_sparse(int k) {
  int kp = 16;
  while (kp < k) kp *= 2;
  return kp;
}

// Slabs of the k x k Gram products: one wavefront per slab of at least 32
// rows (a slab of 32 rows is 128 MFMAs, about 2 us), at most 1024 slabs; past
// 2^20 rows up to 4096 slabs of at least 1024 rows, so more than one
// wavefront per SIMD shares the long slabs' latency. The slabs are summed in
// a fixed order afterwards.
int64_t gram_splits(int64_t rows) {
  int64_t s = cdiv(rows, 32);
  if (s <= 1024) return s < 1 ? 1 : s;
  const int64_t big = cdiv(rows, 1024);
  return big <= 1024 ? 1024 : (big > 4096 ? 4096 : big);
}

// Grams from the updates' row-block shares (MU and HALS at ranks up to 64):
// each update writes its blocks' shares of its output's Gram, and one ordered
// sum (reduce_splits) forms it, so the factor is not read again for its
// Gram and no Gram kernel is launched. A share is KP x KP for a block of
// 16-128 rows, about as large as the rows it covers, so past SHARE_CAP
// blocks (2^17-2^19 rows) the separate Gram, whose slabs grow to at least
// 1024 rows, moves fewer bytes and is used instead. At 65,536 rows and KP =
// 64 (2048 MU shares) the shares took 49.5 us per iteration against 57.6 us
// for the separate Grams. The same rule holds in the plain iteration and in
// the unrolled layers, so their Grams agree bit for bit.
constexpr int64_t SHARE_CAP = 4096;
// Where the shares of a factor's Gram hold at most GSUM_MAX elements (a
// 2000-row factor at k = 10: 16 shares of 16 x 16), the MU update that needs
// the Gram adds them itself as it stages G, so the Grams take no launches of
// their own; each update then keeps its shares in its own buffer.
constexpr int64_t GSUM_MAX = 1 << 14;
struct Shares {
  int rpm = 0, rpn = 0;       // rows per block for W and for H^T (0: no shares)
  int64_t nbm = 0, nbn = 0;   // blocks, that is shares, of each
  bool on() const { return rpm > 0; }
  int64_t blocks() const { return std::max(nbm, nbn); }
};

Shares plan_shares(int algo, int64_t m, int64_t n, int KP) {
  Shares sh;
  if (algo != NMF_MU && algo != NMF_HALS) return sh;
  const nmfk::ShareOf u = algo == NMF_MU ? nmfk::ShareOf::MU : nmfk::ShareOf::HALS;
  const int rpm = nmfk::share_rows(u, m, KP), rpn = nmfk::share_rows(u, n, KP);
  if (rpm <= 0 || rpn <= 0) return sh;
  const int64_t nbm = cdiv(m, rpm), nbn = cdiv(n, rpn);
  if (nbm > SHARE_CAP || nbn > SHARE_CAP) return sh;
  sh.rpm = rpm;
  sh.rpn = rpn;
  sh.nbm = nbm;
  sh.nbn = nbn;
  return sh;
}

// Whether the MU updates add these shares themselves as they stage G (few
// enough: at most 16, which reduce_splits also adds one after another, so
// either way gives the same bits).
bool gsum_fits(const Shares& sh, int KP) {
  return sh.on() && sh.blocks() * KP * KP <= GSUM_MAX && sh.blocks() <= 16;
}

// Elements of the updates' share workspace for an m x n problem: room for
// either update's shares, and for two sets (one per factor) where the MU
// updates add them themselves.
int64_t share_elems(int64_t m, int64_t n, int KP) {
  const Shares mu = plan_shares(NMF_MU, m, n, KP), ha = plan_shares(NMF_HALS, m, n, KP);
  int64_t need = std::max(mu.blocks(), ha.blocks()) * KP * KP;
  if (gsum_fits(mu, KP)) need = std::max<int64_t>(need, 2 * mu.blocks() * KP * KP);
  return need;
}

// G = the ordered sum of nb shares at gsl (Gt, nullable: its transpose).
template <typename T>
nmf_status sum_shares(nmf_ctx* ctx, const T* gsl, int64_t nb, int KP, T* G, T* Gt = nullptr) {
  HIP_TRY(nmfk::reduce_splits<T>(gsl, (int)nb, (int64_t)KP * KP, KP, KP, KP, G, KP, ctx->stream,
                                 Gt));
  return NMF_OK;
}

nmf_status bind_device(nmf_ctx* ctx) {
  if (ctx->device < 0) return fail(ctx, NMF_EDEVICE, "context is not bound to a device");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, NMF_EDEVICE, "hipSetDevice failed");
  return NMF_OK;
}

nmf_status check_common(nmf_ctx* ctx, int64_t m, int64_t n, int k) {
  if (!ctx) return NMF_EINVAL;
  if (m < 1 || n < 1) return fail(ctx, NMF_EINVAL, "m and n must be >= 1");
  if (k < 1 || k > NMF_MAX_K) return fail(ctx, NMF_EINVAL, "k must be in [1, NMF_MAX_K]");
  if (m > ((int64_t)1 << 40) || n > ((int64_t)1 << 40))
    return fail(ctx, NMF_EINVAL, "m or n too large");
  return NMF_OK;
}

bool is_lp(int dtype) { return dtype == NMF_BF16 || dtype == NMF_FP8_E4M3; }

// Reduced-precision A: rows 16-byte aligned, lda a whole number of 16 bytes.
nmf_status check_lp_a(nmf_ctx* ctx, int dtype, const void* A, int64_t lda) {
  const int64_t unit = dtype == NMF_FP8_E4M3 ? 16 : 8;
  if (lda % unit != 0)
    return fail(ctx, NMF_EINVAL, dtype == NMF_FP8_E4M3 ? "FP8 A: lda must be a multiple of 16"
                                                      : "bfloat16 A: lda must be a multiple of 8");
  if (((uintptr_t)A) % 16 != 0)
    return fail(ctx, NMF_EINVAL, "reduced-precision A must be 16-byte aligned");
  return NMF_OK;
}

nmf_status check_opts(nmf_ctx* ctx, const nmf_opts* o, int k, bool have_relerr) {
  if (!o) return fail(ctx, NMF_EINVAL, "opts is NULL");
  if (o->algo < NMF_MU || o->algo > NMF_ABPP) return fail(ctx, NMF_EINVAL, "unknown algorithm");
  if (o->iters < 0) return fail(ctx, NMF_EINVAL, "iters must be >= 0");
  if (o->objective < NMF_OBJ_NONE || o->objective > NMF_OBJ_DIRECT)
    return fail(ctx, NMF_EINVAL, "unknown objective mode");
  if (have_relerr && o->objective == NMF_OBJ_NONE)
    return fail(ctx, NMF_EINVAL, "rel_err requested with objective NMF_OBJ_NONE");
  if (o->algo == NMF_MU && !(o->eps_mu >= 0.0)) return fail(ctx, NMF_EINVAL, "eps_mu must be >= 0");
  if (o->algo == NMF_ABPP && k > 64) return fail(ctx, NMF_EINVAL, "ABPP supports k <= 64");
  if (!(o->tol >= 0.0)) return fail(ctx, NMF_EINVAL, "tol must be >= 0");
  if (o->stop < NMF_STOP_ITERS || o->stop > NMF_STOP_RELERR)
    return fail(ctx, NMF_EINVAL, "unknown stopping test");
  if (o->stop == NMF_STOP_RELERR && o->objective == NMF_OBJ_NONE)
    return fail(ctx, NMF_EINVAL, "NMF_STOP_RELERR needs the objective");
  return NMF_OK;
}

// Per-phase hipEvent timing.
struct Timers {
  bool on = false;
  hipStream_t st = nullptr;
  std::vector<std::pair<hipEvent_t, int>> marks;  // event, phase that starts here (-1 = end)
  void mark(int phase) {
    if (!on) return;
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) { on = false; return; }
    hipEventRecord(e, st);
    marks.push_back({e, phase});
  }
  void collect(nmf_stats* s) {
    if (!on || marks.empty()) return;
    hipEventSynchronize(marks.back().first);
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (size_t i = 0; i + 1 < marks.size(); ++i) {
      float ms = 0.f;
      hipEventElapsedTime(&ms, marks[i].first, marks[i + 1].first);
      if (marks[i].second >= 0) acc[marks[i].second] += ms;
    }
    s->ms_mm_aht += acc[0];
    s->ms_mm_wta += acc[5];
    s->ms_mm += acc[0] + acc[5];
    s->ms_luc += acc[1];
    s->ms_gram += acc[2];
    s->ms_obj += acc[3];
    s->ms_setup += acc[4];
    for (auto& m : marks) hipEventDestroy(m.first);
    marks.clear();
  }
  ~Timers() {
    for (auto& m : marks) hipEventDestroy(m.first);
  }
};
enum { PH_MM = 0, PH_LUC = 1, PH_GRAM = 2, PH_OBJ = 3, PH_SETUP = 4, PH_MM_T = 5, PH_END = -1 };

template <typename T> nmf_dtype dtype_of();
template <> nmf_dtype dtype_of<float>() { return NMF_F32; }
template <> nmf_dtype dtype_of<double>() { return NMF_F64; }

// Everything one AU-NMF call needs on the device.
template <typename T> struct Work {
  T *W, *Ht, *P, *R, *Q, *S, *norms, *part;
  T *Wt, *Hk;  // W^T (KP x m) and H (KP x n): the rank side of the dense products
  double* ginv;  // KP x KP, ABPP
  double *obj_part, *relerr, *normA;
  double *pg_part, *pg_val;  // projected-gradient partials; [0] H half, [1] W half
  T* gsl;  // the updates' Gram shares
  int* status;
  unsigned long long* pivots;
  int64_t obj_np;
};

// Outcome of a call with a stopping test.
struct StopInfo {
  long long iters_done = 0;
  double ratio = NAN;
};

// status points at 4 device ints: [0] ABPP flags, [1] input check, [2] G^-1 ok.
// ginv: KP*KP doubles of scratch for ABPP.
// P: the product, or (MU and HALS) its split slabs, which the update adds in
// slab order. Gslab and Xt (nullable; MU and HALS at KP <= 64): receive the
// row blocks' shares of the updated factor's Gram and its transposed copy
// (KP x rows). Xs (nullable; HALS): scales the incoming rows first (the
// normalisation's compensation of H).
template <typename T>
nmf_status local_update(nmf_ctx* ctx, int algo, T* X, nmfk::Split<T> P, const T* G,
                        int64_t rows, int k, int KP, const nmf_opts* o, int* status,
                        unsigned long long* pivots, double* ginv, T* Gslab = nullptr,
                        T* Xt = nullptr, const T* Xs = nullptr, int gn = 1) {
  hipStream_t st = ctx->stream;
  if (gn != 1 && algo != NMF_MU) return fail(ctx, NMF_EINVAL, "only MU sums Gram shares");
  if (algo == NMF_MU)
    HIP_TRY(nmfk::mu_rows<T>(X, X, P, G, rows, k, KP, (T)o->eps_mu, Xt, nullptr, Gslab, st, gn));
  else if (algo == NMF_HALS)
    HIP_TRY(nmfk::hals_rows<T>(X, X, P, G, rows, k, KP, Xt, Gslab, st, Xs));
  else {
    if (P.n != 1) return fail(ctx, NMF_EINVAL, "ABPP takes the summed product, not its slabs");
    const T* Pm = P.p;
    const int cap = o->max_pivots > 0 ? o->max_pivots : 50 * k;
    // the incoming X (the current iterate) starts each right-hand side's pivoting
    HIP_TRY(nmfk::bpp_rows_compact<T>(X, Pm, G, rows, k, KP, cap, 1, ginv, status + 2, status,
                                      pivots, st));
  }
  return NMF_OK;
}

template <typename T>
nmf_status gram(nmf_ctx* ctx, const T* X, int64_t rows, int KP, T* G, T* part,
                T* Gt = nullptr) {
  nmfk::GemmArgs<T> a{X, KP, X, KP, G, KP, KP, KP, rows, false, 0, Gt};
  HIP_TRY(nmfk::gemm_run<T>(nmfk::GemmKind::TN_GRAM, a, gram_splits(rows), part, ctx->stream));
  return NMF_OK;
}

// Workspace offsets for an AU-NMF call on an m x n problem.
template <typename T>
size_t plan_work(int64_t m, int64_t n, int KP, int iters, int64_t obj_np, int64_t extra_part,
                 Carve& cv, size_t off[18], bool sparse = false) {
  // split partials of the dense products (the sparse products use none)
  const int64_t ps_p = sparse ? 1 : std::max(nmfk::gemm_auto_splits<T>(nmfk::GemmKind::NN, m, KP, n),
                                             nmfk::gemm_auto_splits<T>(nmfk::GemmKind::TN, m, KP, n));
  const int64_t ps_r = sparse ? 1 : nmfk::gemm_auto_splits<T>(nmfk::GemmKind::TN, n, KP, m);
  int64_t part = ps_p > 1 ? ps_p * m * KP : 0;
  part = std::max<int64_t>(part, ps_r > 1 ? ps_r * n * KP : 0);
  part = std::max<int64_t>(part, gram_splits(std::max(m, n)) * KP * KP);
  part = std::max<int64_t>(part, extra_part);
  off[0] = cv.take<T>(m * KP);
  off[1] = cv.take<T>(n * KP);
  off[2] = cv.take<T>(m * KP);
  off[3] = cv.take<T>(n * KP);
  off[4] = cv.take<T>(KP * KP);
  off[5] = cv.take<T>(KP * KP);
  off[6] = cv.take<T>(KP);
  off[7] = cv.take<T>(part);
  off[8] = cv.take<double>(obj_np + 1);
  off[9] = cv.take<double>(iters + 2);
  off[10] = cv.take<int>(4);
  off[11] = cv.take<unsigned long long>(nmfk::BPP_TALLIES);
  // transposed factor copies for the dense products (unused for sparse A)
  off[12] = cv.take<T>(sparse ? 0 : m * KP);
  off[13] = cv.take<T>(sparse ? 0 : n * KP);
  off[14] = cv.take<double>(KP * KP);
  off[15] = cv.take<double>(nmfk::pgrad_partials(std::max(m, n)));
  off[16] = cv.take<double>(4);
  // the updates' Gram shares, for either update that writes them (apart from
  // the product slabs, which an update may still be reading)
  off[17] = cv.take<T>(share_elems(m, n, KP));
  return cv.off;
}

template <typename T>
Work<T> bind_work(nmf_ctx* ctx, const size_t off[18], int64_t obj_np) {
  Work<T> w;
  w.W = at<T>(ctx, off[0]);
  w.Ht = at<T>(ctx, off[1]);
  w.P = at<T>(ctx, off[2]);
  w.R = at<T>(ctx, off[3]);
  w.Q = at<T>(ctx, off[4]);
  w.S = at<T>(ctx, off[5]);
  w.norms = at<T>(ctx, off[6]);
  w.part = at<T>(ctx, off[7]);
  w.obj_part = at<double>(ctx, off[8]);
  w.normA = w.obj_part + obj_np;
  w.relerr = at<double>(ctx, off[9]);
  w.status = at<int>(ctx, off[10]);
  w.pivots = at<unsigned long long>(ctx, off[11]);
  w.Wt = at<T>(ctx, off[12]);
  w.Hk = at<T>(ctx, off[13]);
  w.ginv = at<double>(ctx, off[14]);
  w.pg_part = at<double>(ctx, off[15]);
  w.pg_val = at<double>(ctx, off[16]);
  w.gsl = at<T>(ctx, off[17]);
  w.obj_np = obj_np;
  return w;
}

// Reads the status flags and the BPP tallies (nmfk::BPP_T_*; tallies_out,
// nullable, receives all of them).
nmf_status read_status(nmf_ctx* ctx, const int* dstatus, const unsigned long long* dpiv,
                       long long* pivots_out, unsigned long long* tallies_out = nullptr) {
  int s[2] = {0, 0};
  unsigned long long pv[nmfk::BPP_TALLIES] = {};
  HIP_TRY(hipMemcpyAsync(s, dstatus, 2 * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(hipMemcpyAsync(pv, dpiv, sizeof(pv), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  if (pivots_out) *pivots_out = (long long)pv[nmfk::BPP_T_PIVOTS];
  if (tallies_out) std::memcpy(tallies_out, pv, sizeof(pv));
  if (s[1]) return fail(ctx, NMF_ENUMERIC, "input contains NaN, Inf, negative or malformed entries");
  if (s[0] & 1) return fail(ctx, NMF_ENUMERIC, "ABPP: passive-set system not positive definite");
  if (s[0] & 2) return fail(ctx, NMF_ENOTCONV, "ABPP: pivot cap reached before the KKT conditions held");
  return NMF_OK;
}

// Problem description shared by the dense and CSR drivers.
template <typename T> struct Prob {
  bool sparse = false;
  const T* A = nullptr; int64_t lda = 0;                 // dense
  const T* At = nullptr;                                 // dense A^T (n x m, ld m) or null
  // Reduced-precision A (T = float): lp is NMF_BF16 (bfloat16 bits) or
  // NMF_FP8_E4M3 (FP8 bits), 0 for none. Alp is A (m x n, lda), Alpt its
  // transposed copy (n x m, row pitch ldat); fb holds the packed factor and,
  // for FP8, fscale its KP column scales with fmax KP words of scratch.
  int lp = 0;
  const void* Alp = nullptr;
  const void* Alpt = nullptr;
  int64_t ldat = 0;
  void* fb = nullptr;
  float* fscale = nullptr;
  unsigned* fmax = nullptr;
  const int64_t* rp = nullptr; const int32_t* ci = nullptr; const float* cv = nullptr;  // CSR A
  const int64_t* rpt = nullptr; const int32_t* cit = nullptr; const float* cvt = nullptr; // CSR A^T
  int64_t nnz = 0;
  const nmfk::CsrLongRows* lra = nullptr;   // long rows of A and of A^T (nullable)
  const nmfk::CsrLongRows* lrat = nullptr;
};

// Elements per 16 bytes of a reduced-precision A: the pitch unit of its rows
// and of the packed factor.
int64_t lp_align(int lp) { return lp == NMF_FP8_E4M3 ? 16 : 8; }

// Out (M x KP float) = X F^T-style product on the reduced-precision matrix
// cores: X (M x K, ldx) is A or its transposed copy, F (K x KP float, row
// layout) the factor, packed (transposed, rounded) into pb.fb first.
nmf_status lp_product(nmf_ctx* ctx, const Prob<float>& pb, const void* X, int64_t ldx,
                      int64_t M, int64_t K, const float* F, int KP, float* Out, float* part) {
  const int64_t ldf = round_up(K, lp_align(pb.lp));
  if (pb.lp == NMF_BF16) {
    HIP_TRY(nmfk::pack_bf16_t(F, K, KP, (uint16_t*)pb.fb, ldf, ctx->stream));
    HIP_TRY(nmfk::gemm_bf16_nt((const uint16_t*)X, ldx, (const uint16_t*)pb.fb, ldf, Out, KP, M,
                               KP, K, part, ctx->stream));
    return NMF_OK;
  }
  HIP_TRY(nmfk::pack_fp8_t(F, K, KP, (uint8_t*)pb.fb, ldf, pb.fscale, pb.fmax, ctx->stream));
  HIP_TRY(nmfk::gemm_fp8_nt((const uint8_t*)X, ldx, (const uint8_t*)pb.fb, ldf, pb.fscale, Out,
                            KP, M, KP, K, part, ctx->stream));
  return NMF_OK;
}

// Ft (nullable) is F transposed (KP x rows of F); the dense kernels then read
// the rank-side operand with 16-byte loads.
template <typename T>
nmf_status product_AF(nmf_ctx* ctx, const Prob<T>& pb, int64_t m, int64_t n, const T* F,
                      const T* Ft, int k, int KP, T* Pout, T* part, int* nsplit = nullptr) {
  if (nsplit) *nsplit = 1;
  if (pb.sparse) {
    if constexpr (sizeof(T) == 4) {
      HIP_TRY(nmfk::csr_spmm(pb.rp, pb.ci, pb.cv, m, F, KP, Pout, pb.lra, ctx->stream));
      return NMF_OK;
    }
    return fail(ctx, NMF_EINVAL, "sparse path is float32 only");
  }
  if (pb.lp) {
    // P = A (H^T): H packed as reduced-precision rows (KP x n), K = n contiguous
    if constexpr (sizeof(T) == 4) return lp_product(ctx, pb, pb.Alp, pb.lda, m, n, F, KP, Pout, part);
    return fail(ctx, NMF_EINVAL, "reduced-precision A takes float factors");
  }
  if (pb.At) {
    // A H^T = (A^T)^T H^T: the TN kernel streaming A^T row by row.
    nmfk::GemmArgs<T> a{pb.At, m, Ft ? Ft : F, Ft ? n : (int64_t)KP, Pout, KP, m, KP, n,
                        Ft != nullptr, k};
    HIP_TRY(nmfk::gemm_run<T>(nmfk::GemmKind::TN, a, 0, part, ctx->stream, nsplit));
    return NMF_OK;
  }
  nmfk::GemmArgs<T> a{pb.A, pb.lda, Ft ? Ft : F, Ft ? n : (int64_t)KP, Pout, KP, m, KP, n,
                      Ft != nullptr, k};
  HIP_TRY(nmfk::gemm_run<T>(nmfk::GemmKind::NN, a, 0, part, ctx->stream, nsplit));
  return NMF_OK;
}

template <typename T>
nmf_status product_AtF(nmf_ctx* ctx, const Prob<T>& pb, int64_t m, int64_t n, const T* F,
                       const T* Ft, int k, int KP, T* Rout, T* part, int* nsplit = nullptr) {
  if (nsplit) *nsplit = 1;
  if (pb.sparse) {
    if constexpr (sizeof(T) == 4) {
      HIP_TRY(nmfk::csr_spmm(pb.rpt, pb.cit, pb.cvt, n, F, KP, Rout, pb.lrat, ctx->stream));
      return NMF_OK;
    }
    return fail(ctx, NMF_EINVAL, "sparse path is float32 only");
  }
  if (pb.lp) {
    // R = A^T W on the transposed copy: W packed as reduced-precision rows (KP x m)
    if (!pb.Alpt) return fail(ctx, NMF_EINVAL, "reduced-precision A^T W needs the transposed copy");
    if constexpr (sizeof(T) == 4)
      return lp_product(ctx, pb, pb.Alpt, pb.ldat, n, m, F, KP, Rout, part);
    return fail(ctx, NMF_EINVAL, "reduced-precision A takes float factors");
  }
  nmfk::GemmArgs<T> a{pb.A, pb.lda, Ft ? Ft : F, Ft ? m : (int64_t)KP, Rout, KP, n, KP, m,
                      Ft != nullptr, k};
  HIP_TRY(nmfk::gemm_run<T>(nmfk::GemmKind::TN, a, 0, part, ctx->stream, nsplit));
  return NMF_OK;
}

// Relative error of the current (W, Ht) into relerr[slot]. q_current says
// whether w.Q holds the Gram of the current Ht (the sparse form needs it).
template <typename T>
nmf_status objective(nmf_ctx* ctx, const Prob<T>& pb, int64_t m, int64_t n, int k, int KP,
                     Work<T>& w, int slot, bool grams_current = false) {
  hipStream_t st = ctx->stream;
  if (pb.sparse) {
    if constexpr (sizeof(T) == 4) {
      // <W^T W, H H^T> covers the zeros; both Grams of the current factors
      // (already in S and Q when grams_current).
      if (!grams_current) {
        nmf_status s = gram<T>(ctx, w.W, m, KP, w.S, w.part);
        if (s != NMF_OK) return s;
        s = gram<T>(ctx, w.Ht, n, KP, w.Q, w.part);
        if (s != NMF_OK) return s;
      }
      HIP_TRY(nmfk::csr_residual_sq(pb.rp, pb.ci, pb.cv, m, w.W, w.Ht, KP, w.obj_part, st));
      HIP_TRY(nmfk::finish_relerr<T>(w.obj_part, nmfk::csr_residual_partials(m), w.S, w.Q, KP,
                                     w.normA, w.relerr + slot, st));
      return NMF_OK;
    }
    return NMF_EINVAL;
  }
  if (pb.lp == NMF_BF16) {
    if constexpr (sizeof(T) == 4)
      HIP_TRY((nmfk::residual_sq<float, uint16_t>((const uint16_t*)pb.Alp, pb.lda, m, n, w.W,
                                                  w.Ht, KP, w.obj_part, st)));
  } else if (pb.lp == NMF_FP8_E4M3) {
    if constexpr (sizeof(T) == 4)
      HIP_TRY((nmfk::residual_sq<float, uint8_t>((const uint8_t*)pb.Alp, pb.lda, m, n, w.W,
                                                 w.Ht, KP, w.obj_part, st)));
  } else {
    HIP_TRY((nmfk::residual_sq<T, T>(pb.A, pb.lda, m, n, w.W, w.Ht, KP, w.obj_part, st)));
  }
  HIP_TRY(nmfk::finish_relerr<T>(w.obj_part, nmfk::residual_partials<T>(m, n), (const T*)nullptr,
                                 (const T*)nullptr, KP, w.normA, w.relerr + slot, st));
  (void)k;
  return NMF_OK;
}

template <typename T>
nmf_status norm_sq_A(nmf_ctx* ctx, const Prob<T>& pb, int64_t m, int64_t n, Work<T>& w) {
  hipStream_t st = ctx->stream;
  if (pb.sparse) {
    if constexpr (sizeof(T) == 4) {
      const int64_t np = std::min<int64_t>(w.obj_np, 1024);
      HIP_TRY(nmfk::csr_sumsq(pb.cv, pb.nnz, w.obj_part, np, st));
      HIP_TRY(nmfk::finish_relerr<T>(w.obj_part, np, (const T*)nullptr, (const T*)nullptr, 0,
                                     (const double*)nullptr, w.normA, st));
      return NMF_OK;
    }
    return NMF_EINVAL;
  }
  if (pb.lp == NMF_BF16)
    HIP_TRY(nmfk::sumsq<uint16_t>((const uint16_t*)pb.Alp, pb.lda, m, n, w.obj_part, st));
  else if (pb.lp == NMF_FP8_E4M3)
    HIP_TRY(nmfk::sumsq<uint8_t>((const uint8_t*)pb.Alp, pb.lda, m, n, w.obj_part, st));
  else HIP_TRY(nmfk::sumsq<T>(pb.A, pb.lda, m, n, w.obj_part, st));
  HIP_TRY(nmfk::finish_relerr<T>(w.obj_part, nmfk::sumsq_partials<T>(m, n), (const T*)nullptr,
                                 (const T*)nullptr, 0, (const double*)nullptr, w.normA, st));
  return NMF_OK;
}

// Squared projected gradient of one factor (rows of X against its product P
// and Gram G) into w.pg_val[slot].
template <typename T>
nmf_status pg_half(nmf_ctx* ctx, const T* X, const T* P, const T* G, int64_t rows, int k,
                   int KP, Work<T>& w, int slot) {
  HIP_TRY(nmfk::pgrad_sq<T>(X, P, G, rows, k, KP, w.pg_part, ctx->stream));
  HIP_TRY(nmfk::finish_relerr<T>(w.pg_part, nmfk::pgrad_blocks<T>(rows, KP), (const T*)nullptr,
                                 (const T*)nullptr, 0, (const double*)nullptr, w.pg_val + slot,
                                 ctx->stream));
  return NMF_OK;
}

nmf_status read_doubles(nmf_ctx* ctx, const double* d, double* h, int count) {
  HIP_TRY(hipMemcpyAsync(h, d, sizeof(double) * count, hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return NMF_OK;
}

// Algorithm 1 on the prepared workspace. With a stopping test (Section 6.2)
// the loop reads the metric once per iteration: the projected gradient at
// (W_t, H_t) is its H half, formed right after the H update from that step's
// S = W^T W and R = A^T W, plus its W half, formed at the start of the next
// iteration from Q = H H^T and P = A H^T before W changes.
template <typename T>
nmf_status run_au_nmf(nmf_ctx* ctx, const Prob<T>& pb, int64_t m, int64_t n, int k, int KP,
                      const nmf_opts* o, Work<T>& w, bool want_obj, Timers& tm,
                      StopInfo& si) {
  hipStream_t st = ctx->stream;
  nmf_status s = NMF_OK;
#define RUN(x) do { s = (x); if (s != NMF_OK) return s; } while (0)
  const bool pgstop = o->stop == NMF_STOP_PGRAD;
  const bool errstop = o->stop == NMF_STOP_RELERR;
  si.iters_done = o->iters;
  si.ratio = NAN;
  double pg0 = 0.0;
  if (want_obj) {
    tm.mark(PH_OBJ);
    RUN(norm_sq_A<T>(ctx, pb, m, n, w));
    RUN(objective<T>(ctx, pb, m, n, k, KP, w, 0));
  }
  if (pgstop) {
    // H half at the initial factors
    tm.mark(PH_OBJ);
    RUN(gram<T>(ctx, w.W, m, KP, w.S, w.part));
    RUN(product_AtF<T>(ctx, pb, m, n, w.W, nullptr, k, KP, w.R, w.part));
    RUN(pg_half<T>(ctx, w.Ht, w.R, w.S, n, k, KP, w, 0));
  }
  // Transposed factor copies for the dense products (read with 16-byte loads,
  // so their rows must stay 16-byte aligned). Below 2^22 entries of A the
  // products read the factors in place: the copy's launch would cost more
  // than its loads save.
  const bool big = m * n >= ((int64_t)1 << 22);
  const bool tH = big && !pb.sparse && !pb.lp && (n * (int64_t)sizeof(T)) % 16 == 0;
  const bool tW = big && !pb.sparse && !pb.lp && (m * (int64_t)sizeof(T)) % 16 == 0;
  if (tH && o->iters > 0) HIP_TRY(nmfk::transpose_rows<T>(w.Ht, n, KP, w.Hk, st));
  // the updates' Gram shares (w.gsl); qready: Q already holds the current H's
  // Gram
  int nsp_w_v = 1, nsp_h_v = 1;
  const Shares sh = plan_shares(o->algo, m, n, KP);
  T* gsl = sh.on() ? w.gsl : nullptr;
  bool qready = false;
  // small MU problems: each update sums the other factor's shares itself (S
  // and Q are then not formed, so not with the objective or the
  // projected-gradient stop); the H update's shares (for Q) go to gslq
  const bool gin = o->algo == NMF_MU && !pgstop && !want_obj && gsum_fits(sh, KP);
  T* gslq = gin ? gsl + sh.blocks() * KP * KP : gsl;
  // Dense products hand their split slabs to an MU or HALS update that adds
  // them as the ordered sum would (bit for bit), where that costs the update
  // no occupancy; P and R are then not formed, so not with the
  // projected-gradient stop, which reads them.
  const bool hand = (o->algo == NMF_MU || o->algo == NMF_HALS) && !pgstop && !pb.sparse &&
                    !pb.lp;
  const nmfk::ShareOf upd = o->algo == NMF_MU ? nmfk::ShareOf::MU : nmfk::ShareOf::HALS;
  int* nsp_w = hand && nmfk::takes_slabs(upd, m) ? &nsp_w_v : nullptr;
  int* nsp_h = hand && nmfk::takes_slabs(upd, n) ? &nsp_h_v : nullptr;
  // MU and HALS at KP <= 64 write the transposed copies the next product
  // reads from their own output tiles (not HALS's W, which the
  // normalisation rescales after the sweep)
  const bool own_t = (o->algo == NMF_MU || o->algo == NMF_HALS) && KP <= 64;
  T* Wt_upd = own_t && o->algo == NMF_MU && tW ? w.Wt : nullptr;
  // HALS: the normalisation writes W's copy after rescaling W
  T* Wt_nrm = own_t && o->algo == NMF_HALS && tW ? w.Wt : nullptr;
  // A phase mark records an event on the stream, which costs the stream a few
  // microseconds: marks are set only where work follows them.
  for (int t = 0; t < o->iters; ++t) {
    // W given H: Q = H H^T, P = A H^T, UpdateW.
    if (!sh.on() || !qready) tm.mark(PH_GRAM);
    if (!sh.on()) {
      RUN(gram<T>(ctx, w.Ht, n, KP, w.Q, w.part));
    } else if (!qready) {
      HIP_TRY(nmfk::gram_shares<T>(w.Ht, n, KP, sh.rpn, gslq, st));
      if (!gin) RUN(sum_shares<T>(ctx, gslq, sh.nbn, KP, w.Q));
    }
    tm.mark(PH_MM);
    RUN(product_AF<T>(ctx, pb, m, n, w.Ht, tH ? w.Hk : nullptr, k, KP, w.P, w.part, nsp_w));
    if (pgstop) {
      tm.mark(PH_OBJ);
      RUN(pg_half<T>(ctx, w.W, w.P, w.Q, m, k, KP, w, 1));
      double h[2];
      RUN(read_doubles(ctx, w.pg_val, h, 2));
      const double pg = std::sqrt(std::max(h[0] + h[1], 0.0));
      if (t == 0) pg0 = pg;
      si.ratio = pg0 > 0.0 ? pg / pg0 : 0.0;
      if ((t > 0 || pg0 == 0.0) && si.ratio <= o->tol) {
        si.iters_done = t;
        break;
      }
    }
    tm.mark(PH_LUC);
    const nmfk::Split<T> spw{nsp_w_v > 1 ? w.part : w.P, nsp_w_v, m * KP};
    RUN(local_update<T>(ctx, o->algo, w.W, spw, gin ? gslq : w.Q, m, k, KP, o, w.status,
                        w.pivots, w.ginv, gsl, Wt_upd, nullptr, gin ? (int)sh.nbn : 1));
    // H given W: S = W^T W, (HALS: normalise), R = A^T W, UpdateH.
    if (!gin) tm.mark(PH_GRAM);
    if (!sh.on()) RUN(gram<T>(ctx, w.W, m, KP, w.S, w.part));
    else if (!gin) RUN(sum_shares<T>(ctx, gsl, sh.nbm, KP, w.S));
    if (o->algo == NMF_HALS) {
      tm.mark(PH_LUC);
      // W's columns rescaled here; H's compensation is applied by the H sweep
      // as it reads the rows (the same products, one pass over H fewer)
      HIP_TRY(nmfk::hals_normalize<T>(w.W, w.W, m, w.Ht, w.Ht, 0, w.S, w.norms, k, KP, st,
                                      Wt_nrm));
    }
    if (tW && !Wt_upd && !Wt_nrm) HIP_TRY(nmfk::transpose_rows<T>(w.W, m, KP, w.Wt, st));
    tm.mark(PH_MM_T);
    RUN(product_AtF<T>(ctx, pb, m, n, w.W, tW ? w.Wt : nullptr, k, KP, w.R, w.part, nsp_h));
    tm.mark(PH_LUC);
    const bool next_t = tH && t + 1 < o->iters;
    const nmfk::Split<T> sph{nsp_h_v > 1 ? w.part : w.R, nsp_h_v, n * KP};
    RUN(local_update<T>(ctx, o->algo, w.Ht, sph, gin ? gsl : w.S, n, k, KP, o, w.status,
                        w.pivots, w.ginv, gslq, own_t && next_t ? w.Hk : nullptr,
                        o->algo == NMF_HALS ? w.norms : nullptr, gin ? (int)sh.nbm : 1));
    if (sh.on()) {
      // the next iteration's Q, from the H update's shares
      if (!gin) {
        tm.mark(PH_GRAM);
        RUN(sum_shares<T>(ctx, gslq, sh.nbn, KP, w.Q));
      }
      qready = true;
    }
    if (next_t && !own_t) HIP_TRY(nmfk::transpose_rows<T>(w.Ht, n, KP, w.Hk, st));
    if (pgstop) {
      tm.mark(PH_OBJ);
      RUN(pg_half<T>(ctx, w.Ht, w.R, w.S, n, k, KP, w, 0));
    }
    if (want_obj) {
      tm.mark(PH_OBJ);
      RUN(objective<T>(ctx, pb, m, n, k, KP, w, t + 1, sh.on()));
    }
    if (errstop) {
      double e[2];
      RUN(read_doubles(ctx, w.relerr + t, e, 2));
      if (e[0] - e[1] < o->tol * e[0]) {
        si.iters_done = t + 1;
        break;
      }
    }
    if (pgstop && t + 1 == o->iters) {
      // the W half at the returned factors, for the final ratio
      tm.mark(PH_OBJ);
      RUN(gram<T>(ctx, w.Ht, n, KP, w.Q, w.part));
      RUN(product_AF<T>(ctx, pb, m, n, w.Ht, nullptr, k, KP, w.P, w.part));
      RUN(pg_half<T>(ctx, w.W, w.P, w.Q, m, k, KP, w, 1));
      double h[2];
      RUN(read_doubles(ctx, w.pg_val, h, 2));
      si.ratio = pg0 > 0.0 ? std::sqrt(std::max(h[0] + h[1], 0.0)) / pg0 : 0.0;
    }
  }
  tm.mark(PH_END);
#undef RUN
  return NMF_OK;
}

template <typename T>
nmf_status finish_call(nmf_ctx* ctx, const nmf_opts* o, Work<T>& w, bool want_obj,
                       double* rel_err, nmf_stats* stats, Timers& tm, hipEvent_t t0,
                       hipEvent_t t1, const StopInfo& si) {
  long long piv = 0;
  unsigned long long tl[nmfk::BPP_TALLIES] = {};
  const bool need_status = o->algo == NMF_ABPP || o->check_input;
  if (need_status) {
    nmf_status s = read_status(ctx, w.status, w.pivots, &piv, tl);
    if (s != NMF_OK) return s;
  }
  if (rel_err && want_obj) {
    HIP_TRY(hipMemcpyAsync(rel_err, w.relerr, sizeof(double) * (si.iters_done + 1),
                           hipMemcpyDeviceToHost, ctx->stream));
    for (int t = (int)si.iters_done + 1; t <= o->iters; ++t) rel_err[t] = NAN;
  }
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    HIP_TRY(hipEventSynchronize(t1));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, t0, t1));
    stats->ms_total = ms;
    tm.collect(stats);
    stats->bpp_pivots = piv;
    stats->iters_done = si.iters_done;
    stats->pgrad_ratio = si.ratio;
    stats->bpp_solves = (long long)tl[nmfk::BPP_T_SOLVES];
    stats->bpp_flops = (double)tl[nmfk::BPP_T_FLOPS];
    const double nsol = (double)tl[nmfk::BPP_T_SOLVES];
    stats->bpp_size_mean = nsol > 0 ? (double)tl[nmfk::BPP_T_SIZE] / nsol : 0.0;
    stats->bpp_size_max_mean = nsol > 0 ? (double)tl[nmfk::BPP_T_SIZE_MAX] / nsol : 0.0;
    stats->bpp_size_class_mean = nsol > 0 ? (double)tl[nmfk::BPP_T_SIZE_CLASS] / nsol : 0.0;
  }
  if (rel_err || stats) HIP_TRY(hipStreamSynchronize(ctx->stream));
  return NMF_OK;
}

// A^T into the context's second buffer, when it fits next to everything else
// with a quarter of the device memory to spare; *out stays null otherwise.
template <typename T>
nmf_status transposed_copy(nmf_ctx* ctx, const T* A, int64_t lda, int64_t m, int64_t n,
                           int64_t ldt, const T** out) {
  *out = nullptr;
  const size_t need = (size_t)ldt * (size_t)n * sizeof(T);
  if (ctx->at_bytes < need) {
    size_t freeb = 0, total = 0;
    HIP_TRY(hipMemGetInfo(&freeb, &total));
    const size_t reuse = ctx->at_bytes;
    if (freeb + reuse < need + total / 4) return NMF_OK;
    if (ctx->at) {
      HIP_TRY(hipStreamSynchronize(ctx->stream));
      HIP_TRY(hipFree(ctx->at));
      ctx->at = nullptr;
      ctx->at_bytes = 0;
    }
    if (hipMalloc(&ctx->at, need) != hipSuccess) {
      (void)hipGetLastError();
      ctx->at = nullptr;
      return NMF_OK;
    }
    ctx->at_bytes = need;
  }
  T* At = (T*)ctx->at;
  HIP_TRY(nmfk::transpose_full<T>(A, lda, m, n, At, ldt, ctx->stream));
  *out = At;
  return NMF_OK;
}

// Scratch for reduced-precision products: the packed factor, the split
// partials and the FP8 column scales.
struct LpPlan { int64_t fb_bytes, part_elems; };
LpPlan lp_plan(int lp, int64_t m, int64_t n, int KP) {
  LpPlan p;
  const int64_t esize = lp == NMF_FP8_E4M3 ? 1 : 2;
  p.fb_bytes = (int64_t)KP * round_up(std::max(m, n), lp_align(lp)) * esize;
  const int64_t sp = nmfk::gemm_lp_splits(m, n), sr = nmfk::gemm_lp_splits(n, m);
  p.part_elems = std::max<int64_t>(sp > 1 ? sp * m * KP : 0, sr > 1 ? sr * n * KP : 0);
  return p;
}

// Carves the reduced-precision scratch and points pb at it (after ensure_ws).
struct LpOffsets { size_t fb, fscale, fmax; };
LpOffsets lp_carve(Carve& cv, const LpPlan& p, int KP) {
  LpOffsets o;
  o.fb = cv.take<uint8_t>(p.fb_bytes);
  o.fscale = cv.take<float>(KP);
  o.fmax = cv.take<unsigned>(KP);
  return o;
}

// Points pb at a reduced-precision A and its scratch; with want_t, also
// makes the transposed copy that A^T W streams.
nmf_status lp_bind(nmf_ctx* ctx, Prob<float>& pb, int lp, const void* Alp, int64_t lda, int64_t m,
                   int64_t n, const LpOffsets& lo, bool want_t) {
  pb.lp = lp;
  pb.Alp = Alp;
  pb.lda = lda;
  pb.fb = at<uint8_t>(ctx, lo.fb);
  pb.fscale = at<float>(ctx, lo.fscale);
  pb.fmax = at<unsigned>(ctx, lo.fmax);
  pb.ldat = round_up(m, lp_align(lp));
  if (!want_t) return NMF_OK;
  nmf_status s;
  if (lp == NMF_BF16) {
    const uint16_t* t = nullptr;
    s = transposed_copy<uint16_t>(ctx, (const uint16_t*)Alp, lda, m, n, pb.ldat, &t);
    pb.Alpt = t;
  } else {
    const uint8_t* t = nullptr;
    s = transposed_copy<uint8_t>(ctx, (const uint8_t*)Alp, lda, m, n, pb.ldat, &t);
    pb.Alpt = t;
  }
  if (s != NMF_OK) return s;
  if (!pb.Alpt) return fail(ctx, NMF_ENOMEM, "no room for the transposed reduced-precision copy of A");
  return NMF_OK;
}
template <typename T>
nmf_status lp_bind(nmf_ctx* ctx, Prob<T>&, int, const void*, int64_t, int64_t, int64_t,
                   const LpOffsets&, bool) {
  return fail(ctx, NMF_EINVAL, "reduced-precision A takes float factors");
}

// With lp nonzero, Alp is A in that reduced format (A is then null and T is
// float).
template <typename T>
nmf_status dense_impl(nmf_ctx* ctx, int64_t m, int64_t n, const T* A, int lp, const void* Alp,
                      int64_t lda, int k, const nmf_opts* o, T* W, T* H, double* rel_err,
                      nmf_stats* stats) {
  const int KP = kp_dense(k);
  const bool want_obj = o->objective != NMF_OBJ_NONE;
  const int64_t obj_np = std::max(nmfk::residual_partials<T>(m, n), nmfk::sumsq_partials<T>(m, n));
  const LpPlan bp = lp ? lp_plan(lp, m, n, KP) : LpPlan{0, 0};
  Carve cv;
  size_t off[18];
  plan_work<T>(m, n, KP, o->iters, obj_np, bp.part_elems, cv, off);
  const LpOffsets lo = lp_carve(cv, bp, KP);
  nmf_status s = ensure_ws(ctx, cv.off);
  if (s != NMF_OK) return s;
  Work<T> w = bind_work<T>(ctx, off, obj_np);
  hipStream_t st = ctx->stream;
  HIP_TRY(hipMemsetAsync(w.status, 0, 4 * sizeof(int), st));
  HIP_TRY(hipMemsetAsync(w.pivots, 0, nmfk::BPP_TALLIES * sizeof(unsigned long long), st));
  if (o->check_input) {
    if (lp == NMF_BF16)
      HIP_TRY(nmfk::check_dense<uint16_t>((const uint16_t*)Alp, lda, m, n, w.status + 1, st));
    else if (lp == NMF_FP8_E4M3)
      HIP_TRY(nmfk::check_dense<uint8_t>((const uint8_t*)Alp, lda, m, n, w.status + 1, st));
    else HIP_TRY(nmfk::check_dense<T>(A, lda, m, n, w.status + 1, st));
  }
  Timers tm;
  tm.on = stats && o->timers;
  tm.st = st;
  tm.mark(PH_SETUP);
  HIP_TRY(nmfk::pad_rows<T>(W, m, k, w.W, KP, st));
  HIP_TRY(nmfk::transpose_in<T>(H, k, n, w.Ht, KP, st));
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if (stats) {
    HIP_TRY(hipEventCreate(&t0));
    HIP_TRY(hipEventCreate(&t1));
    HIP_TRY(hipEventRecord(t0, st));
  }
  Prob<T> pb;
  pb.A = A;
  pb.lda = lda;
  if (lp) {
    if ((s = lp_bind(ctx, pb, lp, Alp, lda, m, n, lo, o->iters > 0)) != NMF_OK) return s;
  } else if (o->iters > 0 && o->transpose_a == 0) {
    if ((s = transposed_copy<T>(ctx, A, lda, m, n, m, &pb.At)) != NMF_OK) return s;
  }
  StopInfo si;
  s = run_au_nmf<T>(ctx, pb, m, n, k, KP, o, w, want_obj, tm, si);
  if (stats) HIP_TRY(hipEventRecord(t1, st));
  if (s == NMF_OK) {
    HIP_TRY(nmfk::unpad_rows<T>(w.W, m, k, KP, W, st));
    HIP_TRY(nmfk::transpose_out<T>(w.Ht, k, n, KP, H, st));
    s = finish_call<T>(ctx, o, w, want_obj, rel_err, stats, tm, t0, t1, si);
  }
  if (t0) hipEventDestroy(t0);
  if (t1) hipEventDestroy(t1);
  return s;
}

}  // namespace

// ===========================================================================
// Exported C ABI
// ===========================================================================
extern "C" {

void nmf_default_opts(nmf_opts* o) {
  if (!o) return;
  o->tol = 0.0;
  o->stop = NMF_STOP_ITERS;
  o->algo = NMF_MU;
  o->iters = 0;
  o->eps_mu = 1e-16;
  o->max_pivots = 0;
  o->objective = NMF_OBJ_NONE;
  o->timers = 0;
  o->check_input = 0;
  o->transpose_a = 0;
}

const char* nmf_status_str(nmf_status s) {
  switch (s) {
    case NMF_OK: return "NMF_OK";
    case NMF_EINVAL: return "NMF_EINVAL";
    case NMF_ENOMEM: return "NMF_ENOMEM";
    case NMF_EDEVICE: return "NMF_EDEVICE";
    case NMF_ENUMERIC: return "NMF_ENUMERIC";
    case NMF_ENOTCONV: return "NMF_ENOTCONV";
  }
  return "NMF_UNKNOWN";
}

const char* nmf_last_error(const nmf_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

nmf_status nmf_create(nmf_ctx** out, int device, void* hip_stream) {
  if (!out) return NMF_EINVAL;
  *out = nullptr;
  if (device == -1) {
    nmf_ctx* c = new nmf_ctx();
    c->device = -1;
    *out = c;
    return NMF_OK;
  }
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count < 1) return NMF_EDEVICE;
  if (device < 0 || device >= count) return NMF_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return NMF_EDEVICE;
  nmf_ctx* c = new nmf_ctx();
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  // Set-up of the allocation-free update: this device's address of the
  // fixed scratch array. A failed lookup leaves it null; only
  // nmf_update_noalloc needs it, and it reports the failure.
  hipError_t se;
  c->scratch = scratch_address(device, &se);
  *out = c;
  return NMF_OK;
}

void nmf_destroy(nmf_ctx* ctx) {
  if (!ctx) return;
  if ((ctx->ws || ctx->at || ctx->switch_event) && ctx->device >= 0) {
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->at) (void)hipFree(ctx->at);
    if (ctx->switch_event) (void)hipEventDestroy(ctx->switch_event);
  }
  delete ctx;
}

nmf_status nmf_set_stream(nmf_ctx* ctx, void* hip_stream) {
  if (!ctx) return NMF_EINVAL;
  const hipStream_t next = (hipStream_t)hip_stream;
  if (next != ctx->stream && ctx->device >= 0 && (ctx->ws || ctx->at)) {
    // Work already enqueued on the old stream may still use the workspace:
    // the new stream waits for it before any later call's work starts.
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, NMF_EDEVICE, "hipSetDevice failed");
    if (!ctx->switch_event &&
        hipEventCreateWithFlags(&ctx->switch_event, hipEventDisableTiming) != hipSuccess) {
      ctx->switch_event = nullptr;
      return fail(ctx, NMF_EDEVICE, "hipEventCreateWithFlags failed");
    }
    if (hipEventRecord(ctx->switch_event, ctx->stream) != hipSuccess ||
        hipStreamWaitEvent(next, ctx->switch_event, 0) != hipSuccess)
      return fail(ctx, NMF_EDEVICE, "ordering the new stream after the old one failed");
  }
  ctx->stream = next;
  return NMF_OK;
}

nmf_status nmf_dense(nmf_ctx* ctx, nmf_dtype dtype, int64_t m, int64_t n, const void* A,
                     int64_t lda, int k, const nmf_opts* opts, void* W, void* H, double* rel_err,
                     nmf_stats* stats) {
  nmf_status s = check_common(ctx, m, n, k);
  if (s != NMF_OK) return s;
  if ((s = check_opts(ctx, opts, k, rel_err != nullptr)) != NMF_OK) return s;
  if (!A || !W || !H) return fail(ctx, NMF_EINVAL, "null A, W or H");
  if (lda < n) return fail(ctx, NMF_EINVAL, "lda < n");
  if (dtype != NMF_F32 && dtype != NMF_F64 && !is_lp(dtype))
    return fail(ctx, NMF_EINVAL, "unknown dtype");
  if (is_lp(dtype)) {
    if ((s = check_lp_a(ctx, dtype, A, lda)) != NMF_OK) return s;
    if (opts->transpose_a != 0)
      return fail(ctx, NMF_EINVAL, "reduced-precision A needs its transposed copy (transpose_a 0)");
  }
  if ((s = bind_device(ctx)) != NMF_OK) return s;
  if (is_lp(dtype))
    return dense_impl<float>(ctx, m, n, nullptr, dtype, A, lda, k, opts, (float*)W, (float*)H,
                             rel_err, stats);
  if (dtype == NMF_F32)
    return dense_impl<float>(ctx, m, n, (const float*)A, 0, nullptr, lda, k, opts, (float*)W,
                             (float*)H, rel_err, stats);
  return dense_impl<double>(ctx, m, n, (const double*)A, 0, nullptr, lda, k, opts, (double*)W,
                            (double*)H, rel_err, stats);
}

nmf_status nmf_csr(nmf_ctx* ctx, int64_t m, int64_t n, int64_t nnz, const int64_t* rowptr,
                   const int32_t* colidx, const float* vals, int k, const nmf_opts* opts,
                   float* W, float* H, double* rel_err, nmf_stats* stats) {
  nmf_status s = check_common(ctx, m, n, k);
  if (s != NMF_OK) return s;
  if ((s = check_opts(ctx, opts, k, rel_err != nullptr)) != NMF_OK) return s;
  if (!rowptr || !W || !H || (nnz > 0 && (!colidx || !vals)))
    return fail(ctx, NMF_EINVAL, "null CSR array, W or H");
  if (nnz < 0 || nnz > ((int64_t)1 << 40)) return fail(ctx, NMF_EINVAL, "bad nnz");
  if (n > INT32_MAX || m > INT32_MAX)
    return fail(ctx, NMF_EINVAL, "m and n must fit int32 column ids (of A and of A^T)");
  if (nnz > (int64_t)UINT32_MAX) return fail(ctx, NMF_EINVAL, "nnz must be below 2^32");
  if ((s = bind_device(ctx)) != NMF_OK) return s;
  typedef float T;
  const int KP = kp_sparse(k);
  const bool want_obj = opts->objective != NMF_OBJ_NONE;
  const int64_t obj_np = std::max<int64_t>(nmfk::csr_residual_partials(m), 1024);
  Carve cv;
  size_t off[18];
  plan_work<T>(m, n, KP, opts->iters, obj_np, 0, cv, off, true);
  const size_t o_rpt = cv.take<int64_t>(n + 1);
  const size_t o_cit = cv.take<int32_t>(nnz);
  const size_t o_cvt = cv.take<float>(nnz);
  const size_t o_tw = cv.take<char>(nmfk::csr_transpose_work_bytes(m, n, nnz));
  const size_t o_la = cv.take<char>(nmfk::csr_long_work_bytes(nnz, KP));
  const size_t o_lat = cv.take<char>(nmfk::csr_long_work_bytes(nnz, KP));
  if ((s = ensure_ws(ctx, cv.off)) != NMF_OK) return s;
  Work<T> w = bind_work<T>(ctx, off, obj_np);
  hipStream_t st = ctx->stream;
  HIP_TRY(hipMemsetAsync(w.status, 0, 4 * sizeof(int), st));
  HIP_TRY(hipMemsetAsync(w.pivots, 0, nmfk::BPP_TALLIES * sizeof(unsigned long long), st));
  if (opts->check_input) {
    HIP_TRY(nmfk::check_csr(rowptr, colidx, vals, m, n, nnz, w.status + 1, st));
    // Structure must be valid before the transpose and SpMM read it.
    int flag = 0;
    HIP_TRY(hipMemcpyAsync(&flag, w.status + 1, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (flag) return fail(ctx, NMF_ENUMERIC, "CSR input malformed or has NaN/Inf/negative values");
  }
  Timers tm;
  tm.on = stats && opts->timers;
  tm.st = st;
  tm.mark(PH_SETUP);
  Prob<T> pb;
  pb.sparse = true;
  pb.rp = rowptr;
  pb.ci = colidx;
  pb.cv = vals;
  pb.nnz = nnz;
  pb.rpt = at<int64_t>(ctx, o_rpt);
  pb.cit = at<int32_t>(ctx, o_cit);
  pb.cvt = at<float>(ctx, o_cvt);
  HIP_TRY(nmfk::csr_transpose(rowptr, colidx, vals, m, n, nnz, (int64_t*)pb.rpt, (int32_t*)pb.cit,
                              (float*)pb.cvt, at<char>(ctx, o_tw), st));
  nmfk::CsrLongRows lra, lrat;
  HIP_TRY(nmfk::csr_long_rows(rowptr, m, nnz, KP, at<char>(ctx, o_la), &lra, st));
  HIP_TRY(nmfk::csr_long_rows(pb.rpt, n, nnz, KP, at<char>(ctx, o_lat), &lrat, st));
  pb.lra = &lra;
  pb.lrat = &lrat;
  HIP_TRY(nmfk::pad_rows<T>(W, m, k, w.W, KP, st));
  HIP_TRY(nmfk::transpose_in<T>(H, k, n, w.Ht, KP, st));
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if (stats) {
    HIP_TRY(hipEventCreate(&t0));
    HIP_TRY(hipEventCreate(&t1));
    HIP_TRY(hipEventRecord(t0, st));
  }
  StopInfo si;
  s = run_au_nmf<T>(ctx, pb, m, n, k, KP, opts, w, want_obj, tm, si);
  if (stats) HIP_TRY(hipEventRecord(t1, st));
  if (s == NMF_OK) {
    HIP_TRY(nmfk::unpad_rows<T>(w.W, m, k, KP, W, st));
    HIP_TRY(nmfk::transpose_out<T>(w.Ht, k, n, KP, H, st));
    s = finish_call<T>(ctx, opts, w, want_obj, rel_err, stats, tm, t0, t1, si);
  }
  if (t0) hipEventDestroy(t0);
  if (t1) hipEventDestroy(t1);
  return s;
}

}  // extern "C"

// ---- per-step entry points ------------------------------------------------

namespace {
template <typename T>
nmf_status gram_impl(nmf_ctx* ctx, int64_t rows, int k, const T* X, int64_t ldx, T* G) {
  const int KP = kp_dense(k);
  Carve cv;
  const size_t oX = cv.take<T>(rows * KP);
  const size_t oG = cv.take<T>(KP * KP);
  const size_t oP = cv.take<T>(gram_splits(rows) * KP * KP);
  nmf_status s = ensure_ws(ctx, cv.off);
  if (s != NMF_OK) return s;
  T* Xp = at<T>(ctx, oX);
  T* Gp = at<T>(ctx, oG);
  hipStream_t st = ctx->stream;
  if (ldx == k) HIP_TRY(nmfk::pad_rows<T>(X, rows, k, Xp, KP, st));
  else {
    HIP_TRY(hipMemsetAsync(Xp, 0, sizeof(T) * rows * KP, st));
    HIP_TRY(hipMemcpy2DAsync(Xp, KP * sizeof(T), X, ldx * sizeof(T), k * sizeof(T), rows,
                             hipMemcpyDeviceToDevice, st));
  }
  if ((s = gram<T>(ctx, Xp, rows, KP, Gp, at<T>(ctx, oP))) != NMF_OK) return s;
  HIP_TRY(nmfk::unpad_rows<T>(Gp, k, k, KP, G, st));
  return NMF_OK;
}

template <typename T>
nmf_status pad_any(nmf_ctx* ctx, const T* X, int64_t rows, int k, int64_t ldx, T* Xp, int KP) {
  hipStream_t st = ctx->stream;
  if (ldx == k) HIP_TRY(nmfk::pad_rows<T>(X, rows, k, Xp, KP, st));
  else {
    HIP_TRY(hipMemsetAsync(Xp, 0, sizeof(T) * rows * KP, st));
    HIP_TRY(hipMemcpy2DAsync(Xp, KP * sizeof(T), X, ldx * sizeof(T), k * sizeof(T), rows,
                             hipMemcpyDeviceToDevice, st));
  }
  return NMF_OK;
}

template <typename T>
nmf_status dense_prod_impl(nmf_ctx* ctx, bool transA, int64_t m, int64_t n, const T* A,
                           int64_t lda, int k, const T* F, int64_t ldf, T* Out) {
  const int KP = kp_dense(k);
  const int64_t frows = transA ? m : n, orows = transA ? n : m;
  const int64_t splits = transA ? nmfk::gemm_auto_splits<T>(nmfk::GemmKind::TN, n, KP, m)
                                : nmfk::gemm_auto_splits<T>(nmfk::GemmKind::NN, m, KP, n);
  Carve cv;
  const size_t oF = cv.take<T>(frows * KP);
  const size_t oFt = cv.take<T>(frows * KP);
  const size_t oO = cv.take<T>(orows * KP);
  const size_t oP = cv.take<T>(splits > 1 ? splits * orows * KP : 1);
  nmf_status s = ensure_ws(ctx, cv.off);
  if (s != NMF_OK) return s;
  T* Fp = at<T>(ctx, oF);
  T* Ft = at<T>(ctx, oFt);
  T* Op = at<T>(ctx, oO);
  if ((s = pad_any<T>(ctx, F, frows, k, ldf, Fp, KP)) != NMF_OK) return s;
  // The transposed copy is read with 16-byte loads: rows must stay aligned.
  const bool use_t = (frows * (int64_t)sizeof(T)) % 16 == 0;
  if (use_t) HIP_TRY(nmfk::transpose_rows<T>(Fp, frows, KP, Ft, ctx->stream));
  Prob<T> pb;
  pb.A = A;
  pb.lda = lda;
  s = transA ? product_AtF<T>(ctx, pb, m, n, Fp, use_t ? Ft : nullptr, k, KP, Op, at<T>(ctx, oP))
             : product_AF<T>(ctx, pb, m, n, Fp, use_t ? Ft : nullptr, k, KP, Op, at<T>(ctx, oP));
  if (s != NMF_OK) return s;
  HIP_TRY(nmfk::unpad_rows<T>(Op, orows, k, KP, Out, ctx->stream));
  return NMF_OK;
}

nmf_status dense_prod_lp_impl(nmf_ctx* ctx, bool transA, int lp, int64_t m, int64_t n,
                              const void* Alp, int64_t lda, int k, const float* F, int64_t ldf,
                              float* Out) {
  const int KP = kp_dense(k);
  const int64_t frows = transA ? m : n, orows = transA ? n : m;
  const LpPlan bp = lp_plan(lp, m, n, KP);
  Carve cv;
  const size_t oF = cv.take<float>(frows * KP);
  const size_t oO = cv.take<float>(orows * KP);
  const size_t oP = cv.take<float>(std::max<int64_t>(bp.part_elems, 1));
  const LpOffsets lo = lp_carve(cv, bp, KP);
  nmf_status s = ensure_ws(ctx, cv.off);
  if (s != NMF_OK) return s;
  float* Fp = at<float>(ctx, oF);
  float* Op = at<float>(ctx, oO);
  if ((s = pad_any<float>(ctx, F, frows, k, ldf, Fp, KP)) != NMF_OK) return s;
  Prob<float> pb;
  if ((s = lp_bind(ctx, pb, lp, Alp, lda, m, n, lo, transA)) != NMF_OK) return s;
  s = transA ? product_AtF<float>(ctx, pb, m, n, Fp, nullptr, k, KP, Op, at<float>(ctx, oP))
             : product_AF<float>(ctx, pb, m, n, Fp, nullptr, k, KP, Op, at<float>(ctx, oP));
  if (s != NMF_OK) return s;
  HIP_TRY(nmfk::unpad_rows<float>(Op, orows, k, KP, Out, ctx->stream));
  return NMF_OK;
}

template <typename T>
nmf_status update_impl(nmf_ctx* ctx, int algo, int64_t rows, int k, const T* G, const T* Pm,
                       T* X, const nmf_opts* o, long long* pivots) {
  const int KP = kp_dense(k);
  Carve cv;
  const size_t oG = cv.take<T>(KP * KP);
  const size_t oP = cv.take<T>(rows * KP);
  const size_t oX = cv.take<T>(rows * KP);
  const size_t oS = cv.take<int>(4);
  const size_t oV = cv.take<unsigned long long>(nmfk::BPP_TALLIES);
  const size_t oI = cv.take<double>(KP * KP);
  nmf_status s = ensure_ws(ctx, cv.off);
  if (s != NMF_OK) return s;
  T* Gp = at<T>(ctx, oG);
  T* Pp = at<T>(ctx, oP);
  T* Xp = at<T>(ctx, oX);
  int* dst = at<int>(ctx, oS);
  unsigned long long* dpv = at<unsigned long long>(ctx, oV);
  hipStream_t st = ctx->stream;
  HIP_TRY(hipMemsetAsync(dst, 0, 4 * sizeof(int), st));
  HIP_TRY(hipMemsetAsync(dpv, 0, nmfk::BPP_TALLIES * sizeof(unsigned long long), st));
  HIP_TRY(nmfk::pad_rows<T>(G, k, k, Gp, KP, st));
  if (KP > k) HIP_TRY(hipMemsetAsync(Gp + (size_t)k * KP, 0, sizeof(T) * (KP - k) * KP, st));
  HIP_TRY(nmfk::pad_rows<T>(Pm, rows, k, Pp, KP, st));
  HIP_TRY(nmfk::pad_rows<T>(X, rows, k, Xp, KP, st));
  if ((s = local_update<T>(ctx, algo, Xp, nmfk::Split<T>{Pp, 1, 0}, Gp, rows, k, KP, o, dst, dpv,
                          at<double>(ctx, oI))) !=
      NMF_OK)
    return s;
  HIP_TRY(nmfk::unpad_rows<T>(Xp, rows, k, KP, X, st));
  if (algo == NMF_ABPP) return read_status(ctx, dst, dpv, pivots);
  return NMF_OK;
}

// Slices of the fixed scratch array for update_noalloc_impl: status and
// pivot counters first (cleared together), then the inverse Gram of ABPP's
// active form and the padded G, P and X.
struct NoallocPlan { size_t oS, oV, oI, oG, oP, oX, total; };
template <typename T> NoallocPlan noalloc_plan(int64_t rows, int KP) {
  Carve cv;
  NoallocPlan p;
  p.oS = cv.take<int>(4);
  p.oV = cv.take<unsigned long long>(nmfk::BPP_TALLIES);
  p.oI = cv.take<double>((size_t)KP * KP);
  p.oG = cv.take<T>((size_t)KP * KP);
  p.oP = cv.take<T>((size_t)rows * KP);
  p.oX = cv.take<T>((size_t)rows * KP);
  p.total = cv.off;
  return p;
}

// update_impl on the fixed scratch array: the same kernels and launch
// shapes, no allocation, and fill kernels instead of hipMemsetAsync.
template <typename T>
nmf_status update_noalloc_impl(nmf_ctx* ctx, int algo, int64_t rows, int k, const T* G,
                               const T* Pm, T* X, const nmf_opts* o, long long* pivots) {
  const int KP = kp_dense(k);
  const NoallocPlan pl = noalloc_plan<T>(rows, KP);
  char* base = (char*)ctx->scratch;
  T* Gp = (T*)(base + pl.oG);
  T* Pp = (T*)(base + pl.oP);
  T* Xp = (T*)(base + pl.oX);
  int* dst = (int*)(base + pl.oS);
  unsigned long long* dpv = (unsigned long long*)(base + pl.oV);
  hipStream_t st = ctx->stream;
  // counters: the words from the status slice up to the inverse Gram
  const int64_t nz = (int64_t)(pl.oI - pl.oS) / 4;
  zero_words_kernel<<<(unsigned)cdiv(nz, 256), 256, 0, st>>>((uint32_t*)dst, nz);
  HIP_TRY(hipGetLastError());
  HIP_TRY(nmfk::pad_rows<T>(G, k, k, Gp, KP, st));
  if (KP > k) {
    const int64_t nw = (int64_t)(KP - k) * KP * (int64_t)sizeof(T) / 4;
    zero_words_kernel<<<(unsigned)cdiv(nw, 256), 256, 0, st>>>((uint32_t*)(Gp + (size_t)k * KP), nw);
    HIP_TRY(hipGetLastError());
  }
  HIP_TRY(nmfk::pad_rows<T>(Pm, rows, k, Pp, KP, st));
  HIP_TRY(nmfk::pad_rows<T>(X, rows, k, Xp, KP, st));
  nmf_status s = local_update<T>(ctx, algo, Xp, nmfk::Split<T>{Pp, 1, 0}, Gp, rows, k, KP, o,
                                 dst, dpv,
                                 (double*)(base + pl.oI));
  if (s != NMF_OK) return s;
  HIP_TRY(nmfk::unpad_rows<T>(Xp, rows, k, KP, X, st));
  if (algo == NMF_ABPP) return read_status(ctx, dst, dpv, pivots);
  return NMF_OK;
}

template <typename T>
nmf_status normalize_impl(nmf_ctx* ctx, int64_t m, int64_t n, int k, T* W, T* Ht, T* S,
                          T* norms) {
  const int KP = kp_dense(k);
  Carve cv;
  const size_t oW = cv.take<T>(m * KP);
  const size_t oH = cv.take<T>(n * KP);
  const size_t oS = cv.take<T>(KP * KP);
  const size_t oN = cv.take<T>(KP);
  const size_t oP = cv.take<T>(gram_splits(m) * KP * KP);
  nmf_status s = ensure_ws(ctx, cv.off);
  if (s != NMF_OK) return s;
  T* Wp = at<T>(ctx, oW);
  T* Hp = at<T>(ctx, oH);
  T* Sp = at<T>(ctx, oS);
  T* Np = at<T>(ctx, oN);
  hipStream_t st = ctx->stream;
  HIP_TRY(nmfk::pad_rows<T>(W, m, k, Wp, KP, st));
  HIP_TRY(nmfk::pad_rows<T>(Ht, n, k, Hp, KP, st));
  if ((s = gram<T>(ctx, Wp, m, KP, Sp, at<T>(ctx, oP))) != NMF_OK) return s;
  HIP_TRY(nmfk::hals_normalize<T>(Wp, Wp, m, Hp, Hp, n, Sp, Np, k, KP, st));
  HIP_TRY(nmfk::unpad_rows<T>(Wp, m, k, KP, W, st));
  HIP_TRY(nmfk::unpad_rows<T>(Hp, n, k, KP, Ht, st));
  if (S) HIP_TRY(nmfk::unpad_rows<T>(Sp, k, k, KP, S, st));
  if (norms) HIP_TRY(hipMemcpyAsync(norms, Np, sizeof(T) * k, hipMemcpyDeviceToDevice, st));
  return NMF_OK;
}

template <typename T>
nmf_status relerr_impl(nmf_ctx* ctx, const Prob<T>& pb, int64_t m, int64_t n, int k, const T* W,
                       const T* Ht, double* out) {
  const int KP = pb.sparse ? kp_sparse(k) : kp_dense(k);
  const int64_t obj_np = pb.sparse ? std::max<int64_t>(nmfk::csr_residual_partials(m), 1024)
                                   : std::max(nmfk::residual_partials<T>(m, n),
                                              nmfk::sumsq_partials<T>(m, n));
  Carve cv;
  size_t off[18];
  plan_work<T>(m, n, KP, 0, obj_np, 0, cv, off, pb.sparse);
  nmf_status s = ensure_ws(ctx, cv.off);
  if (s != NMF_OK) return s;
  Work<T> w = bind_work<T>(ctx, off, obj_np);
  HIP_TRY(nmfk::pad_rows<T>(W, m, k, w.W, KP, ctx->stream));
  HIP_TRY(nmfk::pad_rows<T>(Ht, n, k, w.Ht, KP, ctx->stream));
  if ((s = norm_sq_A<T>(ctx, pb, m, n, w)) != NMF_OK) return s;
  if ((s = objective<T>(ctx, pb, m, n, k, KP, w, 0)) != NMF_OK) return s;
  HIP_TRY(hipMemcpyAsync(out, w.relerr, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return NMF_OK;
}
}  // namespace

extern "C" {

nmf_status nmf_gram(nmf_ctx* ctx, nmf_dtype dtype, int64_t rows, int k, const void* X,
                    int64_t ldx, void* G) {
  nmf_status s = check_common(ctx, rows, 1, k);
  if (s != NMF_OK) return s;
  if (!X || !G) return fail(ctx, NMF_EINVAL, "null X or G");
  if (ldx < k) return fail(ctx, NMF_EINVAL, "ldx < k");
  if ((s = bind_device(ctx)) != NMF_OK) return s;
  if (dtype == NMF_F32) return gram_impl<float>(ctx, rows, k, (const float*)X, ldx, (float*)G);
  if (dtype == NMF_F64) return gram_impl<double>(ctx, rows, k, (const double*)X, ldx, (double*)G);
  return fail(ctx, NMF_EINVAL, "unknown dtype");
}

}  // extern "C"

static nmf_status dense_prod(nmf_ctx* ctx, bool transA, nmf_dtype dtype, int64_t m, int64_t n,
                             const void* A, int64_t lda, int k, const void* F, int64_t ldf,
                             void* Out) {
  nmf_status s = check_common(ctx, m, n, k);
  if (s != NMF_OK) return s;
  if (!A || !F || !Out) return fail(ctx, NMF_EINVAL, "null A, F or output");
  if (lda < n) return fail(ctx, NMF_EINVAL, "lda < n");
  if (ldf < k) return fail(ctx, NMF_EINVAL, "ldf < k");
  if (is_lp(dtype) && (s = check_lp_a(ctx, dtype, A, lda)) != NMF_OK) return s;
  if ((s = bind_device(ctx)) != NMF_OK) return s;
  if (is_lp(dtype))
    return dense_prod_lp_impl(ctx, transA, dtype, m, n, A, lda, k, (const float*)F, ldf,
                              (float*)Out);
  if (dtype == NMF_F32)
    return dense_prod_impl<float>(ctx, transA, m, n, (const float*)A, lda, k, (const float*)F,
                                  ldf, (float*)Out);
  if (dtype == NMF_F64)
    return dense_prod_impl<double>(ctx, transA, m, n, (const double*)A, lda, k,
                                   (const double*)F, ldf, (double*)Out);
  return fail(ctx, NMF_EINVAL, "unknown dtype");
}

extern "C" {

nmf_status nmf_dense_AF(nmf_ctx* ctx, nmf_dtype dtype, int64_t m, int64_t n, const void* A,
                        int64_t lda, int k, const void* F, int64_t ldf, void* P) {
  return dense_prod(ctx, false, dtype, m, n, A, lda, k, F, ldf, P);
}

nmf_status nmf_dense_AtF(nmf_ctx* ctx, nmf_dtype dtype, int64_t m, int64_t n, const void* A,
                         int64_t lda, int k, const void* F, int64_t ldf, void* R) {
  return dense_prod(ctx, true, dtype, m, n, A, lda, k, F, ldf, R);
}

nmf_status nmf_csr_AF(nmf_ctx* ctx, int64_t m, int64_t n, int64_t nnz, const int64_t* rowptr,
                      const int32_t* colidx, const float* vals, int k, const float* F, float* P) {
  nmf_status s = check_common(ctx, m, n, k);
  if (s != NMF_OK) return s;
  if (!rowptr || !F || !P || (nnz > 0 && (!colidx || !vals)))
    return fail(ctx, NMF_EINVAL, "null CSR array, F or P");
  if (nnz < 0) return fail(ctx, NMF_EINVAL, "bad nnz");
  if ((s = bind_device(ctx)) != NMF_OK) return s;
  const int KP = kp_sparse(k);
  Carve cv;
  const size_t oF = cv.take<float>(n * KP);
  const size_t oO = cv.take<float>(m * KP);
  const size_t oL = cv.take<char>(nmfk::csr_long_work_bytes(nnz, KP));
  if ((s = ensure_ws(ctx, cv.off)) != NMF_OK) return s;
  float* Fp = at<float>(ctx, oF);
  float* Op = at<float>(ctx, oO);
  HIP_TRY(nmfk::pad_rows<float>(F, n, k, Fp, KP, ctx->stream));
  nmfk::CsrLongRows lr;
  HIP_TRY(nmfk::csr_long_rows(rowptr, m, nnz, KP, at<char>(ctx, oL), &lr, ctx->stream));
  HIP_TRY(nmfk::csr_spmm(rowptr, colidx, vals, m, Fp, KP, Op, &lr, ctx->stream));
  HIP_TRY(nmfk::unpad_rows<float>(Op, m, k, KP, P, ctx->stream));
  return NMF_OK;
}

nmf_status nmf_csr_transpose(nmf_ctx* ctx, int64_t m, int64_t n, int64_t nnz,
                             const int64_t* rowptr, const int32_t* colidx, const float* vals,
                             int64_t* rowptr_t, int32_t* colidx_t, float* vals_t) {
  nmf_status s = check_common(ctx, m, n, 1);
  if (s != NMF_OK) return s;
  if (!rowptr || !rowptr_t || (nnz > 0 && (!colidx || !vals || !colidx_t || !vals_t)))
    return fail(ctx, NMF_EINVAL, "null CSR array");
  if (nnz < 0 || nnz > (int64_t)UINT32_MAX || n > INT32_MAX || m > INT32_MAX)
    return fail(ctx, NMF_EINVAL, "bad sizes");
  if ((s = bind_device(ctx)) != NMF_OK) return s;
  Carve cv;
  const size_t oT = cv.take<char>(nmfk::csr_transpose_work_bytes(m, n, nnz));
  if ((s = ensure_ws(ctx, cv.off)) != NMF_OK) return s;
  HIP_TRY(nmfk::csr_transpose(rowptr, colidx, vals, m, n, nnz, rowptr_t, colidx_t, vals_t,
                              at<char>(ctx, oT), ctx->stream));
  return NMF_OK;
}

nmf_status nmf_update(nmf_ctx* ctx, nmf_algo algo, nmf_dtype dtype, int64_t rows, int k,
                      const void* G, const void* P, void* X, const nmf_opts* opts,
                      long long* pivots) {
  nmf_status s = check_common(ctx, rows, 1, k);
  if (s != NMF_OK) return s;
  if (!G || !P || !X) return fail(ctx, NMF_EINVAL, "null G, P or X");
  nmf_opts o;
  nmf_default_opts(&o);
  if (opts) o = *opts;
  o.algo = algo;
  if ((s = check_opts(ctx, &o, k, false)) != NMF_OK) return s;
  if ((s = bind_device(ctx)) != NMF_OK) return s;
  if (dtype == NMF_F32)
    return update_impl<float>(ctx, algo, rows, k, (const float*)G, (const float*)P, (float*)X, &o,
                              pivots);
  if (dtype == NMF_F64)
    return update_impl<double>(ctx, algo, rows, k, (const double*)G, (const double*)P,
                               (double*)X, &o, pivots);
  return fail(ctx, NMF_EINVAL, "unknown dtype");
}

nmf_status nmf_update_noalloc(nmf_ctx* ctx, nmf_algo algo, nmf_dtype dtype, int64_t rows, int k,
                              const void* G, const void* P, void* X, const nmf_opts* opts,
                              long long* pivots) {
  nmf_status s = check_common(ctx, rows, 1, k);
  if (s != NMF_OK) return s;
  if (!G || !P || !X) return fail(ctx, NMF_EINVAL, "null G, P or X");
  if (dtype != NMF_F32 && dtype != NMF_F64) return fail(ctx, NMF_EINVAL, "unknown dtype");
  nmf_opts o;
  nmf_default_opts(&o);
  if (opts) o = *opts;
  o.algo = algo;
  if ((s = check_opts(ctx, &o, k, false)) != NMF_OK) return s;
  const int KP = kp_dense(k);
  const size_t need = dtype == NMF_F32 ? noalloc_plan<float>(rows, KP).total
                                       : noalloc_plan<double>(rows, KP).total;
  if (need > (size_t)NMF_NOALLOC_SCRATCH_BYTES)
    return fail(ctx, NMF_EINVAL,
                "nmf_update_noalloc: " + std::to_string(rows) + " rows at k = " +
                    std::to_string(k) + " need " + std::to_string(need) +
                    " bytes of scratch, more than the fixed " +
                    std::to_string((size_t)NMF_NOALLOC_SCRATCH_BYTES) + " (use nmf_update)");
  if ((s = bind_device(ctx)) != NMF_OK) return s;
  if (!ctx->scratch) {
    hipError_t e;
    ctx->scratch = scratch_address(ctx->device, &e);
    if (!ctx->scratch)
      return fail(ctx, NMF_EDEVICE,
                  std::string("scratch array address lookup failed: ") + hipGetErrorString(e));
  }
  if (dtype == NMF_F32)
    return update_noalloc_impl<float>(ctx, algo, rows, k, (const float*)G, (const float*)P,
                                      (float*)X, &o, pivots);
  return update_noalloc_impl<double>(ctx, algo, rows, k, (const double*)G, (const double*)P,
                                     (double*)X, &o, pivots);
}

nmf_status nmf_hals_normalize(nmf_ctx* ctx, nmf_dtype dtype, int64_t m, int64_t n, int k,
                              void* W, void* Ht, void* S, void* norms) {
  nmf_status s = check_common(ctx, m, n, k);
  if (s != NMF_OK) return s;
  if (!W || !Ht) return fail(ctx, NMF_EINVAL, "null W or Ht");
  if ((s = bind_device(ctx)) != NMF_OK) return s;
  if (dtype == NMF_F32)
    return normalize_impl<float>(ctx, m, n, k, (float*)W, (float*)Ht, (float*)S, (float*)norms);
  if (dtype == NMF_F64)
    return normalize_impl<double>(ctx, m, n, k, (double*)W, (double*)Ht, (double*)S,
                                  (double*)norms);
  return fail(ctx, NMF_EINVAL, "unknown dtype");
}

nmf_status nmf_dense_relerr(nmf_ctx* ctx, nmf_dtype dtype, int64_t m, int64_t n, const void* A,
                            int64_t lda, int k, const void* W, const void* Ht, double* out) {
  nmf_status s = check_common(ctx, m, n, k);
  if (s != NMF_OK) return s;
  if (!A || !W || !Ht || !out) return fail(ctx, NMF_EINVAL, "null argument");
  if (lda < n) return fail(ctx, NMF_EINVAL, "lda < n");
  if ((s = bind_device(ctx)) != NMF_OK) return s;
  if (dtype == NMF_F32) {
    Prob<float> pb;
    pb.A = (const float*)A;
    pb.lda = lda;
    return relerr_impl<float>(ctx, pb, m, n, k, (const float*)W, (const float*)Ht, out);
  }
  if (dtype == NMF_F64) {
    Prob<double> pb;
    pb.A = (const double*)A;
    pb.lda = lda;
    return relerr_impl<double>(ctx, pb, m, n, k, (const double*)W, (const double*)Ht, out);
  }
  if (is_lp(dtype)) {
    if ((s = check_lp_a(ctx, dtype, A, lda)) != NMF_OK) return s;
    Prob<float> pb;
    pb.lp = dtype;
    pb.Alp = A;
    pb.lda = lda;
    return relerr_impl<float>(ctx, pb, m, n, k, (const float*)W, (const float*)Ht, out);
  }
  return fail(ctx, NMF_EINVAL, "unknown dtype");
}

nmf_status nmf_csr_relerr(nmf_ctx* ctx, int64_t m, int64_t n, int64_t nnz, const int64_t* rowptr,
                          const int32_t* colidx, const float* vals, int k, const float* W,
                          const float* Ht, double* out) {
  nmf_status s = check_common(ctx, m, n, k);
  if (s != NMF_OK) return s;
  if (!rowptr || !W || !Ht || !out || (nnz > 0 && (!colidx || !vals)))
    return fail(ctx, NMF_EINVAL, "null argument");
  if (nnz < 0) return fail(ctx, NMF_EINVAL, "bad nnz");
  if ((s = bind_device(ctx)) != NMF_OK) return s;
  Prob<float> pb;
  pb.sparse = true;
  pb.rp = rowptr;
  pb.ci = colidx;
  pb.cv = vals;
  pb.nnz = nnz;
  return relerr_impl<float>(ctx, pb, m, n, k, W, Ht, out);
}

}  // extern "C"

// ===========================================================================
// Differentiation of T unrolled MU iterations (Section 4.1, Eq. (3)).
// ===========================================================================
namespace {

int64_t mu_ckpt_count(int iters, int every) { return iters <= 0 ? 0 : cdiv(iters, every); }

// Buffers shared by the forward and backward passes.
template <typename T> struct MuWork {
  T *W, *Ht, *P, *R, *Q, *S, *Ft, *part;
};

template <typename T>
size_t mu_plan_common(int64_t m, int64_t n, int KP, Carve& cv, size_t off[8]) {
  const int64_t mx = std::max(m, n);
  const int64_t ps = std::max({nmfk::gemm_auto_splits<T>(nmfk::GemmKind::NN, m, KP, n),
                               nmfk::gemm_auto_splits<T>(nmfk::GemmKind::TN, m, KP, n),
                               nmfk::gemm_auto_splits<T>(nmfk::GemmKind::TN, n, KP, m),
                               nmfk::gemm_auto_splits<T>(nmfk::GemmKind::NN, n, KP, m),
                               (int64_t)1});
  const int64_t part = std::max<int64_t>(ps * mx * KP, gram_splits(mx) * KP * KP);
  off[0] = cv.take<T>(m * KP);
  off[1] = cv.take<T>(n * KP);
  off[2] = cv.take<T>(m * KP);
  off[3] = cv.take<T>(n * KP);
  off[4] = cv.take<T>(KP * KP);
  off[5] = cv.take<T>(KP * KP);
  off[6] = cv.take<T>(mx * KP);
  off[7] = cv.take<T>(part);
  return cv.off;
}

template <typename T>
MuWork<T> mu_bind(nmf_ctx* ctx, const size_t off[8]) {
  return MuWork<T>{at<T>(ctx, off[0]), at<T>(ctx, off[1]), at<T>(ctx, off[2]),
                   at<T>(ctx, off[3]), at<T>(ctx, off[4]), at<T>(ctx, off[5]),
                   at<T>(ctx, off[6]), at<T>(ctx, off[7])};
}

// Rank-side operands of the dense products are read from a transposed copy
// (w.Ft) when its rows are 16-byte aligned. ft_ready: the producer of F has
// already written that copy. With parts set, a split product stays in its
// slabs (in w.part) for the consumer to sum; otherwise Out receives it.
template <typename T>
nmf_status mu_prod_AF(nmf_ctx* ctx, const Prob<T>& pb, int64_t m, int64_t n, const T* F, int k,
                      int KP, T* Out, MuWork<T>& w, bool ft_ready = false,
                      nmfk::Split<T>* parts = nullptr) {
  const bool tf = (n * (int64_t)sizeof(T)) % 16 == 0;
  if (tf && !ft_ready) HIP_TRY(nmfk::transpose_rows<T>(F, n, KP, w.Ft, ctx->stream));
  int ns = 1;
  nmf_status s = product_AF<T>(ctx, pb, m, n, F, tf ? w.Ft : nullptr, k, KP, Out, w.part,
                               parts ? &ns : nullptr);
  if (parts) *parts = nmfk::Split<T>{ns > 1 ? w.part : Out, ns, m * KP};
  return s;
}

template <typename T>
nmf_status mu_prod_AtF(nmf_ctx* ctx, const Prob<T>& pb, int64_t m, int64_t n, const T* F, int k,
                       int KP, T* Out, MuWork<T>& w, bool ft_ready = false,
                       nmfk::Split<T>* parts = nullptr) {
  const bool tf = (m * (int64_t)sizeof(T)) % 16 == 0;
  if (tf && !ft_ready) HIP_TRY(nmfk::transpose_rows<T>(F, m, KP, w.Ft, ctx->stream));
  int ns = 1;
  nmf_status s = product_AtF<T>(ctx, pb, m, n, F, tf ? w.Ft : nullptr, k, KP, Out, w.part,
                                parts ? &ns : nullptr);
  if (parts) *parts = nmfk::Split<T>{ns > 1 ? w.part : Out, ns, n * KP};
  return s;
}

// Whether a row kernel can hand a rows x KP factor to the next product as the
// transposed copy directly (the product reads one for these rows).
template <typename T>
bool rows_transposable(int64_t rows, int KP) {
  return (rows * (int64_t)sizeof(T)) % 16 == 0 && KP <= 64;
}

// One MU iteration from (W, Ht) into (Wn, Htn) (which may alias W, Ht),
// leaving Q = H H^T and S = Wn^T Wn in the given buffers (and their
// transposes in Qt and St where set), and P = A H^T and R = A^T Wn where P
// and R are set (nullable). The products reach the updates as their split
// slabs. *ft: on entry, whether w.Ft holds Ht's transposed copy; on return,
// whether it holds Htn's (the update writes it for the next iteration's
// product). With gsl set (room for plan_shares' blocks), the Grams are
// summed from row-block shares where plan_shares takes them: each update
// writes the shares of its output's Gram into gsl, and *qready says whether
// gsl holds Ht's on entry (else they are formed here); on return it holds
// Htn's. The shares' blocking and order are the same whichever kernel forms
// them, so a recomputation from a checkpoint repeats the Grams of the first
// pass bit for bit.
template <typename T>
nmf_status mu_iteration(nmf_ctx* ctx, const Prob<T>& pb, int64_t m, int64_t n, int k, int KP,
                        T eps, const T* W, const T* Ht, T* Wn, T* Htn, T* P, T* Q, T* R, T* S,
                        MuWork<T>& w, bool* ft, T* Qt = nullptr, T* St = nullptr,
                        T* gsl = nullptr, bool* qready = nullptr) {
  hipStream_t st = ctx->stream;
  nmf_status s;
  const bool tW = rows_transposable<T>(m, KP), tH = rows_transposable<T>(n, KP);
  nmfk::Split<T> sp;
  T* Pd = P ? P : w.P;
  T* Rd = R ? R : w.R;
  const Shares sh = gsl ? plan_shares(NMF_MU, m, n, KP) : Shares{};
  if (!sh.on()) gsl = nullptr;
  if (gsl) {
    if (!*qready) HIP_TRY(nmfk::gram_shares<T>(Ht, n, KP, sh.rpn, gsl, st));
    if ((s = sum_shares<T>(ctx, gsl, sh.nbn, KP, Q, Qt)) != NMF_OK) return s;
  } else if ((s = gram<T>(ctx, Ht, n, KP, Q, w.part, Qt)) != NMF_OK) {
    return s;
  }
  if ((s = mu_prod_AF<T>(ctx, pb, m, n, Ht, k, KP, Pd, w, *ft, &sp)) != NMF_OK) return s;
  HIP_TRY(nmfk::mu_rows<T>(W, Wn, sp, Q, m, k, KP, eps, tW ? w.Ft : nullptr,
                           sp.n > 1 ? P : nullptr, gsl, st));
  if (gsl) {
    if ((s = sum_shares<T>(ctx, gsl, sh.nbm, KP, S, St)) != NMF_OK) return s;
  } else if ((s = gram<T>(ctx, Wn, m, KP, S, w.part, St)) != NMF_OK) {
    return s;
  }
  if ((s = mu_prod_AtF<T>(ctx, pb, m, n, Wn, k, KP, Rd, w, tW, &sp)) != NMF_OK) return s;
  HIP_TRY(nmfk::mu_rows<T>(Ht, Htn, sp, S, n, k, KP, eps, tH ? w.Ft : nullptr,
                           sp.n > 1 ? R : nullptr, gsl, st));
  *ft = tH;
  if (gsl) *qready = true;
  return NMF_OK;
}

template <typename T>
nmf_status mu_prepare_A(nmf_ctx* ctx, const T* A, int64_t lda, int64_t m, int64_t n,
                        Prob<T>& pb) {
  pb.A = A;
  pb.lda = lda;
  return transposed_copy<T>(ctx, A, lda, m, n, m, &pb.At);
}

template <typename T>
nmf_status mu_forward_impl(nmf_ctx* ctx, int64_t m, int64_t n, const T* A, int64_t lda, int k,
                           int iters, T eps, int every, T* W, T* H, T* ckpt) {
  const int KP = kp_dense(k);
  Carve cv;
  size_t off[8];
  mu_plan_common<T>(m, n, KP, cv, off);
  // the updates' Gram shares
  const int64_t nbs = plan_shares(NMF_MU, m, n, KP).blocks();
  const size_t ogsl = cv.take<T>(nbs * KP * KP);
  nmf_status s = ensure_ws(ctx, cv.off);
  if (s != NMF_OK) return s;
  MuWork<T> w = mu_bind<T>(ctx, off);
  T* gsl = nbs > 0 ? at<T>(ctx, ogsl) : nullptr;
  hipStream_t st = ctx->stream;
  HIP_TRY(nmfk::pad_rows<T>(W, m, k, w.W, KP, st));
  HIP_TRY(nmfk::transpose_in<T>(H, k, n, w.Ht, KP, st));
  Prob<T> pb;
  if (iters > 0 && (s = mu_prepare_A<T>(ctx, A, lda, m, n, pb)) != NMF_OK) return s;
  const int64_t slot = (m + n) * KP;
  bool ft = false, qready = false;
  for (int t = 0; t < iters; ++t) {
    if (ckpt && t % every == 0) {
      T* c = ckpt + (int64_t)(t / every) * slot;
      HIP_TRY(hipMemcpyAsync(c, w.W, sizeof(T) * m * KP, hipMemcpyDeviceToDevice, st));
      HIP_TRY(hipMemcpyAsync(c + m * KP, w.Ht, sizeof(T) * n * KP, hipMemcpyDeviceToDevice, st));
    }
    s = mu_iteration<T>(ctx, pb, m, n, k, KP, eps, w.W, w.Ht, w.W, w.Ht, nullptr, w.Q, nullptr,
                        w.S, w, &ft, nullptr, nullptr, gsl, &qready);
    if (s != NMF_OK) return s;
  }
  HIP_TRY(nmfk::unpad_rows<T>(w.W, m, k, KP, W, st));
  HIP_TRY(nmfk::transpose_out<T>(w.Ht, k, n, KP, H, st));
  return NMF_OK;
}

template <typename T>
nmf_status mu_backward_impl(nmf_ctx* ctx, int64_t m, int64_t n, const T* A, int64_t lda, int k,
                            int iters, T eps, int every, const T* ckpt, const T* gWT,
                            const T* gHT, T* gA, int64_t ldga, T* gW0, T* gH0) {
  const int KP = kp_dense(k);
  const int64_t mx = std::max(m, n);
  const int seg = std::min(every, std::max(iters, 1));
  Carve cv;
  size_t off[8];
  mu_plan_common<T>(m, n, KP, cv, off);
  const size_t oWs = cv.take<T>((seg + 1) * m * KP);   // W_t over one segment
  const size_t oHs = cv.take<T>((seg + 1) * n * KP);   // H_t^T over one segment
  const size_t oPs = cv.take<T>(seg * m * KP);         // A H_t^T
  const size_t oRs = cv.take<T>(seg * n * KP);         // A^T W_{t+1}
  const size_t oQs = cv.take<T>(seg * KP * KP);
  const size_t oSs = cv.take<T>(seg * KP * KP);
  const size_t oQts = cv.take<T>(seg * KP * KP);       // their transposes
  const size_t oSts = cv.take<T>(seg * KP * KP);
  const size_t ogRs = cv.take<T>(seg * n * KP);        // dL/dR_t over one segment
  const size_t ogPs = cv.take<T>(seg * m * KP);        // dL/dP_t over one segment
  const size_t ogW = cv.take<T>(m * KP);
  const size_t ogH = cv.take<T>(n * KP);
  const size_t ogW2 = cv.take<T>(m * KP);
  const size_t ogH2 = cv.take<T>(n * KP);
  const size_t ogD = cv.take<T>(mx * KP);
  const size_t otmp = cv.take<T>(mx * KP);
  const size_t ogG = cv.take<T>(KP * KP);
  const size_t ogGt = cv.take<T>(KP * KP);
  const size_t ogGs = cv.take<T>(KP * KP);
  // the adjoints' per-block shares of the Gram gradients
  const int64_t nbm = nmfk::mu_adjoint_blocks<T>(m, KP), nbn = nmfk::mu_adjoint_blocks<T>(n, KP);
  const size_t ogsl = cv.take<T>(std::max(nbm, nbn) * KP * KP);
  // the recomputation's Gram shares
  const int64_t nbs = plan_shares(NMF_MU, m, n, KP).blocks();
  const size_t orsl = cv.take<T>(nbs * KP * KP);
  nmf_status s = ensure_ws(ctx, cv.off);
  if (s != NMF_OK) return s;
  MuWork<T> w = mu_bind<T>(ctx, off);
  T *Ws = at<T>(ctx, oWs), *Hs = at<T>(ctx, oHs), *Ps = at<T>(ctx, oPs), *Rs = at<T>(ctx, oRs);
  T *Qs = at<T>(ctx, oQs), *Ss = at<T>(ctx, oSs), *gRs = at<T>(ctx, ogRs), *gPs = at<T>(ctx, ogPs);
  T *gW = at<T>(ctx, ogW), *gH = at<T>(ctx, ogH), *gW2 = at<T>(ctx, ogW2), *gH2 = at<T>(ctx, ogH2);
  T *gD = at<T>(ctx, ogD), *tmp = at<T>(ctx, otmp), *gG = at<T>(ctx, ogG), *gGs = at<T>(ctx, ogGs);
  T *Qts = at<T>(ctx, oQts), *Sts = at<T>(ctx, oSts), *gGt = at<T>(ctx, ogGt);
  T* gsl = at<T>(ctx, ogsl);
  T* rsl = nbs > 0 ? at<T>(ctx, orsl) : nullptr;
  hipStream_t st = ctx->stream;
  const bool tW = rows_transposable<T>(m, KP), tH = rows_transposable<T>(n, KP);
  HIP_TRY(nmfk::pad_rows<T>(gWT, m, k, gW, KP, st));
  HIP_TRY(nmfk::transpose_in<T>(gHT, k, n, gH, KP, st));
  if (gA && iters == 0) HIP_TRY(hipMemset2DAsync(gA, ldga * sizeof(T), 0, n * sizeof(T), m, st));
  Prob<T> pb;
  if (iters > 0 && (s = mu_prepare_A<T>(ctx, A, lda, m, n, pb)) != NMF_OK) return s;
  const int64_t slot = (m + n) * KP;
  const int64_t nck = mu_ckpt_count(iters, every);
  // After the first reverse step, the gradient reaching a factor has three
  // parts: the direct term of the later half-step's adjoint (gW, gH), what
  // that half-step's product passes back (tmp = A gR or A^T gP) and what its
  // Gram passes back (X (gG + gG^T)); the adjoint kernel adds the last two.
  bool pre = false;
  nmfk::Split<T> yp{nullptr, 0, 0};
  for (int64_t j = nck - 1; j >= 0; --j) {
    const int t0 = (int)(j * every);
    const int L = std::min(iters, t0 + every) - t0;
    // recompute the segment's states from its checkpoint
    HIP_TRY(hipMemcpyAsync(Ws, ckpt + j * slot, sizeof(T) * m * KP, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(Hs, ckpt + j * slot + m * KP, sizeof(T) * n * KP,
                           hipMemcpyDeviceToDevice, st));
    bool ft = false, qready = false;
    for (int i = 0; i < L; ++i) {
      s = mu_iteration<T>(ctx, pb, m, n, k, KP, eps, Ws + i * m * KP, Hs + i * n * KP,
                          Ws + (i + 1) * m * KP, Hs + (i + 1) * n * KP, Ps + i * m * KP,
                          Qs + i * KP * KP, Rs + i * n * KP, Ss + i * KP * KP, w, &ft,
                          Qts + i * KP * KP, Sts + i * KP * KP, rsl, &qready);
      if (s != NMF_OK) return s;
    }
    for (int i = L - 1; i >= 0; --i) {
      const T* W0s = Ws + i * m * KP;
      const T* W1s = Ws + (i + 1) * m * KP;
      const T* H0s = Hs + i * n * KP;
      const T* H1s = Hs + (i + 1) * n * KP;
      T* gR = gRs + i * n * KP;
      T* gP = gPs + i * m * KP;
      // H step: Ht' = Ht * R / (Ht S + eps), R = A^T W1, S = W1^T W1
      HIP_TRY(nmfk::mu_adjoint_rows<T>(H0s, H1s, Rs + i * n * KP, Ss + i * KP * KP,
                                       Sts + i * KP * KP, gH,
                                       pre ? yp : nmfk::Split<T>{nullptr, 0, 0},
                                       pre ? gG : nullptr, gGt, n, k, KP, eps, gR,
                                       tH ? w.Ft : nullptr, gD, gH2, gsl, st));
      // dL/dS = H0^T gD: the adjoint's per-block shares, summed in order
      HIP_TRY(nmfk::reduce_splits<T>(gsl, (int)nbn, KP * KP, KP, KP, KP, gG, KP, st, gGt));
      if ((s = mu_prod_AF<T>(ctx, pb, m, n, gR, k, KP, tmp, w, tH, &yp)) != NMF_OK) return s;
      // W step: W1 = W0 * P / (W0 Q + eps), P = A H0^T, Q = H0 H0^T; the
      // gradient reaching W1 is gW + A gR + W1 (gG + gG^T)
      HIP_TRY(nmfk::mu_adjoint_rows<T>(W0s, W1s, Ps + i * m * KP, Qs + i * KP * KP,
                                       Qts + i * KP * KP, gW, yp, gG, gGt, m, k, KP, eps, gP,
                                       tW ? w.Ft : nullptr, gD, gW2, gsl, st));
      HIP_TRY(nmfk::reduce_splits<T>(gsl, (int)nbm, KP * KP, KP, KP, KP, gG, KP, st, gGt));
      // A^T gP reaches the next H step as slabs, except across a segment
      // boundary (the recomputation reuses w.part) and at the end
      if (i > 0) {
        if ((s = mu_prod_AtF<T>(ctx, pb, m, n, gP, k, KP, tmp, w, tW, &yp)) != NMF_OK) return s;
      } else {
        if ((s = mu_prod_AtF<T>(ctx, pb, m, n, gP, k, KP, tmp, w, tW)) != NMF_OK) return s;
        yp = nmfk::Split<T>{tmp, 1, 0};
      }
      pre = true;
      std::swap(gW, gW2);
      std::swap(gH, gH2);
    }
    // dL/dA (+)= sum over the segment of W_{t+1} gR_t^T (from R = A^T W1)
    // + gP_t H_t (from P = A H0^T); the last segment (first in this loop)
    // writes D, the others add to it
    if (gA)
      HIP_TRY(nmfk::rank_update<T>(gA, ldga, m, n, Ws + m * KP, gRs, gPs, Hs, KP, L,
                                   j == nck - 1 ? 0 : 1, st));
  }
  if (pre) {
    // H_0 also fed the first W step: dL/dH_0 += A^T gP_0 + H_0 (gG + gG^T)
    HIP_TRY(nmfk::add_to<T>(gH, tmp, n * KP, st));
    HIP_TRY(nmfk::symmetrize<T>(gG, KP, gGs, st));
    HIP_TRY(nmfk::rowmm_add<T>(Hs, gGs, n, k, KP, gH, st));
  }
  HIP_TRY(nmfk::unpad_rows<T>(gW, m, k, KP, gW0, st));
  HIP_TRY(nmfk::transpose_out<T>(gH, k, n, KP, gH0, st));
  return NMF_OK;
}

// ---------------------------------------------------------------------------
// Differentiation of T unrolled HALS iterations (Section 4.2, Eq. (5)).
// ---------------------------------------------------------------------------

// One HALS iteration from (W, Ht) into (Wn, Htn) (which may alias W, Ht) in
// the order nmf_dense runs it: Q = H H^T, P = A H^T, the W sweep, S = W^T W,
// the normalisation (W, H and S rescaled; norms into nrm), R = A^T W, the H
// sweep. Wp and Hc (nullable) receive W after the sweep and H^T after the
// rescaling, which the backward pass needs; every step writes its output
// where the next one reads it, so nothing is copied. *ft: on entry, whether
// w.Ft holds Ht's transposed copy; on return, whether it holds Htn's. gsl
// and *qready: the Gram shares, as for mu_iteration (with the sweeps'
// blocking).
template <typename T>
nmf_status hals_iteration(nmf_ctx* ctx, const Prob<T>& pb, int64_t m, int64_t n, int k, int KP,
                          const T* W, const T* Ht, T* Wn, T* Htn, T* Wp, T* Hc, T* nrm, T* Q,
                          T* S, MuWork<T>& w, bool* ft, T* gsl, bool* qready) {
  hipStream_t st = ctx->stream;
  nmf_status s;
  const bool tH = rows_transposable<T>(n, KP);
  nmfk::Split<T> sp;
  T* Wsw = Wp ? Wp : Wn;    // the W sweep's output
  T* Hsc = Hc ? Hc : Htn;   // H^T after the rescaling
  const Shares sh = gsl ? plan_shares(NMF_HALS, m, n, KP) : Shares{};
  if (!sh.on()) gsl = nullptr;
  if (gsl) {
    if (!*qready) HIP_TRY(nmfk::gram_shares<T>(Ht, n, KP, sh.rpn, gsl, st));
    if ((s = sum_shares<T>(ctx, gsl, sh.nbn, KP, Q)) != NMF_OK) return s;
  } else if ((s = gram<T>(ctx, Ht, n, KP, Q, w.part)) != NMF_OK) {
    return s;
  }
  if ((s = mu_prod_AF<T>(ctx, pb, m, n, Ht, k, KP, w.P, w, *ft, &sp)) != NMF_OK) return s;
  HIP_TRY(nmfk::hals_rows<T>(W, Wsw, sp, Q, m, k, KP, nullptr, gsl, st));
  if (gsl) {
    if ((s = sum_shares<T>(ctx, gsl, sh.nbm, KP, S)) != NMF_OK) return s;
  } else if ((s = gram<T>(ctx, Wsw, m, KP, S, w.part)) != NMF_OK) {
    return s;
  }
  // the normalisation writes Wn's transposed copy for the product (w.Ft, whose
  // copy of Ht the product above has read)
  const bool tW = rows_transposable<T>(m, KP);
  HIP_TRY(nmfk::hals_normalize<T>(Wsw, Wn, m, Ht, Hsc, n, S, nrm, k, KP, st,
                                  tW ? w.Ft : nullptr));
  if ((s = mu_prod_AtF<T>(ctx, pb, m, n, Wn, k, KP, w.R, w, tW, &sp)) != NMF_OK) return s;
  HIP_TRY(nmfk::hals_rows<T>(Hsc, Htn, sp, S, n, k, KP, tH ? w.Ft : nullptr, gsl, st));
  *ft = tH;
  if (gsl) *qready = true;
  return NMF_OK;
}

template <typename T>
nmf_status hals_forward_impl(nmf_ctx* ctx, int64_t m, int64_t n, const T* A, int64_t lda, int k,
                             int iters, int every, T* W, T* H, T* ckpt) {
  const int KP = kp_dense(k);
  Carve cv;
  size_t off[8];
  mu_plan_common<T>(m, n, KP, cv, off);
  const size_t onrm = cv.take<T>(KP);
  const int64_t nbs = plan_shares(NMF_HALS, m, n, KP).blocks();
  const size_t ogsl = cv.take<T>(nbs * KP * KP);   // the sweeps' Gram shares
  nmf_status s = ensure_ws(ctx, cv.off);
  if (s != NMF_OK) return s;
  MuWork<T> w = mu_bind<T>(ctx, off);
  T* nrm = at<T>(ctx, onrm);
  T* gsl = nbs > 0 ? at<T>(ctx, ogsl) : nullptr;
  hipStream_t st = ctx->stream;
  HIP_TRY(nmfk::pad_rows<T>(W, m, k, w.W, KP, st));
  HIP_TRY(nmfk::transpose_in<T>(H, k, n, w.Ht, KP, st));
  Prob<T> pb;
  if (iters > 0 && (s = mu_prepare_A<T>(ctx, A, lda, m, n, pb)) != NMF_OK) return s;
  const int64_t slot = (m + n) * KP;
  bool ft = false, qready = false;
  for (int t = 0; t < iters; ++t) {
    if (ckpt && t % every == 0) {
      T* c = ckpt + (int64_t)(t / every) * slot;
      HIP_TRY(hipMemcpyAsync(c, w.W, sizeof(T) * m * KP, hipMemcpyDeviceToDevice, st));
      HIP_TRY(hipMemcpyAsync(c + m * KP, w.Ht, sizeof(T) * n * KP, hipMemcpyDeviceToDevice, st));
    }
    s = hals_iteration<T>(ctx, pb, m, n, k, KP, w.W, w.Ht, w.W, w.Ht, nullptr, nullptr, nrm,
                          w.Q, w.S, w, &ft, gsl, &qready);
    if (s != NMF_OK) return s;
  }
  HIP_TRY(nmfk::unpad_rows<T>(w.W, m, k, KP, W, st));
  HIP_TRY(nmfk::transpose_out<T>(w.Ht, k, n, KP, H, st));
  return NMF_OK;
}

// Reverse pass, per iteration (H step first): the H sweep's adjoint gives
// dL/dHc and dL/dR (its deltas); R = A^T Wn and S = Wn^T Wn pass them on to
// Wn and A; the normalisation's adjoint gives dL/dW' and part of dL/dH; the
// W sweep's adjoint gives dL/dW and dL/dP; P = A H^T and Q = H H^T pass
// those on to H and A.
template <typename T>
nmf_status hals_backward_impl(nmf_ctx* ctx, int64_t m, int64_t n, const T* A, int64_t lda,
                              int k, int iters, int every, const T* ckpt, const T* gWT,
                              const T* gHT, T* gA, int64_t ldga, T* gW0, T* gH0) {
  const int KP = kp_dense(k);
  const int64_t mx = std::max(m, n);
  const int seg = std::min(every, std::max(iters, 1));
  Carve cv;
  size_t off[8];
  mu_plan_common<T>(m, n, KP, cv, off);
  const size_t oWs = cv.take<T>((seg + 1) * m * KP);   // W_t over one segment
  const size_t oHs = cv.take<T>((seg + 1) * n * KP);   // H_t^T over one segment
  const size_t oWp = cv.take<T>(seg * m * KP);         // W after the sweep
  const size_t oHc = cv.take<T>(seg * n * KP);         // H^T after the rescaling
  const size_t oNs = cv.take<T>(seg * KP);             // column norms
  const size_t oQs = cv.take<T>(seg * KP * KP);
  const size_t oSs = cv.take<T>(seg * KP * KP);
  const size_t ogW = cv.take<T>(m * KP);
  const size_t ogH = cv.take<T>(n * KP);
  const size_t ogW2 = cv.take<T>(m * KP);
  const size_t ogH2 = cv.take<T>(n * KP);
  const size_t ogRs = cv.take<T>(seg * n * KP);       // dL/dR_t over one segment
  const size_t ogPs = cv.take<T>(seg * m * KP);       // dL/dP_t over one segment
  const size_t ogHc = cv.take<T>(n * KP);
  const size_t ogWp = cv.take<T>(m * KP);
  const size_t otmp = cv.take<T>(mx * KP);
  const size_t oM = cv.take<T>(KP * KP);
  // the reverse sweeps' per-block shares of their two Gram products
  const int64_t hbm = nmfk::hals_adjoint_blocks<T>(m, KP), hbn = nmfk::hals_adjoint_blocks<T>(n, KP);
  const size_t otsl = cv.take<T>(2 * std::max(hbm, hbn) * KP * KP);
  // the recomputation's Gram shares
  const int64_t nbs = plan_shares(NMF_HALS, m, n, KP).blocks();
  const size_t orsl = cv.take<T>(nbs * KP * KP);
  const size_t odots = cv.take<double>(2 * KP);
  const size_t odpart = cv.take<double>(nmfk::coldot_partials(KP));
  nmf_status s = ensure_ws(ctx, cv.off);
  if (s != NMF_OK) return s;
  MuWork<T> w = mu_bind<T>(ctx, off);
  T *Ws = at<T>(ctx, oWs), *Hs = at<T>(ctx, oHs), *Wps = at<T>(ctx, oWp), *Hcs = at<T>(ctx, oHc);
  T *Ns = at<T>(ctx, oNs), *Qs = at<T>(ctx, oQs), *Ss = at<T>(ctx, oSs);
  T *gW = at<T>(ctx, ogW), *gH = at<T>(ctx, ogH), *gW2 = at<T>(ctx, ogW2), *gH2 = at<T>(ctx, ogH2);
  T *gRs = at<T>(ctx, ogRs), *gPs = at<T>(ctx, ogPs), *gHc = at<T>(ctx, ogHc);
  T* gWp = at<T>(ctx, ogWp);
  T *tmp = at<T>(ctx, otmp), *M = at<T>(ctx, oM);
  double *dots = at<double>(ctx, odots), *dpart = at<double>(ctx, odpart);
  T* tsl = at<T>(ctx, otsl);
  T* rsl = nbs > 0 ? at<T>(ctx, orsl) : nullptr;
  hipStream_t st = ctx->stream;
  const bool tW = rows_transposable<T>(m, KP), tH = rows_transposable<T>(n, KP);
  nmfk::Split<T> yp{nullptr, 0, 0};
  HIP_TRY(nmfk::pad_rows<T>(gWT, m, k, gW, KP, st));
  HIP_TRY(nmfk::transpose_in<T>(gHT, k, n, gH, KP, st));
  if (gA && iters == 0) HIP_TRY(hipMemset2DAsync(gA, ldga * sizeof(T), 0, n * sizeof(T), m, st));
  Prob<T> pb;
  if (iters > 0 && (s = mu_prepare_A<T>(ctx, A, lda, m, n, pb)) != NMF_OK) return s;
  const int64_t slot = (m + n) * KP;
  const int64_t nck = mu_ckpt_count(iters, every);
  for (int64_t j = nck - 1; j >= 0; --j) {
    const int t0 = (int)(j * every);
    const int L = std::min(iters, t0 + every) - t0;
    HIP_TRY(hipMemcpyAsync(Ws, ckpt + j * slot, sizeof(T) * m * KP, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(Hs, ckpt + j * slot + m * KP, sizeof(T) * n * KP,
                           hipMemcpyDeviceToDevice, st));
    bool ft = false, qready = false;
    for (int i = 0; i < L; ++i) {
      s = hals_iteration<T>(ctx, pb, m, n, k, KP, Ws + i * m * KP, Hs + i * n * KP,
                            Ws + (i + 1) * m * KP, Hs + (i + 1) * n * KP, Wps + i * m * KP,
                            Hcs + i * n * KP, Ns + i * KP, Qs + i * KP * KP, Ss + i * KP * KP, w,
                            &ft, rsl, &qready);
      if (s != NMF_OK) return s;
    }
    for (int i = L - 1; i >= 0; --i) {
      const T* W0s = Ws + i * m * KP;
      const T* W1s = Ws + (i + 1) * m * KP;   // normalised W, the H step's fixed factor
      const T* H0s = Hs + i * n * KP;
      const T* H1s = Hs + (i + 1) * n * KP;
      const T* Wp = Wps + i * m * KP;
      const T* Hc = Hcs + i * n * KP;
      T* gR = gRs + i * n * KP;
      T* gP = gPs + i * m * KP;
      // H sweep on the rows of Hc with R = A^T Wn and S = Wn^T Wn
      HIP_TRY(nmfk::hals_adjoint_rows<T>(H1s, Ss + i * KP * KP, gH, n, k, KP, gHc, gR,
                                         tH ? w.Ft : nullptr, Hc, tsl, st));
      // M from T1 = H1^T gR and T2 = Hc^T gR, summed from the blocks' shares
      HIP_TRY(nmfk::hals_gram_grad<T>(tsl, (int)hbn, KP, M, st));
      // gW += A gR (the product's slabs) + Wn M
      if ((s = mu_prod_AF<T>(ctx, pb, m, n, gR, k, KP, tmp, w, tH, &yp)) != NMF_OK) return s;
      HIP_TRY(nmfk::rowmm_add<T>(W1s, M, m, k, KP, gW, st, yp));
      // normalisation: Wn = W' / s, Hc = s H
      HIP_TRY(nmfk::coldot2<T>(gW, W1s, m, gHc, H0s, n, KP, dpart, dots, st));
      HIP_TRY(nmfk::hals_norm_adjoint<T>(gW, W1s, m, gHc, n, Ns + i * KP, dots, k, KP, gWp, gH2,
                                         st));
      // W sweep with P = A H^T and Q = H H^T
      HIP_TRY(nmfk::hals_adjoint_rows<T>(Wp, Qs + i * KP * KP, gWp, m, k, KP, gW2, gP,
                                         tW ? w.Ft : nullptr, W0s, tsl, st));
      HIP_TRY(nmfk::hals_gram_grad<T>(tsl, (int)hbm, KP, M, st));
      // gH += A^T gP (the product's slabs) + H M
      if ((s = mu_prod_AtF<T>(ctx, pb, m, n, gP, k, KP, tmp, w, tW, &yp)) != NMF_OK) return s;
      HIP_TRY(nmfk::rowmm_add<T>(H0s, M, n, k, KP, gH2, st, yp));
      std::swap(gW, gW2);
      std::swap(gH, gH2);
    }
    // dL/dA (+)= sum over the segment of Wn gR^T (from R = A^T Wn) + gP H^T
    // (from P = A H^T); the last segment (first in this loop) writes D
    if (gA)
      HIP_TRY(nmfk::rank_update<T>(gA, ldga, m, n, Ws + m * KP, gRs, gPs, Hs, KP, L,
                                   j == nck - 1 ? 0 : 1, st));
  }
  HIP_TRY(nmfk::unpad_rows<T>(gW, m, k, KP, gW0, st));
  HIP_TRY(nmfk::transpose_out<T>(gH, k, n, KP, gH0, st));
  return NMF_OK;
}

nmf_status mu_check(nmf_ctx* ctx, nmf_dtype dtype, int64_t m, int64_t n, const void* A,
                    int64_t lda, int k, int iters, double eps, int every) {
  nmf_status s = check_common(ctx, m, n, k);
  if (s != NMF_OK) return s;
  if (dtype != NMF_F32 && dtype != NMF_F64) return fail(ctx, NMF_EINVAL, "dtype must be F32 or F64");
  if (k > 64) return fail(ctx, NMF_EINVAL, "unrolled gradients support k <= 64");
  if (!A) return fail(ctx, NMF_EINVAL, "null A");
  if (lda < n) return fail(ctx, NMF_EINVAL, "lda < n");
  if (iters < 0 || every < 1) return fail(ctx, NMF_EINVAL, "iters < 0 or ckpt_every < 1");
  if (!(eps >= 0.0)) return fail(ctx, NMF_EINVAL, "eps must be >= 0");
  return NMF_OK;
}

}  // namespace

extern "C" {

int64_t nmf_mu_ckpt_elems(int64_t m, int64_t n, int k, int iters, int ckpt_every) {
  if (m < 1 || n < 1 || k < 1 || k > 64 || iters < 0 || ckpt_every < 1) return -1;
  return mu_ckpt_count(iters, ckpt_every) * (m + n) * (int64_t)kp_dense(k);
}

nmf_status nmf_mu_unrolled_forward(nmf_ctx* ctx, nmf_dtype dtype, int64_t m, int64_t n,
                                   const void* A, int64_t lda, int k, int iters, double eps,
                                   int ckpt_every, void* W, void* H, void* ckpt) {
  nmf_status s = mu_check(ctx, dtype, m, n, A, lda, k, iters, eps, ckpt_every);
  if (s != NMF_OK) return s;
  if (!W || !H) return fail(ctx, NMF_EINVAL, "null W or H");
  if ((s = bind_device(ctx)) != NMF_OK) return s;
  if (dtype == NMF_F32)
    return mu_forward_impl<float>(ctx, m, n, (const float*)A, lda, k, iters, (float)eps,
                                  ckpt_every, (float*)W, (float*)H, (float*)ckpt);
  return mu_forward_impl<double>(ctx, m, n, (const double*)A, lda, k, iters, eps, ckpt_every,
                                 (double*)W, (double*)H, (double*)ckpt);
}

nmf_status nmf_mu_unrolled_backward(nmf_ctx* ctx, nmf_dtype dtype, int64_t m, int64_t n,
                                    const void* A, int64_t lda, int k, int iters, double eps,
                                    int ckpt_every, const void* ckpt, const void* gW,
                                    const void* gH, void* gA, int64_t ldga, void* gW0,
                                    void* gH0) {
  nmf_status s = mu_check(ctx, dtype, m, n, A, lda, k, iters, eps, ckpt_every);
  if (s != NMF_OK) return s;
  if (!gW || !gH || !gW0 || !gH0 || (iters > 0 && !ckpt))
    return fail(ctx, NMF_EINVAL, "null checkpoint or gradient array");
  if (gA && ldga < n) return fail(ctx, NMF_EINVAL, "ldga < n");
  if ((s = bind_device(ctx)) != NMF_OK) return s;
  if (dtype == NMF_F32)
    return mu_backward_impl<float>(ctx, m, n, (const float*)A, lda, k, iters, (float)eps,
                                   ckpt_every, (const float*)ckpt, (const float*)gW,
                                   (const float*)gH, (float*)gA, ldga, (float*)gW0,
                                   (float*)gH0);
  return mu_backward_impl<double>(ctx, m, n, (const double*)A, lda, k, iters, eps, ckpt_every,
                                  (const double*)ckpt, (const double*)gW, (const double*)gH,
                                  (double*)gA, ldga, (double*)gW0, (double*)gH0);
}

nmf_status nmf_hals_unrolled_forward(nmf_ctx* ctx, nmf_dtype dtype, int64_t m, int64_t n,
                                     const void* A, int64_t lda, int k, int iters,
                                     int ckpt_every, void* W, void* H, void* ckpt) {
  nmf_status s = mu_check(ctx, dtype, m, n, A, lda, k, iters, 0.0, ckpt_every);
  if (s != NMF_OK) return s;
  if (!W || !H) return fail(ctx, NMF_EINVAL, "null W or H");
  if ((s = bind_device(ctx)) != NMF_OK) return s;
  if (dtype == NMF_F32)
    return hals_forward_impl<float>(ctx, m, n, (const float*)A, lda, k, iters, ckpt_every,
                                    (float*)W, (float*)H, (float*)ckpt);
  return hals_forward_impl<double>(ctx, m, n, (const double*)A, lda, k, iters, ckpt_every,
                                   (double*)W, (double*)H, (double*)ckpt);
}

nmf_status nmf_hals_unrolled_backward(nmf_ctx* ctx, nmf_dtype dtype, int64_t m, int64_t n,
                                      const void* A, int64_t lda, int k, int iters,
                                      int ckpt_every, const void* ckpt, const void* gW,
                                      const void* gH, void* gA, int64_t ldga, void* gW0,
                                      void* gH0) {
  nmf_status s = mu_check(ctx, dtype, m, n, A, lda, k, iters, 0.0, ckpt_every);
  if (s != NMF_OK) return s;
  if (!gW || !gH || !gW0 || !gH0 || (iters > 0 && !ckpt))
    return fail(ctx, NMF_EINVAL, "null checkpoint or gradient array");
  if (gA && ldga < n) return fail(ctx, NMF_EINVAL, "ldga < n");
  if ((s = bind_device(ctx)) != NMF_OK) return s;
  if (dtype == NMF_F32)
    return hals_backward_impl<float>(ctx, m, n, (const float*)A, lda, k, iters, ckpt_every,
                                     (const float*)ckpt, (const float*)gW, (const float*)gH,
                                     (float*)gA, ldga, (float*)gW0, (float*)gH0);
  return hals_backward_impl<double>(ctx, m, n, (const double*)A, lda, k, iters, ckpt_every,
                                    (const double*)ckpt, (const double*)gW, (const double*)gH,
                                    (double*)gA, ldga, (double*)gW0, (double*)gH0);
}

}  // extern "C"

namespace {
template <typename T>
nmf_status pgrad_impl(nmf_ctx* ctx, int64_t rows, int k, const T* X, const T* Pm, const T* G,
                      double* out) {
  const int KP = kp_dense(k);
  Carve cv;
  const size_t oX = cv.take<T>(rows * KP);
  const size_t oP = cv.take<T>(rows * KP);
  const size_t oG = cv.take<T>(KP * KP);
  const size_t oq = cv.take<double>(nmfk::pgrad_partials(rows));
  const size_t ov = cv.take<double>(1);
  nmf_status s = ensure_ws(ctx, cv.off);
  if (s != NMF_OK) return s;
  hipStream_t st = ctx->stream;
  T* Xp = at<T>(ctx, oX);
  T* Pp = at<T>(ctx, oP);
  T* Gp = at<T>(ctx, oG);
  HIP_TRY(nmfk::pad_rows<T>(X, rows, k, Xp, KP, st));
  HIP_TRY(nmfk::pad_rows<T>(Pm, rows, k, Pp, KP, st));
  HIP_TRY(nmfk::pad_rows<T>(G, k, k, Gp, KP, st));
  if (KP > k) HIP_TRY(hipMemsetAsync(Gp + (size_t)k * KP, 0, sizeof(T) * (KP - k) * KP, st));
  HIP_TRY(nmfk::pgrad_sq<T>(Xp, Pp, Gp, rows, k, KP, at<double>(ctx, oq), st));
  HIP_TRY(nmfk::finish_relerr<T>(at<double>(ctx, oq), nmfk::pgrad_blocks<T>(rows, KP),
                                 (const T*)nullptr, (const T*)nullptr, 0, (const double*)nullptr,
                                 at<double>(ctx, ov), st));
  return read_doubles(ctx, at<double>(ctx, ov), out, 1);
}
}  // namespace

extern "C" {

nmf_status nmf_projected_gradient_sq(nmf_ctx* ctx, nmf_dtype dtype, int64_t rows, int k,
                                     const void* X, const void* P, const void* G,
                                     double* out) {
  nmf_status s = check_common(ctx, rows, 1, k);
  if (s != NMF_OK) return s;
  if (!X || !P || !G || !out) return fail(ctx, NMF_EINVAL, "null argument");
  if ((s = bind_device(ctx)) != NMF_OK) return s;
  if (dtype == NMF_F32)
    return pgrad_impl<float>(ctx, rows, k, (const float*)X, (const float*)P, (const float*)G,
                             out);
  if (dtype == NMF_F64)
    return pgrad_impl<double>(ctx, rows, k, (const double*)X, (const double*)P,
                              (const double*)G, out);
  return fail(ctx, NMF_EINVAL, "dtype must be F32 or F64");
}

}  // extern "C"
