// Sparse A (CSR, float32): the large products A H^T and (W^T A)^T = A^T W of
// Algorithm 1 as row-wise SpMM, the one-time CSR transpose that gives A^T,
// and the sparse forms of the objective and input checks.
//
// SpMM layout: one wavefront per output row. The wave splits into groups of
// KP/4 lanes; each group takes one stored entry (j, a_ij) at a time and
// gathers the 16-byte slices of row j of the dense operand (n x KP, row
// major), so a group reads one whole dense row with one instruction and the
// wave keeps 64/(KP/4) gathers in flight per step. Group partial sums are
// combined with cross-lane shuffles at the end of the row, in a fixed order.
// Rows longer than CSR_LONG entries are cut into chunks of that length (one
// wave each) whose partials are added in chunk order.
#include <cstring>
#include <rocprim/device/device_radix_sort.hpp>

#include "common.h"
#include "grid.h"
#include "kernels.h"

namespace nmfk {

// Sum over the stored entries b..e-1 of a row of a_ij F[j] (one output row of
// KP floats), computed by the whole wave and returned, complete, in the
// lanes of group 0 (lane sub holds columns 4 sub .. 4 sub + 3).
template <int KP>
__device__ __forceinline__ float4 segment_sum(const int32_t* __restrict__ colidx,
                                              const float* __restrict__ vals,
                                              const float* __restrict__ F, int64_t b, int64_t e,
                                              int grp, int sub) {
  constexpr int LPN = KP / 4;     // lanes per stored entry
  constexpr int GPW = 64 / LPN;   // entries in flight per wave step
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
  int64_t p = b + grp;
  // unrolled by 4 entries per group
  for (; p + 3 * GPW < e; p += 4 * GPW) {
    int32_t j[4];
    float v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      j[u] = __builtin_nontemporal_load(colidx + p + u * GPW);
      v[u] = __builtin_nontemporal_load(vals + p + u * GPW);
    }
    float4 f[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) f[u] = *reinterpret_cast<const float4*>(F + (int64_t)j[u] * KP + 4 * sub);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      acc.x = fmaf(v[u], f[u].x, acc.x);
      acc.y = fmaf(v[u], f[u].y, acc.y);
      acc.z = fmaf(v[u], f[u].z, acc.z);
      acc.w = fmaf(v[u], f[u].w, acc.w);
    }
  }
  for (; p < e; p += GPW) {
    const int32_t j = colidx[p];
    const float v = vals[p];
    const float4 f = *reinterpret_cast<const float4*>(F + (int64_t)j * KP + 4 * sub);
    acc.x = fmaf(v, f.x, acc.x);
    acc.y = fmaf(v, f.y, acc.y);
    acc.z = fmaf(v, f.z, acc.z);
    acc.w = fmaf(v, f.w, acc.w);
  }
#pragma unroll
  for (int off = LPN; off < 64; off <<= 1) {
    acc.x += __shfl_xor(acc.x, off, 64);
    acc.y += __shfl_xor(acc.y, off, 64);
    acc.z += __shfl_xor(acc.z, off, 64);
    acc.w += __shfl_xor(acc.w, off, 64);
  }
  return acc;
}

// One wave per output row; rows with more than long_limit stored entries
// are left to the chunked path below.
template <int KP>
__global__ __launch_bounds__(256) void csr_spmm_kernel(const int64_t* __restrict__ rowptr,
                                                       const int32_t* __restrict__ colidx,
                                                       const float* __restrict__ vals,
                                                       int64_t m, const float* __restrict__ F,
                                                       float* __restrict__ P, int64_t long_limit) {
  constexpr int LPN = KP / 4;
  const int lane = threadIdx.x & 63;
  const int grp = lane / LPN, sub = lane % LPN;
  const int64_t wpb = blockDim.x >> 6, stride = (int64_t)gridDim.x * wpb;
  for (int64_t row = (int64_t)blockIdx.x * wpb + (threadIdx.x >> 6); row < m; row += stride) {
    const int64_t b = rowptr[row], e = rowptr[row + 1];
    if (e - b > long_limit) continue;
    const float4 acc = segment_sum<KP>(colidx, vals, F, b, e, grp, sub);
    if (grp == 0) *reinterpret_cast<float4*>(P + row * KP + 4 * sub) = acc;
  }
}

// Long rows (power-law sparsity puts much of the work in a few of them): each
// is cut into chunks of CSR_LONG stored entries, one wave per chunk writes
// its partial sums, and the partials of a row are then added in chunk order,
// so the result does not depend on scheduling.
constexpr int64_t CSR_LONG = 4096;

template <int KP>
__global__ __launch_bounds__(256) void csr_chunk_kernel(
    const int64_t* __restrict__ rowptr, const int32_t* __restrict__ colidx,
    const float* __restrict__ vals, const float* __restrict__ F, const int64_t* __restrict__ ids,
    const int64_t* __restrict__ chunk_off, int64_t nlong, int64_t nchunks,
    float* __restrict__ part) {
  constexpr int LPN = KP / 4;
  const int lane = threadIdx.x & 63;
  const int grp = lane / LPN, sub = lane % LPN;
  const int64_t c = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (c >= nchunks) return;
  // the long row that holds chunk c: the last i with chunk_off[i] <= c
  int64_t lo = 0, hi = nlong - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (chunk_off[mid] <= c) lo = mid;
    else hi = mid - 1;
  }
  const int64_t row = ids[lo];
  const int64_t b = rowptr[row] + (c - chunk_off[lo]) * CSR_LONG;
  const int64_t e = b + CSR_LONG < rowptr[row + 1] ? b + CSR_LONG : rowptr[row + 1];
  const float4 acc = segment_sum<KP>(colidx, vals, F, b, e, grp, sub);
  if (grp == 0) *reinterpret_cast<float4*>(part + c * KP + 4 * sub) = acc;
}

template <int KP>
__global__ __launch_bounds__(256) void csr_chunk_reduce_kernel(
    const int64_t* __restrict__ ids, const int64_t* __restrict__ chunk_off, int64_t nlong,
    const float* __restrict__ part, float* __restrict__ P) {
  constexpr int Q = KP / 4;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = t / Q;
  const int q = (int)(t % Q);
  if (i >= nlong) return;
  float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int64_t c = chunk_off[i]; c < chunk_off[i + 1]; ++c) {
    const float4 v = *reinterpret_cast<const float4*>(part + c * KP + 4 * q);
    s.x += v.x;
    s.y += v.y;
    s.z += v.z;
    s.w += v.w;
  }
  *reinterpret_cast<float4*>(P + ids[i] * KP + 4 * q) = s;
}

hipError_t csr_spmm(const int64_t* rowptr, const int32_t* colidx, const float* vals, int64_t m,
                    const float* F, int KP, float* P, const CsrLongRows* lr, hipStream_t st) {
  if (m <= 0) return hipSuccess;
  const bool split = lr != nullptr && lr->nlong > 0;
  const int64_t limit = split ? CSR_LONG : INT64_MAX;
  const unsigned blocks = capped_grid(cdiv(m, 4));
#define CASE(K)                                                                               \
  case K:                                                                                     \
    csr_spmm_kernel<K><<<blocks, 256, 0, st>>>(rowptr, colidx, vals, m, F, P, limit);         \
    if (split) {                                                                              \
      csr_chunk_kernel<K><<<(unsigned)cdiv(lr->nchunks, 4), 256, 0, st>>>(                    \
          rowptr, colidx, vals, F, lr->ids, lr->chunk_off, lr->nlong, lr->nchunks, lr->part);  \
      csr_chunk_reduce_kernel<K><<<(unsigned)cdiv(lr->nlong * (K / 4), 256), 256, 0, st>>>(    \
          lr->ids, lr->chunk_off, lr->nlong, lr->part, P);                                    \
    }                                                                                         \
    break;
  switch (KP) {
    CASE(16) CASE(32) CASE(64) CASE(128)
    default: return hipErrorInvalidValue;
  }
#undef CASE
  return NMF_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// CSR transpose: a stable radix sort of the entries by column, then the new
// row pointers from the sorted column ids (the first position of each
// column; a column without entries starts where the next column with
// entries does).
// ---------------------------------------------------------------------------
__global__ void fill_i64_kernel(int64_t* __restrict__ p, int64_t n, int64_t v) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) p[q] = v;
}

// rowptr_t[c] = first position of column c in the sorted ids, for every
// column with entries (the others keep -1).
__global__ void column_starts_kernel(const uint32_t* __restrict__ keys, int64_t nnz,
                                     int64_t* __restrict__ rowptr_t) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnz; p += stride)
    if (p == 0 || keys[p] != keys[p - 1]) rowptr_t[keys[p]] = p;
}

// Columns without entries: the first position whose id exceeds c (binary
// search over the sorted ids); rowptr_t[n] = nnz.
__global__ void empty_column_starts_kernel(const uint32_t* __restrict__ keys, int64_t nnz,
                                           int64_t n, int64_t* __restrict__ rowptr_t) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c > n) return;
  if (c == n) {
    rowptr_t[n] = nnz;
    return;
  }
  if (rowptr_t[c] >= 0) return;
  int64_t lo = 0, hi = nnz;
  while (lo < hi) {
    const int64_t mid = lo + ((hi - lo) >> 1);
    if ((int64_t)keys[mid] < c) lo = mid + 1;
    else hi = mid;
  }
  rowptr_t[c] = lo;
}

constexpr int SCAN_BLOCK = 1024;  // elements per block (256 threads x 4)

// Exclusive scan of 1024 int64 values held 4 per thread; returns block total.
__device__ int64_t block_exclusive_scan4(int64_t (&v)[4]) {
  __shared__ int64_t sh[256];
  const int t = threadIdx.x;
  int64_t s = v[0] + v[1] + v[2] + v[3];
  sh[t] = s;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const int64_t add = t >= off ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  const int64_t incl = sh[t];
  const int64_t total = sh[255];
  int64_t run = incl - s;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t x = v[q];
    v[q] = run;
    run += x;
  }
  __syncthreads();
  return total;
}

// Single block: exclusive scan of nb block sums, in place.
__global__ __launch_bounds__(256) void scan_top_kernel(int64_t* __restrict__ bsum, int64_t nb) {
  __shared__ int64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t c0 = 0; c0 < nb; c0 += SCAN_BLOCK) {
    int64_t v[4];
    const int64_t base = c0 + 4 * threadIdx.x;
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = base + q < nb ? bsum[base + q] : 0;
    const int64_t tot = block_exclusive_scan4(v);
    const int64_t cy = carry;
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (base + q < nb) bsum[base + q] = v[q] + cy;
    __syncthreads();
    if (threadIdx.x == 0) carry = cy + tot;
    __syncthreads();
  }
}

// One wave per source row: each stored entry's payload is its row id (high
// 32 bits) and its value's bits (low 32 bits).
__global__ __launch_bounds__(256) void entry_payload_kernel(const int64_t* __restrict__ rowptr,
                                                            int64_t m,
                                                            const float* __restrict__ vals,
                                                            uint64_t* __restrict__ pay) {
  const int lane = threadIdx.x & 63;
  const int64_t wpb = blockDim.x >> 6, stride = (int64_t)gridDim.x * wpb;
  for (int64_t i = (int64_t)blockIdx.x * wpb + (threadIdx.x >> 6); i < m; i += stride) {
    const uint64_t hi = (uint64_t)i << 32;
    for (int64_t p = rowptr[i] + lane; p < rowptr[i + 1]; p += 64)
      pay[p] = hi | (uint64_t)__float_as_uint(vals[p]);
  }
}

__global__ void unpack_payload_kernel(const uint64_t* __restrict__ pay, int64_t nnz,
                                      int32_t* __restrict__ colidx_t, float* __restrict__ vals_t) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nnz; q += stride) {
    const uint64_t v = pay[q];
    colidx_t[q] = (int32_t)(v >> 32);
    vals_t[q] = __uint_as_float((unsigned)(v & 0xffffffffu));
  }
}

// Key bits of the column ids (enough for n - 1).
static unsigned col_bits(int64_t n) {
  unsigned b = 1;
  while (b < 32 && ((int64_t)1 << b) < n) ++b;
  return b;
}

static size_t sort_temp_bytes(int64_t n, int64_t nnz) {
  size_t bytes = 0;
  if (nnz > 0)
    (void)rocprim::radix_sort_pairs(nullptr, bytes, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                                    (const uint64_t*)nullptr, (uint64_t*)nullptr, (size_t)nnz, 0u,
                                    col_bits(n), (hipStream_t)0);
  return bytes;
}

size_t csr_transpose_work_bytes(int64_t m, int64_t n, int64_t nnz) {
  (void)m;
  return round_up((size_t)nnz * 4, 256) + 2 * round_up((size_t)nnz * 8, 256) +
         round_up(sort_temp_bytes(n, nnz), 256);
}

// Counts per column and their exclusive scan give the new row pointers; a
// stable radix sort of the entries (in row-major order) by column then puts
// each new row's entries in increasing order of their source row, so the
// result is unique and the same on every run, whatever the row lengths.
hipError_t csr_transpose(const int64_t* rowptr, const int32_t* colidx, const float* vals,
                         int64_t m, int64_t n, int64_t nnz, int64_t* rowptr_t,
                         int32_t* colidx_t, float* vals_t, void* work, hipStream_t st) {
  char* w = (char*)work;
  uint32_t* keys_out = (uint32_t*)w;
  w += round_up((size_t)nnz * 4, 256);
  uint64_t* pay_in = (uint64_t*)w;
  w += round_up((size_t)nnz * 8, 256);
  uint64_t* pay_out = (uint64_t*)w;
  w += round_up((size_t)nnz * 8, 256);
  void* temp = w;
  hipError_t e;
  if (nnz == 0) {
    fill_i64_kernel<<<(unsigned)cdiv(n + 1, 256), 256, 0, st>>>(rowptr_t, n + 1, 0);
    return NMF_LAUNCH_CHECK();
  }
  entry_payload_kernel<<<capped_grid(cdiv(m, 4)), 256, 0, st>>>(rowptr, m, vals, pay_in);
  if ((e = NMF_LAUNCH_CHECK()) != hipSuccess) return e;
  size_t temp_bytes = sort_temp_bytes(n, nnz);
  e = rocprim::radix_sort_pairs(temp, temp_bytes, (const uint32_t*)colidx, keys_out, pay_in,
                                pay_out, (size_t)nnz, 0u, col_bits(n), st);
  if (e != hipSuccess) return e;
  fill_i64_kernel<<<(unsigned)cdiv(n + 1, 256), 256, 0, st>>>(rowptr_t, n + 1, -1);
  column_starts_kernel<<<capped_grid(cdiv(nnz, 256)), 256, 0, st>>>(keys_out, nnz, rowptr_t);
  empty_column_starts_kernel<<<(unsigned)cdiv(n + 1, 256), 256, 0, st>>>(keys_out, nnz, n,
                                                                         rowptr_t);
  if ((e = NMF_LAUNCH_CHECK()) != hipSuccess) return e;
  unpack_payload_kernel<<<capped_grid(cdiv(nnz, 256)), 256, 0, st>>>(pay_out, nnz, colidx_t,
                                                                  vals_t);
  return NMF_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Long rows of a CSR matrix for the chunked SpMM path (built once per call).
// ---------------------------------------------------------------------------
__global__ void find_long_kernel(const int64_t* __restrict__ rowptr, int64_t m, int64_t cap,
                                 int64_t* __restrict__ ids,
                                 unsigned long long* __restrict__ count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (rowptr[i + 1] - rowptr[i] > CSR_LONG) {
      const unsigned long long slot = atomicAdd(count, 1ull);
      if ((int64_t)slot < cap) ids[slot] = i;
    }
  }
}

// off[i] = chunks of long row ids[i] (i < nlong), off[nlong] = 0; an
// exclusive scan then turns off into the chunk offsets and off[nlong] into
// the chunk count.
__global__ void long_chunks_kernel(const int64_t* __restrict__ rowptr,
                                   const int64_t* __restrict__ ids, int64_t nlong,
                                   int64_t* __restrict__ off) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > nlong) return;
  off[i] = i < nlong ? cdiv(rowptr[ids[i] + 1] - rowptr[ids[i]], CSR_LONG) : 0;
}

static int64_t long_cap(int64_t nnz) { return nnz / CSR_LONG + 1; }

size_t csr_long_work_bytes(int64_t nnz, int KP) {
  const int64_t cap = long_cap(nnz);
  return 256 + round_up((size_t)cap * 8, 256) + round_up((size_t)(cap + 1) * 8, 256) +
         round_up((size_t)(2 * cap) * KP * 4, 256);
}

hipError_t csr_long_rows(const int64_t* rowptr, int64_t m, int64_t nnz, int KP, void* work,
                         CsrLongRows* out, hipStream_t st) {
  *out = CsrLongRows{};
  if (m <= 0 || nnz <= CSR_LONG) return hipSuccess;  // no row can be long
  const int64_t cap = long_cap(nnz);
  char* w = (char*)work;
  unsigned long long* count = (unsigned long long*)w;
  w += 256;
  int64_t* ids = (int64_t*)w;
  w += round_up((size_t)cap * 8, 256);
  int64_t* off = (int64_t*)w;
  w += round_up((size_t)(cap + 1) * 8, 256);
  float* part = (float*)w;
  hipError_t e = hipMemsetAsync(count, 0, sizeof(unsigned long long), st);
  if (e != hipSuccess) return e;
  const int64_t blocks = cdiv(m, 256) < 4096 ? cdiv(m, 256) : 4096;
  find_long_kernel<<<(unsigned)blocks, 256, 0, st>>>(rowptr, m, cap, ids, count);
  unsigned long long nlong = 0;
  if ((e = hipMemcpyAsync(&nlong, count, sizeof(nlong), hipMemcpyDeviceToHost, st)) != hipSuccess)
    return e;
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
  if (nlong == 0) return hipSuccess;
  if ((int64_t)nlong > cap) return hipErrorInvalidValue;  // a row longer than nnz allows
  long_chunks_kernel<<<(unsigned)cdiv((int64_t)nlong + 1, 256), 256, 0, st>>>(
      rowptr, ids, (int64_t)nlong, off);
  scan_top_kernel<<<1, 256, 0, st>>>(off, (int64_t)nlong + 1);
  int64_t nchunks = 0;
  if ((e = hipMemcpyAsync(&nchunks, off + nlong, sizeof(nchunks), hipMemcpyDeviceToHost, st)) !=
      hipSuccess)
    return e;
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
  if (nchunks > 2 * cap) return hipErrorInvalidValue;
  out->nlong = (int64_t)nlong;
  out->nchunks = nchunks;
  out->ids = ids;
  out->chunk_off = off;
  out->part = part;
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// Objective for sparse A: per stored entry (a - wh)^2 - wh^2, one lane per
// entry, the row of W read with wave-uniform loads.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

constexpr int RES_ROWS_PER_BLOCK = 64;

template <int KP>
__global__ __launch_bounds__(256) void csr_residual_kernel(const int64_t* __restrict__ rowptr,
                                                           const int32_t* __restrict__ colidx,
                                                           const float* __restrict__ vals,
                                                           int64_t m, const float* __restrict__ W,
                                                           const float* __restrict__ Ht,
                                                           double* __restrict__ partial) {
  __shared__ double sh[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double local = 0.0;
  const int64_t r0 = (int64_t)blockIdx.x * RES_ROWS_PER_BLOCK;
  for (int64_t i = r0 + wave; i < r0 + RES_ROWS_PER_BLOCK && i < m; i += 4) {
    const float* wr = W + i * KP;
    const int64_t b = rowptr[i], e = rowptr[i + 1];
    for (int64_t p = b + lane; p < e; p += 64) {
      const float* hr = Ht + (int64_t)colidx[p] * KP;
      float wh = 0.f;
#pragma unroll
      for (int q = 0; q < KP; q += 4) {
        const float4 h = *reinterpret_cast<const float4*>(hr + q);
        wh = fmaf(wr[q], h.x, wh);
        wh = fmaf(wr[q + 1], h.y, wh);
        wh = fmaf(wr[q + 2], h.z, wh);
        wh = fmaf(wr[q + 3], h.w, wh);
      }
      const double a = (double)vals[p], d = a - (double)wh;
      local += d * d - (double)wh * (double)wh;
    }
  }
  local = wave_sum_d(local);
  if (lane == 0) sh[wave] = local;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

int64_t csr_residual_partials(int64_t m) { return cdiv(m, RES_ROWS_PER_BLOCK); }

hipError_t csr_residual_sq(const int64_t* rowptr, const int32_t* colidx, const float* vals,
                           int64_t m, const float* W, const float* Ht, int KP, double* partial,
                           hipStream_t st) {
  const unsigned blocks = (unsigned)cdiv(m, RES_ROWS_PER_BLOCK);
  switch (KP) {
#define C(K) case K: csr_residual_kernel<K><<<blocks, 256, 0, st>>>(rowptr, colidx, vals, m, W, Ht, partial); break;
    C(16) C(32) C(48) C(64) C(80) C(96) C(112) C(128)
#undef C
    default: return hipErrorInvalidValue;
  }
  return NMF_LAUNCH_CHECK();
}

__global__ __launch_bounds__(256) void csr_sumsq_kernel(const float* __restrict__ vals,
                                                        int64_t nnz, double* __restrict__ partial) {
  __shared__ double sh[4];
  double local = 0.0;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnz;
       p += (int64_t)gridDim.x * blockDim.x) {
    const double a = vals[p];
    local += a * a;
  }
  local = wave_sum_d(local);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = local;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

hipError_t csr_sumsq(const float* vals, int64_t nnz, double* partial, int64_t np,
                     hipStream_t st) {
  csr_sumsq_kernel<<<(unsigned)np, 256, 0, st>>>(vals, nnz, partial);
  return NMF_LAUNCH_CHECK();
}

// CSR validity: rowptr nondecreasing from 0 to nnz, columns in range and
// strictly increasing within a row, values finite and >= 0.
__global__ void check_csr_kernel(const int64_t* __restrict__ rowptr,
                                 const int32_t* __restrict__ colidx,
                                 const float* __restrict__ vals, int64_t m, int64_t n,
                                 int64_t nnz, int* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const int64_t b = rowptr[i], e = rowptr[i + 1];
  // Row bounds are checked before any entry is read.
  int bad = (b < 0 || e < b || e > nnz || (i == 0 && b != 0) || (i == m - 1 && e != nnz)) ? 2 : 0;
  if (!bad) {
    int32_t prev = -1;
    for (int64_t p = b; p < e; ++p) {
      const int32_t j = colidx[p];
      const float v = vals[p];
      if (j < 0 || j >= n || j <= prev) { bad = 2; break; }
      if (!(v >= 0.f) || v == INFINITY) bad = bad ? bad : 1;
      prev = j;
    }
  }
  if (bad) atomicOr(flag, bad);
}

hipError_t check_csr(const int64_t* rowptr, const int32_t* colidx, const float* vals, int64_t m,
                     int64_t n, int64_t nnz, int* flag, hipStream_t st) {
  check_csr_kernel<<<(unsigned)cdiv(m, 256), 256, 0, st>>>(rowptr, colidx, vals, m, n, nnz, flag);
  return NMF_LAUNCH_CHECK();
}

}  // namespace nmfk
