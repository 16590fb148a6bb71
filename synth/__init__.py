"""Seeded synthetic inputs for NMF (A ~= W H, W, H >= 0).

This module only draws random numbers and assembles input matrices. It holds
none of the factorisation's arithmetic, and both the CPU oracle and the GPU
library consume what it returns (arrays, never code).

Workload shapes follow the paper's synthetic data sets (Section 6.1.1, "Data
Sets"): a dense low-rank matrix built as the product of two U(0,1) factors,
and an Erdos-Renyi sparse matrix in which every entry is nonzero
independently with a fixed probability. For the shapes of its web-crawl
data, a power-law sparsity generator stands in (powerlaw_csr_torch). The dense generator adds
|N(0, sigma)| noise so that the planted factorisation is not exact; the
initial factors are U(0,1) from their own seed, shared across the three
algorithms as Section 6.1.3 asks ("the same random seed" for the initial H).

All generators use numpy's PCG64 bit generator, so a (shape, seed) pair fixes
every value on every machine. The large dense workloads can also be drawn on
a GPU with torch (``planted_dense_torch``); that path is reproducible on one
device type and is only used where a host copy of the whole matrix would be
wasteful. Whatever array a generator returns is the authoritative input for
both sides.
"""
from __future__ import annotations

import dataclasses

import numpy as np

DATA_SEED = 1609
INIT_SEED = 9154


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform(shape, seed: int, dtype=np.float64) -> np.ndarray:
    """U(0,1) array of the given shape (float64 draw, then cast)."""
    return _rng(seed).random(shape, dtype=np.float64).astype(dtype, copy=False)


def init_factors(m: int, n: int, k: int, seed: int = INIT_SEED, dtype=np.float64):
    """Initial W0 (m x k) and H0 (k x n), entries U(0,1).

    H0 is drawn first from its own stream so that it does not depend on m:
    the same seed gives the same H0 for every algorithm and every m.
    """
    rng = _rng(seed)
    H0 = rng.random((k, n), dtype=np.float64)
    W0 = rng.random((m, k), dtype=np.float64)
    return W0.astype(dtype, copy=False), H0.astype(dtype, copy=False)


def planted_dense(m: int, n: int, k_true: int, sigma: float = 0.01,
                  seed: int = DATA_SEED, dtype=np.float64, return_factors=False):
    """A = W0 H0 + |N(0, sigma)|, with W0 (m x k_true), H0 (k_true x n) U(0,1).

    The product is formed in float64 and rounded once to ``dtype``. ``sigma``
    is the standard deviation of the normal before the absolute value.
    """
    rng = _rng(seed)
    W0 = rng.random((m, k_true), dtype=np.float64)
    H0 = rng.random((k_true, n), dtype=np.float64)
    A = W0 @ H0
    if sigma > 0:
        A += np.abs(rng.standard_normal((m, n), dtype=np.float64)) * sigma
    A = A.astype(dtype, copy=False)
    if return_factors:
        return A, W0, H0
    return A


def planted_dense_torch(m: int, n: int, k_true: int, sigma: float = 0.01,
                        seed: int = DATA_SEED, device="cuda", dtype=None,
                        row_block: int = 4096):
    """Device-side version of :func:`planted_dense` for matrices of many GB.

    W0 and H0 come from the same PCG64 stream as :func:`planted_dense`; the
    product and the noise are formed on ``device`` in float32 row blocks and
    the noise comes from torch's seeded generator on that device. The result
    is not bit-identical to the host version (different noise stream and
    rounding), so a caller that needs the values on the host copies the
    returned tensor back.
    """
    import torch

    dtype = dtype or torch.float32
    rng = _rng(seed)
    W0 = torch.from_numpy(rng.random((m, k_true), dtype=np.float64).astype(np.float32))
    H0 = torch.from_numpy(rng.random((k_true, n), dtype=np.float64).astype(np.float32))
    W0 = W0.to(device)
    H0 = H0.to(device)
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    A = torch.empty((m, n), dtype=dtype, device=device)
    for r0 in range(0, m, row_block):
        r1 = min(m, r0 + row_block)
        blk = W0[r0:r1].double() @ H0.double()
        if sigma > 0:
            noise = torch.randn((r1 - r0, n), generator=gen, device=device,
                                dtype=torch.float32).abs_().mul_(sigma)
            blk += noise.double()
        A[r0:r1] = blk.to(dtype)
    return A


@dataclasses.dataclass
class CSR:
    """Compressed sparse rows: int64 row pointers, int32 sorted column ids."""
    m: int
    n: int
    rowptr: np.ndarray  # (m+1,) int64
    colidx: np.ndarray  # (nnz,) int32, strictly increasing within a row
    vals: np.ndarray    # (nnz,) float32 or float64

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_dense(self) -> np.ndarray:
        D = np.zeros((self.m, self.n), dtype=np.float64)
        rows = np.repeat(np.arange(self.m), np.diff(self.rowptr))
        D[rows, self.colidx] = self.vals
        return D


def erdos_renyi_csr(m: int, n: int, density: float, seed: int = DATA_SEED,
                    dtype=np.float32, chunk: int = 1 << 24) -> CSR:
    """Every entry of an m x n matrix is nonzero with probability ``density``,
    independently; nonzero values are U(0,1).

    Positions are drawn exactly as a Bernoulli process over the row-major
    flattening of the matrix: the gaps between successive nonzeros are
    geometric(density). Columns within a row are therefore distinct and
    sorted, and row lengths are Binomial(n, density).
    """
    rng = _rng(seed)
    total = m * n
    pieces = []
    pos = -1
    while density > 0:
        gaps = rng.geometric(density, size=chunk).astype(np.int64)
        p = pos + np.cumsum(gaps)
        cut = np.searchsorted(p, total)
        pieces.append(p[:cut])
        if cut < chunk:
            break
        pos = int(p[-1])
    flat = np.concatenate(pieces) if pieces else np.zeros(0, np.int64)
    rows = flat // n
    cols = (flat - rows * n).astype(np.int32)
    counts = np.bincount(rows, minlength=m).astype(np.int64)
    rowptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    vals = rng.random(flat.size, dtype=np.float64).astype(dtype)
    return CSR(m, n, rowptr, cols, vals)


def powerlaw_csr_torch(m: int, n: int, nnz: int, seed: int = DATA_SEED, row_tail: float = 2.5,
                       col_skew: float = 0.7, device="cpu"):
    """Web-graph-like sparsity (a stand-in for the crawl matrices the paper
    factorises, such as webbase-2001): row lengths and column popularity
    both follow power laws.

    - Row lengths: w_i = u_i^(-1 / (row_tail - 1)) for u_i ~ U(0, 1]
      (a Pareto tail with exponent row_tail), scaled so that they sum to
      ``nnz`` and rounded stochastically, at most n.
    - Columns: each entry picks a popularity rank r in [0, n) from the
      density proportional to (r + 1)^(-col_skew) by inverse-CDF sampling,
      and the column is perm[r] for a seeded random permutation perm, so the
      hub columns (the long rows of A^T) are scattered.
    - A column drawn twice in one row is kept once, so the stored count is
      a little below ``nnz``; columns are sorted within each row; values are
      U(0, 1).

    Drawn with torch's seeded generator on ``device`` (the same seed gives
    the same matrix on one device type). Returns (rowptr int64 (m+1),
    colidx int32, vals float32) as tensors on ``device``."""
    import torch

    dev = torch.device(device)
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    u = 1.0 - torch.rand(m, generator=g, device=dev, dtype=torch.float64)      # (0, 1]
    w = u.pow(-1.0 / (row_tail - 1.0))
    want = w * (float(nnz) / float(w.sum()))
    lengths = torch.floor(want + torch.rand(m, generator=g, device=dev, dtype=torch.float64))
    lengths = lengths.clamp_(0, n).to(torch.int64)
    total = int(lengths.sum())
    rows = torch.repeat_interleave(torch.arange(m, device=dev, dtype=torch.int64), lengths)
    v = torch.rand(total, generator=g, device=dev, dtype=torch.float64)
    a = 1.0 - col_skew
    span = float(n + 1) ** a - 1.0
    rank = torch.floor((1.0 + v * span).pow(1.0 / a) - 1.0).clamp_(0, n - 1).to(torch.int64)
    del v
    perm = torch.randperm(n, generator=g, device=dev)
    key = rows * n + perm[rank]
    del rows, rank, perm
    key = torch.unique(key, sorted=True)            # sorted by (row, column), duplicates gone
    r = torch.div(key, n, rounding_mode="floor")
    colidx = (key - r * n).to(torch.int32)
    counts = torch.bincount(r, minlength=m)
    del key, r
    rowptr = torch.zeros(m + 1, dtype=torch.int64, device=dev)
    torch.cumsum(counts, 0, out=rowptr[1:])
    vals = torch.rand(colidx.numel(), generator=g, device=dev, dtype=torch.float32)
    return rowptr, colidx, vals


def csr_from_dense(D: np.ndarray, dtype=None) -> CSR:
    """CSR view of a small dense array (zeros dropped)."""
    D = np.asarray(D)
    m, n = D.shape
    rows, cols = np.nonzero(D)
    counts = np.bincount(rows, minlength=m).astype(np.int64)
    rowptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    vals = D[rows, cols].astype(dtype or D.dtype)
    return CSR(m, n, rowptr, cols.astype(np.int32), vals)


def spd_gram(k: int, rows: int, seed: int, dtype=np.float64):
    """A k x k Gram matrix X^T X of a rows x k U(0,1) matrix (positive
    definite for rows >= k almost surely), plus X itself."""
    X = uniform((rows, k), seed)
    return (X.T @ X).astype(dtype), X


def planted_nnls(rows: int, k: int, seed: int, gram_cols: int = 0):
    """Nonnegative least-squares instances with a known answer.

    G = B B^T for a k x gram_cols U(0,1) matrix B (default 4k columns),
    rounded to float32 values so both storage types hold it exactly. Row r
    gets a support F_r whose size is drawn uniformly from 0..k (so every
    size, the empty and the full set included, occurs), values xs on F_r and
    slacks ys off F_r both U(0.5, 1.5) x the size of G's entries, and
    right-hand side p_r = G xs_r - ys_r (float64). Then xs_r >= 0, ys_r >= 0,
    xs_r * ys_r = 0 and G xs_r - p_r = ys_r: the optimality conditions of
    min_{x >= 0} 1/2 x^T G x - p_r^T x hold at xs_r, which is therefore the
    unique solution (G is positive definite almost surely).

    Returns (G, P, XS), P and XS of shape rows x k."""
    rng = _rng(seed)
    c = gram_cols or 4 * k
    B = rng.random((k, c))
    G = (B @ B.T).astype(np.float32).astype(np.float64)
    scale = float(np.abs(G).max())
    sizes = rng.integers(0, k + 1, size=rows)
    if rows >= 2:
        sizes[0], sizes[1] = 0, k
    XS = np.zeros((rows, k))
    YS = np.zeros((rows, k))
    for r in range(rows):
        sup = rng.permutation(k)[: sizes[r]]
        on = np.zeros(k, dtype=bool)
        on[sup] = True
        XS[r, on] = rng.uniform(0.5, 1.5, size=int(on.sum()))
        YS[r, ~on] = rng.uniform(0.5, 1.5, size=int((~on).sum())) * scale
    P = XS @ G - YS
    return G, P, XS


# Workloads of the benchmark and parity suite, named by shape. Each entry:
# (kind, m, n, k, algorithm, iterations, dtype, extra)
WORKLOADS = {
    "dense-2000x1000-k10-mu-f64": dict(kind="dense", m=2000, n=1000, k=10, k_true=10,
                                       algo="mu", iters=20, dtype="f64"),
    "dense-65536x65536-k50-hals-f32": dict(kind="dense", m=65536, n=65536, k=50, k_true=50,
                                           algo="hals", iters=30, dtype="f32"),
    "csr-1048576x1048576-d1e-4-k50-abpp-f32": dict(kind="csr", m=1 << 20, n=1 << 20, k=50,
                                                   density=1e-4, algo="abpp", iters=20,
                                                   dtype="f32"),
}
