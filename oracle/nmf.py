"""FP64 reference NMF: the Gram and large products, the MU / HALS / ABPP
updates and the relative error, following Algorithm 1 step by step.

Test infrastructure only; see the package docstring.

Shapes follow the paper's notation (Section 1 and Table 2): A is m x n,
W is m x k, H is k x n. A may be a dense ndarray or a scipy.sparse matrix.
"""
from __future__ import annotations

import numpy as np

from .bpp import bpp_nnls

# Section 4.1 gives MU without a rule for a zero denominator. The oracle adds
# this constant to every denominator (reading taken for the whole build);
# for positive data the denominators are many orders larger.
MU_EPS = 1e-16


def _f64(X):
    return np.asarray(X, dtype=np.float64)


def _is_sparse(A) -> bool:
    return hasattr(A, "tocsr") and not isinstance(A, np.ndarray)


# --- bfloat16 rounding of a product operand --------------------------------

def round_bf16(X):
    """Values of X rounded to bfloat16 (8 significant bits, float32's
    exponent range), round to nearest with ties to even, returned as float64.

    Written from the format's definition: a float32 whose low 16 bits are
    dropped keeps its sign, exponent and 7 stored fraction bits, so rounding
    adds half a unit of the kept last place (0x8000 in the low half), minus
    one when the kept last bit is 0 so that exact ties go to the even
    neighbour, and then clears the low half. Values are first rounded to
    float32, the type the GPU factors are stored in. NaN is not expected."""
    x32 = np.ascontiguousarray(np.asarray(X, dtype=np.float64).astype(np.float32))
    u = x32.view(np.uint32).astype(np.uint64)
    keep_lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = (u + np.uint64(0x7FFF) + keep_lsb) & np.uint64(0xFFFF0000)
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


# --- FP8 (E4M3) rounding of a product operand -----------------------------

FP8_E4M3_MAX = 448.0


def round_fp8_e4m3(X):
    """Values of X rounded to FP8 E4M3, round to nearest with ties to even,
    saturating at the largest finite value 448; returned as float64.

    E4M3 has a sign, 4 exponent bits (bias 7) and 3 fraction bits: for
    2^e <= |x| < 2^(e+1) with -6 <= e <= 8 the representable values are the
    multiples of 2^(e-3), and below 2^-6 (the subnormals) the multiples of
    2^-9. Rounding is therefore: find the binade, divide by its spacing,
    round to the nearest integer with ties to even (np.rint), multiply
    back; all of it exact in float64. A result past 448 is clamped to 448.
    Values are first rounded to float32, the type the GPU factors are
    stored in. NaN is not expected."""
    x = np.asarray(X, dtype=np.float64).astype(np.float32).astype(np.float64)
    a = np.abs(x)
    _, E = np.frexp(a)                 # a = f 2^E with f in [0.5, 1)
    e = np.maximum(E - 1, -6)          # binade exponent, subnormals share -6
    spacing = np.ldexp(1.0, e - 3)
    r = np.minimum(np.rint(a / spacing) * spacing, FP8_E4M3_MAX)
    return np.copysign(r, x)


def fp8_column_scales(X, rank_axis: int):
    """Per rank index j (along ``rank_axis`` of X), the scale s_j = 2^p of
    the FP8 product operand: the smallest power of two with
    max |X_j| <= 448 s_j, and 1 when X_j is all zero. Taken on the float32
    values of X."""
    x = np.abs(np.asarray(X, dtype=np.float64).astype(np.float32).astype(np.float64))
    other = 1 - rank_axis
    mx = x.max(axis=other) if x.shape[other] else np.zeros(x.shape[rank_axis])
    s = np.ones(len(mx))
    for j, v in enumerate(mx):
        if v == 0.0:
            continue
        p = int(np.floor(np.log2(v / FP8_E4M3_MAX)))
        while FP8_E4M3_MAX * 2.0 ** p < v:          # not yet large enough
            p += 1
        while FP8_E4M3_MAX * 2.0 ** (p - 1) >= v:   # a smaller power still fits
            p -= 1
        s[j] = 2.0 ** p
    return s


def round_fp8_scaled(X, rank_axis: int):
    """The FP8 product operand as values: each rank slice X_j divided by its
    scale s_j (fp8_column_scales), rounded to E4M3, multiplied back by s_j.
    Since s_j is a power of two, a product with this operand equals the
    product of the E4M3 codes with the output column multiplied by s_j."""
    s = fp8_column_scales(X, rank_axis)
    shape = [1, 1]
    shape[rank_axis] = -1
    s = s.reshape(shape)
    x32 = np.asarray(X, dtype=np.float64).astype(np.float32).astype(np.float64)
    return round_fp8_e4m3(x32 / s) * s


# --- the four products of Algorithm 1 ------------------------------------

def gram_fixed_H(H):
    """H H^T (k x k), used by the W update (Algorithm 1, W step)."""
    H = _f64(H)
    return H @ H.T


def gram_fixed_W(W):
    """W^T W (k x k), used by the H update (Algorithm 1, H step)."""
    W = _f64(W)
    return W.T @ W


def product_AHt(A, H):
    """A H^T (m x k)."""
    H = _f64(H)
    if _is_sparse(A):
        return np.asarray(A.tocsr().astype(np.float64) @ H.T)
    return _f64(A) @ H.T


def product_WtA(A, W):
    """W^T A (k x n)."""
    W = _f64(W)
    if _is_sparse(A):
        return np.asarray(A.tocsc().astype(np.float64).T @ W).T
    return W.T @ _f64(A)


# --- Section 4.1: multiplicative update, Eq. (3) -------------------------

def mu_update_W(W, Q, P, eps=MU_EPS):
    """w_ij <- w_ij (A H^T)_ij / (W H H^T)_ij, all entries at once.

    Q = H H^T, P = A H^T. ``eps`` is added to the denominator.
    """
    W = _f64(W)
    return W * _f64(P) / (W @ _f64(Q) + eps)


def mu_update_H(H, S, R, eps=MU_EPS):
    """h_ij <- h_ij (W^T A)_ij / (W^T W H)_ij.  S = W^T W, R = W^T A (k x n)."""
    H = _f64(H)
    return H * _f64(R) / (_f64(S) @ H + eps)


# --- Section 4.2: HALS, Eqs. (4)-(5) -------------------------------------

def hals_update_W(W, H, Q, P, on_column=None):
    """One HALS sweep over the columns of W, then the column normalisation.

    Eq. (5) updates w^i for i = 1..k in order, each time with the newest
    values of the other columns (Section 4.2 says the columns are updated in
    order so that the most up-to-date values are used), and normalises w^i.

    Readings taken (the printed rule omits the divisor and leaves H alone):
    HALS is the 2k-block coordinate descent of Eq. (4), so the exact
    minimiser of ||A - sum_j w^j h_j||_F over w^i >= 0 with everything else
    fixed is used,

        w^i <- max(0, w^i + ((A H^T)^i - W (H H^T)^i) / (H H^T)_ii),

    skipped when (H H^T)_ii = 0; and the normalisation w^i <- w^i / s_i,
    s_i = ||w^i||_2 > 0, is compensated by h_i <- s_i h_i so that W H is
    unchanged. After rescaling row i of H, Q and P are rescaled to match
    (Q_i. and Q_.i by s_i, P^i by s_i), which is what recomputing them from
    the new H would give.

    Returns (W_new, H_rescaled). ``on_column(i, W, H)``, if given, is called
    right after column i is updated and before it is normalised.
    """
    W = _f64(W).copy()
    H = _f64(H).copy()
    Q = _f64(Q).copy()
    P = _f64(P).copy()
    k = W.shape[1]
    for i in range(k):
        if Q[i, i] > 0:
            W[:, i] = np.maximum(0.0, W[:, i] + (P[:, i] - W @ Q[:, i]) / Q[i, i])
        if on_column is not None:
            on_column(i, W.copy(), H.copy())
        s = np.linalg.norm(W[:, i])
        if s > 0:
            W[:, i] /= s
            H[i, :] *= s
            Q[i, :] *= s
            Q[:, i] *= s
            P[:, i] *= s
    return W, H


def hals_update_H(H, S, R, on_row=None):
    """One HALS sweep over the rows of H (Eq. (5), third rule).

        h_i <- max(0, h_i + ((W^T A)_i - (W^T W)_i H) / (W^T W)_ii),

    for i = 1..k in order with the newest rows, skipped when S_ii = 0. After
    the W normalisation S_ii = 1 for every nonzero column, so the division
    only matters for robustness; the paper prints the rule without it.
    """
    H = _f64(H).copy()
    S = _f64(S)
    R = _f64(R)
    k = H.shape[0]
    for i in range(k):
        if S[i, i] > 0:
            H[i, :] = np.maximum(0.0, H[i, :] + (R[i, :] - S[i, :] @ H) / S[i, i])
        if on_row is not None:
            on_row(i, H.copy())
    return H


# --- Section 4.3: ANLS with BPP ------------------------------------------

def abpp_update_W(Q, P, max_pivots=None):
    """W <- argmin_{W>=0} ||A - W H||_F, row by row (Eq. (2), first line).

    Row r of W solves min_{x>=0} 1/2 x^T Q x - p_r^T x with Q = H H^T and
    p_r the r-th row of P = A H^T, i.e. SolveBPP(H H^T, H A^T)^T.
    """
    return bpp_nnls(Q, _f64(P).T, max_pivots=max_pivots).T


def abpp_update_H(S, R, max_pivots=None):
    """H <- argmin_{H>=0} ||A - W H||_F column by column: SolveBPP(W^T W, W^T A)."""
    return bpp_nnls(S, R, max_pivots=max_pivots)


# --- Section 6.2: relative error -----------------------------------------

def objective_sq(A, W, H, row_block: int = 2048) -> float:
    """||A - W H||_F^2 evaluated directly.

    Dense A: the residual is formed explicitly, a row block at a time.
    Sparse A: sum over stored entries of (a_ij - (WH)_ij)^2 - (WH)_ij^2, plus
    ||W H||_F^2 = <W^T W, H H^T>; the stored-entry part is the residual at
    those entries and the rest accounts for the zeros, so the value is
    ||A - W H||_F^2 exactly (up to rounding).
    """
    W = _f64(W)
    H = _f64(H)
    if _is_sparse(A):
        C = A.tocoo()
        total = float(np.sum(gram_fixed_W(W) * gram_fixed_H(H)))
        rows = C.row.astype(np.int64)
        cols = C.col.astype(np.int64)
        vals = C.data.astype(np.float64)
        step = 1 << 20
        for s in range(0, vals.size, step):
            r, c, v = rows[s:s + step], cols[s:s + step], vals[s:s + step]
            wh = np.einsum("ij,ji->i", W[r], H[:, c])
            total += float(np.sum((v - wh) ** 2 - wh ** 2))
        return total
    total = 0.0
    m = W.shape[0]
    for r0 in range(0, m, row_block):
        r1 = min(m, r0 + row_block)
        D = _f64(A[r0:r1]) - W[r0:r1] @ H
        total += float(np.sum(D * D))
    return total


def _norm_sq(A) -> float:
    if _is_sparse(A):
        d = A.tocoo().data.astype(np.float64)
        return float(np.sum(d * d))
    total = 0.0
    for r0 in range(0, A.shape[0], 4096):
        blk = _f64(A[r0:r0 + 4096])
        total += float(np.sum(blk * blk))
    return total


def relative_error(A, W, H, normA_sq: float | None = None) -> float:
    """||A - W H||_F / ||A||_F (Section 6.2)."""
    if normA_sq is None:
        normA_sq = _norm_sq(A)
    return float(np.sqrt(max(objective_sq(A, W, H), 0.0) / normA_sq))


# --- stationarity: the projected gradient (Section 6.2) --------------------
#
# Section 6.2 names the projected gradient, beside the relative error, as a
# measure of the factors' quality and as a stopping test, without a formula;
# the definition below is the usual one for bound-constrained problems (Lin's,
# also used by the NMF survey the paper cites there). For
# f(W, H) = 1/2 ||A - W H||_F^2:
#     grad_W f = W (H H^T) - A H^T,      grad_H f = (W^T W) H - W^T A,
# and the projection onto the feasible directions at x >= 0 keeps a gradient
# entry where x > 0 and only its negative part where x = 0. The norm is zero
# exactly at the stationary points of the constrained problem (the KKT
# conditions of Section 4.3, Eq. (7), for both factors at once).

def gradients(A, W, H):
    """(grad_W, grad_H) of 1/2 ||A - W H||_F^2."""
    W = _f64(W)
    H = _f64(H)
    gW = W @ gram_fixed_H(H) - product_AHt(A, H)
    gH = gram_fixed_W(W) @ H - product_WtA(A, W)
    return gW, gH


def projected_gradient_sq(X, G) -> float:
    """Sum of squares of the projected gradient G at X >= 0."""
    X = _f64(X)
    G = _f64(G)
    P = np.where(X > 0, G, np.minimum(G, 0.0))
    return float(np.sum(P * P))


def projected_gradient_norm(A, W, H) -> float:
    """||(proj grad_W f, proj grad_H f)||_F at (W, H)."""
    gW, gH = gradients(A, W, H)
    return float(np.sqrt(projected_gradient_sq(W, gW) + projected_gradient_sq(H, gH)))


# --- Algorithm 1 ---------------------------------------------------------

def run(A, k: int, algo: str, iters: int, W0, H0, eps: float = MU_EPS,
        max_pivots=None, track_error: bool = True, bf16_products: bool = False,
        fp8_products: bool = False):
    """AU-NMF (Algorithm 1) for ``iters`` iterations from (W0, H0).

    One iteration: Q = H H^T, P = A H^T, update W; S = W^T W, R = W^T A,
    update H. ABPP does not read W0 (its W update is an exact solve). Returns
    (W, H, rel_err) with rel_err[t] the relative error after t iterations
    (rel_err[0] at the initial factors), or an empty list when
    ``track_error`` is False.

    bf16_products: the reduced-precision variant of the two large products
    (A stored in bfloat16 is passed in as its float64 values): the factor
    operand of A H^T and W^T A is rounded to bfloat16 first (round_bf16);
    the products are then exact in float64, and the Grams, updates and the
    error use the unrounded factors as before.

    fp8_products: the same with A stored in FP8 E4M3 and the factor operand
    scaled per rank index and rounded to E4M3 (round_fp8_scaled).
    """
    if bf16_products and fp8_products:
        raise ValueError("choose one reduced-precision product variant")
    if bf16_products:
        frH = frW = round_bf16
    elif fp8_products:
        frH = lambda X: round_fp8_scaled(X, 0)   # H is k x n: rank along rows
        frW = lambda X: round_fp8_scaled(X, 1)   # W is m x k: rank along columns
    else:
        frH = frW = lambda X: X
    algo = algo.lower()
    if algo not in ("mu", "hals", "abpp"):
        raise ValueError("unknown algorithm %r" % algo)
    W = _f64(W0).copy()
    H = _f64(H0).copy()
    assert W.shape[1] == k and H.shape[0] == k
    errs = []
    normA_sq = _norm_sq(A) if track_error else None
    if track_error:
        errs.append(relative_error(A, W, H, normA_sq))
    for _ in range(iters):
        Q = gram_fixed_H(H)
        P = product_AHt(A, frH(H))
        if algo == "mu":
            W = mu_update_W(W, Q, P, eps)
        elif algo == "hals":
            W, H = hals_update_W(W, H, Q, P)
        else:
            W = abpp_update_W(Q, P, max_pivots)
        S = gram_fixed_W(W)
        R = product_WtA(A, frW(W))
        if algo == "mu":
            H = mu_update_H(H, S, R, eps)
        elif algo == "hals":
            H = hals_update_H(H, S, R)
        else:
            H = abpp_update_H(S, R, max_pivots)
        if track_error:
            errs.append(relative_error(A, W, H, normA_sq))
    return W, H, errs


def run_until(A, k: int, algo: str, max_iters: int, W0, H0, stop: str, tol: float,
              eps: float = MU_EPS, max_pivots=None):
    """Algorithm 1 with a stopping criterion (Section 6.2: the iteration
    count together with a tolerance on a quality metric). After iteration t
    it stops when
      stop == "pgrad":  ||proj grad f(W_t, H_t)|| <= tol ||proj grad f(W_0, H_0)||
      stop == "relerr": e_{t-1} - e_t < tol e_{t-1}  (relative error improvement)
    or when t == max_iters. Returns (W, H, rel_err[0..t], pg_ratio[0..t], t)."""
    if stop not in ("pgrad", "relerr"):
        raise ValueError("unknown stopping metric %r" % stop)
    W = _f64(W0).copy()
    H = _f64(H0).copy()
    normA_sq = _norm_sq(A)
    errs = [relative_error(A, W, H, normA_sq)]
    pg0 = projected_gradient_norm(A, W, H)
    ratios = [1.0]
    t = 0
    while t < max_iters:
        W, H, _ = run(A, k, algo, 1, W, H, eps, max_pivots, track_error=False)
        t += 1
        errs.append(relative_error(A, W, H, normA_sq))
        ratios.append(projected_gradient_norm(A, W, H) / pg0)
        if stop == "pgrad" and ratios[-1] <= tol:
            break
        if stop == "relerr" and errs[-2] - errs[-1] < tol * errs[-2]:
            break
    return W, H, errs, ratios, t
