"""Nonnegative least squares by block principal pivoting (oracle, FP64).

Test infrastructure only; see the package docstring.

Section 4.3 defines SolveBPP(C^T C, C^T B): for every column b of B solve
Eq. (6), min_{x >= 0} ||C x - b||_2, whose optimality conditions are the
KKT system of Eq. (7):

    y = C^T C x - C^T b,   y >= 0,   x >= 0,   x_i y_i = 0 for all i.

Only the normal-equation data G = C^T C and r = C^T b enter (Section 4.3
solves the passive-set least squares through the normal equations), so the
problem is written here as min_{x>=0} 1/2 x^T G x - r^T x with y = G x - r.

The paper describes BPP in words (greedy exchange of indices between the
active and passive sets until the KKT conditions hold) and defers the
details to Kim and Park's method, which it cites. The exchange rule used
here is that method's: a full exchange of every infeasible index while the
number of infeasible indices keeps falling, at most three full exchanges
without progress, then a single exchange of the largest infeasible index
(which guarantees termination). Passive-set systems G_FF x_F = r_F are
solved directly (dense LU through ``numpy.linalg.solve``) on the matrix
G_FF padded with the identity outside F, so that x is zero off F.

Degenerate Gram matrices: an index i whose row of G and whose r_i are zero
(a zero row of the fixed factor) has y_i = 0 at x_i = 0, which is feasible,
so the strict "< 0" tests never move it into the passive set and x_i stays 0.
"""
from __future__ import annotations

import numpy as np


def passive_solve(G: np.ndarray, R: np.ndarray, F: np.ndarray):
    """Solve the passive-set systems for a batch of right-hand sides.

    G: (k, k); R: (k, c) right-hand sides r; F: (k, c) bool passive sets.
    Returns (X, Y) with X_F = G_FF^{-1} r_F, X off F = 0, Y = G X - R and
    Y on F set to exactly 0 (Eq. (7) with x_F solved exactly).
    """
    G = np.asarray(G, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    k, c = R.shape
    Fm = F.T.astype(np.float64)                       # (c, k)
    # M_b = D_b G D_b + (I - D_b),  D_b = diag(F[:, b])
    M = G[None, :, :] * Fm[:, :, None] * Fm[:, None, :]
    M[:, np.arange(k), np.arange(k)] += 1.0 - Fm
    rhs = (R.T * Fm)[:, :, None]
    X = np.linalg.solve(M, rhs)[:, :, 0].T            # (k, c)
    X[~F] = 0.0
    Y = G @ X - R
    Y[F] = 0.0
    return X, Y


def bpp_nnls(G: np.ndarray, R: np.ndarray, max_pivots: int | None = None,
             return_steps: bool = False):
    """Columns x of X solve min_{x>=0} 1/2 x^T G x - r^T x, one per column r of R.

    All right-hand sides advance through the same pivoting state machine in
    lock step; each column's sequence of passive sets is exactly that of the
    single-column method. Raises RuntimeError if some column has not reached
    a KKT point within ``max_pivots`` passive-set solves (default 50 k).
    """
    G = np.asarray(G, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    squeeze = R.ndim == 1
    if squeeze:
        R = R[:, None]
    k, c = R.shape
    if max_pivots is None:
        max_pivots = 50 * k
    X = np.zeros((k, c))
    Y = -R.copy()                                     # y = G*0 - r
    F = np.zeros((k, c), dtype=bool)                  # passive sets, start empty
    budget = np.full(c, 3, dtype=np.int64)            # full exchanges left without progress
    best = np.full(c, k + 1, dtype=np.int64)          # fewest infeasible indices seen
    steps = np.zeros(c, dtype=np.int64)
    todo = np.arange(c)
    for _ in range(max_pivots + 1):
        Fs, Xs, Ys = F[:, todo], X[:, todo], Y[:, todo]
        V = (Fs & (Xs < 0)) | (~Fs & (Ys < 0))        # infeasible indices
        nv = V.sum(axis=0)
        alive = nv > 0
        todo, V, nv = todo[alive], V[:, alive], nv[alive]
        if todo.size == 0:
            break
        if np.any(steps[todo] >= max_pivots):
            raise RuntimeError("BPP did not reach a KKT point within %d pivots" % max_pivots)
        progress = nv < best[todo]
        best[todo[progress]] = nv[progress]
        budget[todo[progress]] = 3
        spend = ~progress & (budget[todo] >= 1)
        budget[todo[spend]] -= 1
        single = ~progress & ~spend
        flip = V.copy()
        if np.any(single):
            # backup rule: exchange only the largest infeasible index
            cols = np.nonzero(single)[0]
            last = k - 1 - np.argmax(V[::-1, cols], axis=0)
            flip[:, cols] = False
            flip[last, cols] = True
        F[:, todo] ^= flip
        X[:, todo], Y[:, todo] = passive_solve(G, R[:, todo], F[:, todo])
        steps[todo] += 1
    if squeeze:
        X = X[:, 0]
    if return_steps:
        return X, steps
    return X
