"""A float32 model of Algorithm 1 for sizing FP32 parity bars (test
infrastructure, CPU only).

The GPU path stores A, W, H, the two large products and the two Grams in
float32 and accumulates the products in float32; the updates themselves
(the BPP solves in particular) run on those float32 values. This module
replays that precision on the CPU around the oracle's own update rules: the
products and Grams are sums over K accumulated one term at a time in
float32 (each product and each partial sum rounded, the textbook model of a
float32 dot product) in a seeded order of the K terms, the factors are
rounded to float32 after every update, and everything else is the oracle's
FP64 arithmetic. Different orders of the K terms give different, equally
valid float32 results; the spread of the relative-error trajectory across
them against the plain FP64 oracle is how far float32 arithmetic alone moves
that trajectory on a given case. A bar looser than 1e-5 must sit above that
spread, and is set as a small multiple of it."""
from __future__ import annotations

import numpy as np

import oracle


def _f32(X):
    return np.asarray(X, dtype=np.float32)


def seq_f32_matmul(X, Y, order=None):
    """X (a x K) @ Y (K x b) summed over K one term at a time in float32, in
    the order `order` (a permutation of range(K); None = natural order)."""
    X = _f32(X)
    Y = _f32(Y)
    K = X.shape[1]
    acc = np.zeros((X.shape[0], Y.shape[1]), dtype=np.float32)
    for l in (range(K) if order is None else order):
        acc += np.multiply.outer(X[:, l], Y[l])
    return acc.astype(np.float64)


def run_fp32(A, k, algo, iters, W0, H0, seed=None, round_operand=None):
    """Algorithm 1 from (W0, H0) with the float32 model above. seed picks the
    order of the K terms of every sum (None: natural order). round_operand,
    if given, is applied to the factor operand of the two large products
    (the reduced-precision product variants). Returns the relative error
    after every iteration, evaluated in FP64 as the oracle does."""
    rng = None if seed is None else np.random.default_rng(seed)
    fr = round_operand or (lambda X: X)
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape

    def order(K):
        return None if rng is None else rng.permutation(K)

    def r(X):
        return _f32(X).astype(np.float64)

    W = r(W0)
    H = r(H0)
    normA_sq = float(np.sum(A * A))
    errs = [oracle.relative_error(A, W, H, normA_sq)]
    for _ in range(iters):
        Q = seq_f32_matmul(H, H.T, order(n))
        P = seq_f32_matmul(A, fr(H).T, order(n))
        if algo == "mu":
            W = r(oracle.mu_update_W(W, Q, P))
        elif algo == "hals":
            W, H = oracle.hals_update_W(W, H, Q, P)
            W, H = r(W), r(H)
        else:
            W = r(oracle.abpp_update_W(Q, P))
        S = seq_f32_matmul(W.T, W, order(m))
        R = seq_f32_matmul(fr(W).T, A, order(m))
        if algo == "mu":
            H = r(oracle.mu_update_H(H, S, R))
        elif algo == "hals":
            H = r(oracle.hals_update_H(H, S, R))
        else:
            H = r(oracle.abpp_update_H(S, R))
        errs.append(oracle.relative_error(A, W, H, normA_sq))
    return np.array(errs)


def trajectory_spread(A, k, algo, iters, W0, H0, seeds=(None, 1, 2, 3), round_operand=None,
                      reference=None):
    """Largest relative difference per realization between the float32
    model's trajectory and the FP64 oracle's (reference, or oracle.run on the
    same float32-valued inputs), one entry per seed."""
    if reference is None:
        kw = {}
        if round_operand is oracle.round_bf16:
            kw["bf16_products"] = True
        _, _, reference = oracle.run(A, k, algo, iters, np.asarray(W0, np.float64),
                                     np.asarray(H0, np.float64), **kw)
    ref = np.asarray(reference, dtype=np.float64)
    out = []
    for s in seeds:
        e = run_fp32(A, k, algo, iters, W0, H0, seed=s, round_operand=round_operand)
        out.append(float(np.max(np.abs(e - ref) / ref)))
    return out
