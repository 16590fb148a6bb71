"""Pins for the oracle's block principal pivoting NNLS (Section 4.3).

Each check is independent of the oracle's own code: hand-solved fixtures,
exhaustive enumeration of passive sets, the KKT conditions of Eq. (7) and
SciPy's Lawson-Hanson NNLS.
"""
import itertools

import numpy as np
import pytest
import scipy.optimize

import oracle
from synth import uniform


def _random_problem(k, c, seed, cond_boost=0.0):
    rng = np.random.default_rng(seed)
    C = rng.standard_normal((k + 3, k))
    if cond_boost:
        C[:, 0] = C[:, 1] + cond_boost * C[:, 0]
    G = C.T @ C
    R = rng.standard_normal((k, c)) * 2.0
    return G, R


def _kkt_violation(G, R, X):
    Y = G @ X - R
    scale = np.abs(G).max() * np.abs(X).max() + np.abs(R).max() + 1.0
    return max(float(-X.min()), float(-Y.min()), float(np.abs(X * Y).max()) / scale) / scale


def test_hand_solved_instances(golden):
    for name, G, r, x, y in golden("nnls_hand.txt"):
        r = r[0]
        got = oracle.bpp_nnls(G, r)
        np.testing.assert_allclose(got, x[0], rtol=0, atol=1e-14, err_msg=name)
        np.testing.assert_allclose(G @ got - r, y[0], rtol=0, atol=1e-14, err_msg=name)


@pytest.mark.parametrize("k", [1, 2, 3, 5, 8])
def test_brute_force_enumeration(k):
    """Exactly one passive set satisfies Eq. (7) for positive-definite G."""
    G, R = _random_problem(k, 40, seed=100 + k)
    X = oracle.bpp_nnls(G, R)
    for b in range(R.shape[1]):
        r = R[:, b]
        hits = []
        for bits in itertools.product([False, True], repeat=k):
            F = np.array(bits)
            x = np.zeros(k)
            if F.any():
                x[F] = np.linalg.solve(G[np.ix_(F, F)], r[F])
            y = G @ x - r
            if np.all(x[F] >= -1e-12) and np.all(y[~F] >= -1e-12):
                hits.append(x)
        assert len(hits) == 1, (k, b, len(hits))
        np.testing.assert_allclose(X[:, b], hits[0], rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("k,c", [(10, 200), (50, 300), (64, 100)])
def test_kkt_conditions(k, c):
    G, R = _random_problem(k, c, seed=7 * k)
    X = oracle.bpp_nnls(G, R)
    assert _kkt_violation(G, R, X) < 1e-12


def test_ill_conditioned_kkt():
    G, R = _random_problem(20, 200, seed=3, cond_boost=1e-3)
    X = oracle.bpp_nnls(G, R)
    assert _kkt_violation(G, R, X) < 1e-10


@pytest.mark.parametrize("k", [4, 16, 50])
def test_matches_scipy_lawson_hanson(k):
    """G = L L^T turns Eq. (6) into min ||L^T x - L^{-1} r||, which SciPy solves."""
    G, R = _random_problem(k, 30, seed=11 * k)
    L = np.linalg.cholesky(G)
    X = oracle.bpp_nnls(G, R)
    for b in range(R.shape[1]):
        rhs = np.linalg.solve(L, R[:, b])
        ref, _ = scipy.optimize.nnls(L.T, rhs, maxiter=50 * k)
        np.testing.assert_allclose(X[:, b], ref, rtol=1e-8, atol=1e-10)


def test_nmf_shaped_problems():
    """Gram of a U(0,1) factor and right-hand sides of nonnegative data."""
    k = 50
    H = uniform((k, 3000), seed=5)
    A = uniform((200, 3000), seed=6)
    G = H @ H.T
    R = H @ A.T
    X = oracle.bpp_nnls(G, R)
    assert _kkt_violation(G, R, X) < 1e-12
    assert (X == 0).any() and (X > 0).any()


def test_lockstep_equals_one_column_at_a_time():
    G, R = _random_problem(12, 60, seed=21)
    X = oracle.bpp_nnls(G, R)
    for b in range(R.shape[1]):
        np.testing.assert_array_equal(oracle.bpp_nnls(G, R[:, b]), X[:, b])


def test_degenerate_gram_zero_row():
    """A zero row of the fixed factor: G_ii = 0, r_i = 0 -> x_i = 0 (tie-break)."""
    G, R = _random_problem(6, 50, seed=9)
    G[2, :] = 0.0
    G[:, 2] = 0.0
    R[2, :] = 0.0
    X = oracle.bpp_nnls(G, R)
    assert np.all(X[2] == 0.0)
    assert _kkt_violation(G, R, X) < 1e-12


def test_pivot_cap_raises():
    """x = 0 is infeasible when some r_i > 0, so zero allowed pivots must fail."""
    G, R = _random_problem(8, 10, seed=1)
    with pytest.raises(RuntimeError):
        oracle.bpp_nnls(G, np.abs(R) + 0.1, max_pivots=0)


@pytest.mark.parametrize("k", [1, 7, 33, 50])
def test_planted_kkt_solutions_recovered(k):
    """Instances built to satisfy the optimality conditions at a chosen point
    (every support size from empty to full): the oracle must return that
    point, which no property of the oracle itself decides."""
    from synth import planted_nnls

    G, P, XS = planted_nnls(120, k, seed=300 + k)
    X = oracle.abpp_update_W(G, P)
    assert np.max(np.abs(X - XS)) <= 1e-9 * np.abs(XS).max()
