"""Pins for the oracle's MU, HALS and ABPP iterations and its objective.

Checks come from closed forms, theorems about the updates, special cases in
which two methods must coincide, brute force and library routines, so that a
dropped term, a wrong sign or index or a transposed operand fails one of them.
"""
import numpy as np
import pytest
import scipy.optimize
import scipy.sparse

import oracle
from synth import csr_from_dense, erdos_renyi_csr, init_factors, planted_dense, uniform


def _small(m=30, n=20, k=4, seed=3, noise=0.01):
    A = planted_dense(m, n, k, sigma=noise, seed=seed)
    W0, H0 = init_factors(m, n, k, seed=seed + 1)
    return A, W0, H0


# --- hand-worked fixtures --------------------------------------------------

def test_hand_worked_iterations(golden):
    for algo, A, W0, H0, W1, H1, e0, e1 in golden("updates_hand.txt"):
        W, H, errs = oracle.run(A, 1, algo, 1, W0, H0)
        np.testing.assert_allclose(W, W1, rtol=1e-14, atol=1e-14, err_msg=algo)
        np.testing.assert_allclose(H, H1, rtol=1e-14, atol=1e-14, err_msg=algo)
        np.testing.assert_allclose(errs, [e0[0, 0], e1[0, 0]], rtol=1e-13, atol=1e-7)


# --- products and objective -----------------------------------------------

def test_products_against_loops():
    """Brute-force sums for H H^T, A H^T, W^T W and W^T A on a tiny case."""
    rng = np.random.default_rng(0)
    A = rng.random((5, 4))
    W = rng.random((5, 3))
    H = rng.random((3, 4))
    Q = np.zeros((3, 3)); P = np.zeros((5, 3)); S = np.zeros((3, 3)); R = np.zeros((3, 4))
    for a in range(3):
        for b in range(3):
            Q[a, b] = sum(H[a, j] * H[b, j] for j in range(4))
            S[a, b] = sum(W[i, a] * W[i, b] for i in range(5))
    for i in range(5):
        for c in range(3):
            P[i, c] = sum(A[i, j] * H[c, j] for j in range(4))
    for c in range(3):
        for j in range(4):
            R[c, j] = sum(W[i, c] * A[i, j] for i in range(5))
    np.testing.assert_allclose(oracle.gram_fixed_H(H), Q, rtol=1e-14)
    np.testing.assert_allclose(oracle.product_AHt(A, H), P, rtol=1e-14)
    np.testing.assert_allclose(oracle.gram_fixed_W(W), S, rtol=1e-14)
    np.testing.assert_allclose(oracle.product_WtA(A, W), R, rtol=1e-14)
    As = scipy.sparse.csr_matrix(A)
    np.testing.assert_allclose(oracle.product_AHt(As, H), P, rtol=1e-14)
    np.testing.assert_allclose(oracle.product_WtA(As, W), R, rtol=1e-14)


def test_objective_direct_vs_trace_identity():
    """||A-WH||^2 = ||A||^2 - 2<W, A H^T> + <W^T W, H H^T> in FP64."""
    A, W, H = _small(40, 25, 5, seed=8, noise=0.5)
    direct = oracle.objective_sq(A, W, H)
    trace = (np.sum(A * A) - 2 * np.sum(W * (A @ H.T)) + np.sum((W.T @ W) * (H @ H.T)))
    assert abs(direct - trace) <= 1e-10 * np.sum(A * A)
    brute = sum((A[i, j] - W[i] @ H[:, j]) ** 2 for i in range(40) for j in range(25))
    assert abs(direct - brute) <= 1e-12 * brute


def test_sparse_objective_matches_dense():
    csr = erdos_renyi_csr(60, 45, 0.1, seed=4, dtype=np.float64)
    D = csr.to_dense()
    S = scipy.sparse.csr_matrix((csr.vals, csr.colidx, csr.rowptr), shape=(60, 45))
    W, H = init_factors(60, 45, 6, seed=2)
    assert abs(oracle.objective_sq(S, W, H) - oracle.objective_sq(D, W, H)) <= 1e-10 * oracle.objective_sq(D, W, H)


# --- MU (Section 4.1) -----------------------------------------------------

def test_mu_scalar_closed_form():
    """m = n = k = 1: w <- a/h, then h unchanged, so f_1 = 0."""
    a, w, h = 3.0, 0.7, 0.4
    W, H, errs = oracle.run(np.array([[a]]), 1, "mu", 1, np.array([[w]]), np.array([[h]]))
    assert W[0, 0] == pytest.approx(a / h, rel=1e-14)
    assert H[0, 0] == pytest.approx(h, rel=1e-14)
    assert errs[1] < 1e-14


def test_mu_exact_factorisation_is_fixed_point():
    W0 = uniform((12, 3), seed=1) + 0.1
    H0 = uniform((3, 9), seed=2) + 0.1
    A = W0 @ H0
    W, H, errs = oracle.run(A, 3, "mu", 5, W0, H0)
    np.testing.assert_allclose(W, W0, rtol=1e-12)
    np.testing.assert_allclose(H, H0, rtol=1e-12)


def test_mu_monotone():
    """Lee and Seung: the objective never increases under Eq. (3)."""
    A, W0, H0 = _small(50, 40, 6, seed=5, noise=0.3)
    _, _, errs = oracle.run(A, 6, "mu", 40, W0, H0)
    assert all(b <= a * (1 + 1e-12) for a, b in zip(errs, errs[1:]))
    assert errs[-1] < errs[0]


# --- HALS (Section 4.2) ---------------------------------------------------

def test_hals_monotone_after_every_column():
    A, W0, H0 = _small(40, 30, 5, seed=6, noise=0.2)
    H = H0.copy()
    W = W0.copy()
    vals = [oracle.objective_sq(A, W, H)]
    for _ in range(5):
        Q = oracle.gram_fixed_H(H)
        P = oracle.product_AHt(A, H)
        W, H = oracle.hals_update_W(W, H, Q, P,
                                    on_column=lambda i, Wc, Hc: vals.append(oracle.objective_sq(A, Wc, Hc)))
        vals.append(oracle.objective_sq(A, W, H))  # after normalisation: unchanged
        S = oracle.gram_fixed_W(W)
        R = oracle.product_WtA(A, W)
        H = oracle.hals_update_H(H, S, R, on_row=lambda i, Hc: vals.append(oracle.objective_sq(A, W, Hc)))
    assert all(b <= a * (1 + 1e-12) for a, b in zip(vals, vals[1:]))


def test_hals_each_column_is_a_block_minimiser():
    """Right after its update, column i satisfies the KKT conditions of
    min_{w^i >= 0} ||A - sum_j w^j h_j|| with the other columns as they are
    at that moment (Gauss-Seidel order)."""
    A, W0, H0 = _small(35, 28, 5, seed=12, noise=0.2)
    Q = oracle.gram_fixed_H(H0)
    P = oracle.product_AHt(A, H0)
    checked = []

    def check(i, Wc, Hc):
        g = Wc @ (Hc @ Hc.T)[:, i] - A @ Hc[i]  # gradient wrt column i (halved)
        pos = Wc[:, i] > 0
        assert np.all(np.abs(g[pos]) <= 1e-10 * np.abs(A @ Hc[i]).max())
        assert np.all(g[~pos] >= -1e-10 * np.abs(A @ Hc[i]).max())
        checked.append(i)

    oracle.hals_update_W(W0, H0, Q, P, on_column=check)
    assert checked == list(range(5))


def test_hals_normalisation():
    A, W0, H0 = _small(30, 20, 4, seed=13)
    W, H, _ = oracle.run(A, 4, "hals", 3, W0, H0)
    np.testing.assert_allclose(np.linalg.norm(W, axis=0), 1.0, rtol=1e-14)


def test_hals_equals_abpp_for_rank_one():
    """k = 1: each HALS block is the whole factor, so both are exact ANLS."""
    A, W0, H0 = _small(25, 18, 1, seed=14, noise=0.3)
    Wh, Hh, eh = oracle.run(A, 1, "hals", 6, W0, H0)
    Wa, Ha, ea = oracle.run(A, 1, "abpp", 6, W0, H0)
    np.testing.assert_allclose(Wh @ Hh, Wa @ Ha, rtol=1e-12)
    np.testing.assert_allclose(eh[1:], ea[1:], rtol=1e-12)


# --- ABPP (Section 4.3) ---------------------------------------------------

def test_abpp_rank_one_exact_in_one_iteration():
    rng = np.random.default_rng(4)
    u = rng.random(9) + 0.5
    v = rng.random(7) + 0.5
    A = np.outer(u, v)
    _, _, errs = oracle.run(A, 1, "abpp", 1, np.ones((9, 1)), rng.random((1, 7)) + 0.1)
    assert errs[1] < 1e-14


def test_abpp_half_step_solves_the_least_squares_problem():
    """Row r of the new W minimises ||H^T x - a_r|| over x >= 0 (Eq. (2))."""
    A, _, H0 = _small(15, 40, 6, seed=15, noise=0.5)
    W = oracle.abpp_update_W(oracle.gram_fixed_H(H0), oracle.product_AHt(A, H0))
    for r in range(A.shape[0]):
        ref, _ = scipy.optimize.nnls(H0.T, A[r], maxiter=500)
        np.testing.assert_allclose(W[r], ref, rtol=1e-8, atol=1e-10)
    Wf = uniform((15, 6), seed=3)
    H = oracle.abpp_update_H(oracle.gram_fixed_W(Wf), oracle.product_WtA(A, Wf))
    for c in range(A.shape[1]):
        ref, _ = scipy.optimize.nnls(Wf, A[:, c], maxiter=500)
        np.testing.assert_allclose(H[:, c], ref, rtol=1e-8, atol=1e-10)


def test_abpp_monotone():
    A, W0, H0 = _small(60, 40, 8, seed=16, noise=0.2)
    _, _, errs = oracle.run(A, 8, "abpp", 10, W0, H0)
    assert all(b <= a * (1 + 1e-12) for a, b in zip(errs[1:], errs[2:]))


# --- all three -------------------------------------------------------------

@pytest.mark.parametrize("algo,iters", [("abpp", 300), ("hals", 500)])
def test_planted_recovery(algo, iters):
    """Smoke test only (nonconvex, and U(0,1) factors converge slowly): an
    exact planted rank-3 matrix is approximated to 1e-3 from a fixed seed."""
    A = planted_dense(200, 150, 3, sigma=0.0, seed=40)
    W0, H0 = init_factors(200, 150, 3, seed=41)
    _, _, errs = oracle.run(A, 3, algo, iters, W0, H0)
    assert errs[-1] < 1e-3 and errs[-1] < 0.01 * errs[0]


def test_final_error_ordering_is_plausible():
    """Soft check in the spirit of Section 6.2: ABPP <= HALS <= MU * (1+tol)."""
    A, W0, H0 = _small(80, 60, 8, seed=19, noise=0.3)
    e = {a: oracle.run(A, 8, a, 30, W0, H0)[2][-1] for a in ("mu", "hals", "abpp")}
    assert e["abpp"] <= e["hals"] * 1.01 and e["hals"] <= e["mu"] * 1.01


@pytest.mark.parametrize("algo", ["mu", "hals", "abpp"])
def test_row_permutation(algo):
    """Permuting the rows of A (and of W0) permutes W and leaves H alone."""
    A, W0, H0 = _small(30, 22, 4, seed=20)
    perm = np.random.default_rng(1).permutation(30)
    W, H, e = oracle.run(A, 4, algo, 5, W0, H0)
    Wp, Hp, ep = oracle.run(A[perm], 4, algo, 5, W0[perm], H0)
    np.testing.assert_allclose(Wp, W[perm], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(Hp, H, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(ep, e, rtol=1e-10)


@pytest.mark.parametrize("algo", ["mu", "hals", "abpp"])
def test_sparse_input_same_as_dense(algo):
    csr = erdos_renyi_csr(50, 40, 0.2, seed=22, dtype=np.float64)
    D = csr.to_dense()
    S = scipy.sparse.csr_matrix((csr.vals, csr.colidx, csr.rowptr), shape=(50, 40))
    W0, H0 = init_factors(50, 40, 5, seed=23)
    Wd, Hd, ed = oracle.run(D, 5, algo, 4, W0, H0)
    Ws, Hs, es = oracle.run(S, 5, algo, 4, W0, H0)
    np.testing.assert_allclose(Ws, Wd, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(Hs, Hd, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(es, ed, rtol=1e-9)


def test_generators():
    csr = erdos_renyi_csr(300, 200, 0.05, seed=1)
    assert csr.rowptr[0] == 0 and csr.rowptr[-1] == csr.colidx.size
    for r in range(300):
        c = csr.colidx[csr.rowptr[r]:csr.rowptr[r + 1]]
        assert np.all(np.diff(c) > 0) and (c.size == 0 or (c[0] >= 0 and c[-1] < 200))
    assert abs(csr.nnz / (300 * 200) - 0.05) < 0.01
    assert np.all((csr.vals > 0) & (csr.vals < 1))
    D = csr.to_dense()
    back = csr_from_dense(D)
    np.testing.assert_array_equal(back.rowptr, csr.rowptr)
    A1 = planted_dense(20, 10, 3, seed=5)
    A2 = planted_dense(20, 10, 3, seed=5)
    np.testing.assert_array_equal(A1, A2)
    assert A1.min() >= 0
