"""Factors with more than 2^32 padded entries and CSR matrices with more than
2^26 rows: the sizes at which a one-dispatch grid over rows x KP entries, or
one wavefront per row, would pass the 32-bit work-item count of a dispatch.
The library caps those grids and strides over the rest; these runs check
every row.

A is 70,000,001 x 2^20 in CSR with one stored entry per row (seeded
columns, values U(0,1)), k = 40 (padded to KP = 64, so W holds 4.5e9 padded
entries and the SpMM runs one wavefront per row over 7e7 rows).
- iters = 0: W and H come back bit for bit (the padding copies and the H
  transposes over all rows), and e_0 matches the oracle's FP64 relative
  error of the same factors.
- one MU iteration: e_1 against the oracle's relative error of the GPU's own
  (W_1, H_1) at full size; sampled rows of W_1 against the oracle's MU step
  from (W_0, H_0) (row-local: Q = H_0 H_0^T and row r of A H_0^T); sampled
  columns of H_1 against the oracle's MU step from the GPU's W_1 (S = W_1^T W_1
  over all rows, R on the sampled columns).
- one HALS iteration from a scaled-down W_0 (so that no column is clipped to
  zero): every column of W_1 has unit norm over all rows (the normalisation
  scales (m + n) x KP entries)."""
import numpy as np
import pytest
import scipy.sparse

import oracle
import paper_1609_09154_amd as nmf
from synth import uniform
from tests.gpu_util import host, step

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

M, N, K = 70_000_001, 1 << 20, 40


@pytest.fixture(scope="module")
def case():
    import torch

    rng = np.random.default_rng(2024)
    ci = rng.integers(0, N, size=M, dtype=np.int64).astype(np.int32)
    cv = rng.random(M, dtype=np.float64).astype(np.float32)
    rp = np.arange(M + 1, dtype=np.int64)
    dev = torch.device("cuda:0")
    gen = torch.Generator(device=dev)
    gen.manual_seed(9154)
    W0 = torch.rand((M, K), generator=gen, device=dev, dtype=torch.float32)
    H0 = uniform((K, N), seed=9155).astype(np.float32)
    A = scipy.sparse.csr_matrix((cv.astype(np.float64), ci, rp), shape=(M, N))
    d = dict(rp=torch.from_numpy(rp).to(dev), ci=torch.from_numpy(ci).to(dev),
             cv=torch.from_numpy(cv).to(dev), W0=W0, H0=torch.from_numpy(H0).to(dev))
    assert M * 64 > 1 << 32 and M > 1 << 26
    return A, d


def test_round_trip_and_initial_error(case):
    import torch

    A, d = case
    W, H = d["W0"].clone(), d["H0"].clone()
    step("large rows: iters = 0 round trip, %d x %d, k = %d" % (M, N, K))
    errs, _ = nmf.nmf_csr(d["rp"], d["ci"], d["cv"], N, W, H, algo="mu", iters=0, objective=True)
    torch.cuda.synchronize()
    assert torch.equal(W, d["W0"]) and torch.equal(H, d["H0"])
    step("large rows: oracle e_0")
    e0 = oracle.relative_error(A, host(W), host(H))
    print("large rows e_0 gpu %.9f oracle %.9f" % (errs[0], e0))
    assert abs(errs[0] - e0) <= 1e-5 * e0


def test_mu_iteration_every_row(case):
    import torch

    A, d = case
    W, H = d["W0"].clone(), d["H0"].clone()
    step("large rows: one MU iteration")
    errs, _ = nmf.nmf_csr(d["rp"], d["ci"], d["cv"], N, W, H, algo="mu", iters=1, objective=True)
    torch.cuda.synchronize()
    W1, H1 = host(W), host(H)
    assert np.isfinite(W1).all() and (W1 >= 0).all() and (H1 >= 0).all()
    step("large rows: oracle e_1 of the GPU's factors")
    e1 = oracle.relative_error(A, W1, H1)
    print("large rows e_1 gpu %.9f oracle %.9f" % (errs[1], e1))
    assert abs(errs[1] - e1) <= 1e-5 * e1

    step("large rows: oracle MU step on sampled rows and columns")
    rng = np.random.default_rng(7)
    H0 = host(d["H0"]).astype(np.float64)
    Q = oracle.gram_fixed_H(H0)
    rows = np.sort(np.concatenate([rng.choice(M, 2000, replace=False), [0, M - 1]]))
    W0r = host(d["W0"][torch.from_numpy(rows).to(d["W0"].device)]).astype(np.float64)
    Wref = oracle.mu_update_W(W0r, Q, oracle.product_AHt(A[rows], H0))
    dW = float(np.max(np.abs(W1[rows] - Wref) / np.maximum(np.abs(Wref), 1e-30)))
    S = oracle.gram_fixed_W(W1)
    cols = np.sort(np.concatenate([rng.choice(N, 500, replace=False), [0, N - 1]]))
    R = oracle.product_WtA(A[:, cols].tocsr(), W1)
    Href = oracle.mu_update_H(H0[:, cols], S, R)
    dH = float(np.max(np.abs(H1[:, cols] - Href)) / np.abs(Href).max())
    print("large rows MU: sampled W rows max rel %.2e, sampled H columns max %.2e" % (dW, dH))
    assert dW <= 1e-4 and dH <= 1e-4


def test_hals_normalisation_every_row(case):
    import torch

    A, d = case
    # W0 scaled down so that every column survives the sweep (with U(0,1) W0
    # the first columns' steps (p_i - (W Q)_i) / Q_ii are far below -w_i and
    # clip whole columns to zero, which the normalisation then skips)
    W, H = d["W0"] * 1e-8, d["H0"].clone()
    step("large rows: one HALS iteration")
    nmf.nmf_csr(d["rp"], d["ci"], d["cv"], N, W, H, algo="hals", iters=1, objective=False)
    torch.cuda.synchronize()
    W1 = host(W)
    sq = np.zeros(K)
    for r0 in range(0, M, 1 << 22):
        blk = W1[r0:r0 + (1 << 22)].astype(np.float64)
        sq += np.sum(blk * blk, axis=0)
    norms = np.sqrt(sq)
    print("large rows HALS column norms of W_1: min %.9f max %.9f" % (norms.min(), norms.max()))
    np.testing.assert_allclose(norms, 1.0, rtol=1e-5)
    assert (W1 >= 0).all() and (host(H) >= 0).all()
