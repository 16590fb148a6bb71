"""Parity at the full workload sizes, in the launch configuration bench.py times.

Dense: A = W0 H0 + |N(0, 0.01)|, 65536 x 65536 float32 (17.2 GB, generated on
the GPU), k = 50, one HALS iteration through nmf_dense with the default options
(the transposed copy of A, the tuned product kernels). The oracle repeats the
same iteration in FP64 from host copies of A streamed in row blocks: P = A H^T
block by block, the HALS W step, W^T W, R = A^T W block by block, the H step,
and the relative error before and after.

Sparse: Erdos-Renyi 2^20 x 2^20, density 1e-4 (~1.1e8 stored entries), k = 50,
ABPP. The oracle solves sampled right-hand sides of the W and H steps exactly
(the NNLS solution is unique, so sampled rows are a complete check of those
rows), from products it forms on the host.
"""
import numpy as np
import pytest
import scipy.sparse

import oracle
import paper_1609_09154_amd as nmf
from synth import erdos_renyi_csr, init_factors, planted_dense, planted_dense_torch
from tests.gpu_util import host, rel_diff, step

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

ROWS = 4096  # host block height for the oracle's passes over A


def _blocks(A):
    m = A.shape[0]
    for r0 in range(0, m, ROWS):
        r1 = min(m, r0 + ROWS)
        yield r0, r1, A[r0:r1].double().cpu().numpy()


def test_dense_65536_hals_one_iteration_full_parity():
    import torch

    m = n = 65536
    k = 50
    dev = torch.device("cuda:0")
    step("fullsize dense: generate A 65536^2 fp32")
    A = planted_dense_torch(m, n, 50, sigma=0.01, seed=1609, device=dev, dtype=torch.float32)
    W0n, H0n = init_factors(m, n, k, seed=9154)
    W0n = W0n.astype(np.float32)
    H0n = H0n.astype(np.float32)
    W = torch.from_numpy(W0n).to(dev)
    H = torch.from_numpy(H0n).to(dev)
    step("fullsize dense: one HALS iteration on the GPU")
    errs, st = nmf.nmf_dense(A, W, H, algo="hals", iters=1, objective=True)
    torch.cuda.synchronize()
    Wg, Hg = host(W).astype(np.float64), host(H).astype(np.float64)

    step("fullsize dense: oracle iteration from host blocks of A")
    W0 = W0n.astype(np.float64)
    H0 = H0n.astype(np.float64)
    Q = oracle.gram_fixed_H(H0)
    P = np.empty((m, k))
    normA = 0.0
    res0 = 0.0
    for r0, r1, Ab in _blocks(A):
        P[r0:r1] = oracle.product_AHt(Ab, H0)
        normA += float(np.sum(Ab * Ab))
        res0 += oracle.objective_sq(Ab, W0[r0:r1], H0)
    W1, Hs = oracle.hals_update_W(W0, H0, Q, P)
    S = oracle.gram_fixed_W(W1)
    R = np.zeros((k, n))
    for r0, r1, Ab in _blocks(A):
        R += oracle.product_WtA(Ab, W1[r0:r1])
    H1 = oracle.hals_update_H(Hs, S, R)
    res1 = 0.0
    for r0, r1, Ab in _blocks(A):
        res1 += oracle.objective_sq(Ab, W1[r0:r1], H1)
    e_ref = [np.sqrt(res0 / normA), np.sqrt(res1 / normA)]
    d_e = rel_diff(errs, e_ref)
    d_w = float(np.max(np.abs(Wg - W1)) / np.abs(W1).max())
    d_h = float(np.max(np.abs(Hg - H1)) / np.abs(H1).max())
    print("fullsize dense HALS: rel err gpu %s oracle %s; objective diff %.2e, "
          "max |dW|/max|W| %.2e, max |dH|/max|H| %.2e" % (errs, e_ref, d_e, d_w, d_h))
    assert d_e <= 1e-5
    assert d_w <= 1e-3 and d_h <= 1e-3
    np.testing.assert_allclose(np.linalg.norm(Wg, axis=0), 1.0, rtol=1e-5)


def _csr_full():
    csr = erdos_renyi_csr(1 << 20, 1 << 20, 1e-4, seed=1609)
    return csr


def test_csr_2e20_abpp_sampled_parity():
    import torch

    dev = torch.device("cuda:0")
    k = 50
    step("fullsize csr: generate ER 2^20 x 2^20, d = 1e-4")
    csr = _csr_full()
    m, n = csr.m, csr.n
    assert abs(csr.nnz / (m * float(n)) - 1e-4) < 2e-6
    A = scipy.sparse.csr_matrix((csr.vals.astype(np.float64), csr.colidx, csr.rowptr), shape=(m, n))
    W0n, H0n = init_factors(m, n, k, seed=9154)
    W0n = W0n.astype(np.float32)
    H0n = H0n.astype(np.float32)
    rp = torch.from_numpy(csr.rowptr).to(dev)
    ci = torch.from_numpy(csr.colidx).to(dev)
    cv = torch.from_numpy(csr.vals.astype(np.float32)).to(dev)

    # W step in the driver's configuration: one full ABPP iteration.
    step("fullsize csr: one ABPP iteration on the GPU")
    W = torch.from_numpy(W0n).to(dev)
    H = torch.from_numpy(H0n).to(dev)
    errs, st = nmf.nmf_csr(rp, ci, cv, n, W, H, algo="abpp", iters=1, objective=True)
    torch.cuda.synchronize()
    Wg = host(W).astype(np.float64)
    Hg = host(H).astype(np.float64)
    print("fullsize csr ABPP: rel err %s, pivots %d" % (errs, st["bpp_pivots"]))

    step("fullsize csr: oracle W step on sampled rows")
    H0 = H0n.astype(np.float64)
    Q = oracle.gram_fixed_H(H0)
    rng = np.random.default_rng(5)
    rows = np.sort(rng.choice(m, 1500, replace=False))
    P_rows = oracle.product_AHt(A[rows], H0)
    W_ref = oracle.abpp_update_W(Q, P_rows)
    scale = np.abs(W_ref).max()
    dW = float(np.max(np.abs(Wg[rows] - W_ref)) / scale)
    print("sampled W rows: max |dW| / max|W| = %.2e" % dW)
    assert dW <= 1e-3

    # H step from generator inputs (W0): GPU products, Gram and update at full
    # size through the per-step calls, oracle on sampled columns.
    step("fullsize csr: H step from W0 via per-step calls")
    rpt, cit, cvt = nmf.nmf_csr_transpose(rp, ci, cv, n)
    Wd = torch.from_numpy(W0n).to(dev)
    Rt = nmf.nmf_csr_AF(rpt, cit, cvt, m, Wd)           # (A^T W0), n x k
    Sg = nmf.nmf_gram(Wd)
    X = torch.zeros((n, k), dtype=torch.float32, device=dev)
    nmf.nmf_update("abpp", Sg, Rt, X)
    torch.cuda.synchronize()
    W0 = W0n.astype(np.float64)
    S = oracle.gram_fixed_W(W0)
    cols = np.sort(rng.choice(n, 1500, replace=False))
    R_cols = oracle.product_WtA(A[:, cols].tocsr(), W0)  # k x |cols|
    np.testing.assert_allclose(host(Sg), S, rtol=1e-4)
    dR = rel_diff(host(Rt)[cols].T, R_cols)
    H_ref = oracle.abpp_update_H(S, R_cols)
    dH = float(np.max(np.abs(host(X)[cols].T - H_ref)) / np.abs(H_ref).max())
    print("sampled H columns: R rel diff %.2e, max |dH| / max|H| = %.2e" % (dR, dH))
    assert dR <= 1e-4 and dH <= 1e-3

    # Whole-run properties at full size: nonnegative factors, objective below
    # its start, and e_t against the oracle's evaluation of the same factors.
    assert (Wg >= 0).all() and (Hg >= 0).all()
    assert errs[1] < errs[0]


def test_csr_scaled_copy_abpp_20_iterations():
    """The sparse workload scaled down to 8192 x 8192 at the same mean row
    length (about 105 stored entries per row), k = 50, all 20 ABPP iterations
    of a run against the FP64 oracle's relative error per iteration."""
    m = n = 8192
    k, iters = 50, 20
    csr = erdos_renyi_csr(m, n, 104.9 / n, seed=1609)
    A = scipy.sparse.csr_matrix((csr.vals.astype(np.float64), csr.colidx, csr.rowptr),
                                shape=(m, n))
    W0, H0 = init_factors(m, n, k, seed=9154)
    W0, H0 = W0.astype(np.float32), H0.astype(np.float32)
    import torch

    dev = torch.device("cuda:0")
    rp = torch.from_numpy(csr.rowptr).to(dev)
    ci = torch.from_numpy(csr.colidx).to(dev)
    cv = torch.from_numpy(csr.vals.astype(np.float32)).to(dev)
    W = torch.from_numpy(W0).to(dev)
    H = torch.from_numpy(H0).to(dev)
    step("scaled csr 8192^2: 20 ABPP iterations on the GPU")
    errs, _ = nmf.nmf_csr(rp, ci, cv, n, W, H, algo="abpp", iters=iters, objective=True)
    step("scaled csr 8192^2: oracle")
    _, _, er = oracle.run(A, k, "abpp", iters, W0.astype(np.float64), H0.astype(np.float64))
    d = rel_diff(errs, er)
    print("scaled csr ABPP 20 iterations: max rel objective diff %.3e; e_T %.6f" % (d, errs[-1]))
    assert d <= 1e-5, (errs, er)


@pytest.mark.parametrize("fmt", ["bf16", "fp8"])
def test_lowp_131072x65536_k100_hals_one_iteration_full_parity(fmt):
    """Precision workloads at full size: A = W0 H0 + |N(0, 0.01)| stored in
    bfloat16 (131072 x 65536, 17.2 GB) or FP8 E4M3 (8.6 GB), k = 100, one
    HALS iteration with the products on the BF16 or FP8 matrix cores. The
    oracle repeats the iteration in FP64 on the same stored values, rounding
    the product's factor operand as the method does (oracle.round_bf16, or
    oracle.round_fp8_scaled with its per-column scales taken over the whole
    factor), from host copies of A streamed in row blocks."""
    import torch

    m, n, k = 131072, 65536, 100
    dev = torch.device("cuda:0")
    step("fullsize %s: generate A 131072 x 65536" % fmt)
    if fmt == "bf16":
        A = planted_dense_torch(m, n, 100, sigma=0.01, seed=1609, device=dev,
                                dtype=torch.bfloat16)
        round_H, round_W = oracle.round_bf16, oracle.round_bf16
    else:
        A = planted_dense_torch(m, n, 100, sigma=0.01, seed=1609, device=dev,
                                dtype=torch.float32).to(torch.float8_e4m3fn)
        torch.cuda.synchronize()
        round_H = lambda X: oracle.round_fp8_scaled(X, 0)   # noqa: E731  (k x n)
        round_W = lambda X: oracle.round_fp8_scaled(X, 1)   # noqa: E731  (m x k)
    W0n, H0n = init_factors(m, n, k, seed=9154)
    W0n = W0n.astype(np.float32)
    H0n = H0n.astype(np.float32)
    W = torch.from_numpy(W0n).to(dev)
    H = torch.from_numpy(H0n).to(dev)
    step("fullsize %s: one HALS iteration on the GPU" % fmt)
    errs, st = nmf.nmf_dense(A, W, H, algo="hals", iters=1, objective=True)
    torch.cuda.synchronize()
    Wg, Hg = host(W).astype(np.float64), host(H).astype(np.float64)

    def blocks(what):
        for r0 in range(0, m, ROWS):
            r1 = min(m, r0 + ROWS)
            if r0 % (8 * ROWS) == 0:
                step("fullsize %s oracle: %s, rows %d of %d" % (fmt, what, r0, m))
            yield r0, r1, A[r0:r1].float().cpu().to(torch.float64).numpy()

    step("fullsize %s: oracle iteration from host blocks of A" % fmt)
    W0 = W0n.astype(np.float64)
    H0 = H0n.astype(np.float64)
    Q = oracle.gram_fixed_H(H0)
    H0r = round_H(H0)
    P = np.empty((m, k))
    normA = 0.0
    res0 = 0.0
    for r0, r1, Ab in blocks("A H^T"):
        P[r0:r1] = oracle.product_AHt(Ab, H0r)
        normA += float(np.sum(Ab * Ab))
        res0 += oracle.objective_sq(Ab, W0[r0:r1], H0)
    W1, Hs = oracle.hals_update_W(W0, H0, Q, P)
    S = oracle.gram_fixed_W(W1)
    W1r = round_W(W1)
    R = np.zeros((k, n))
    for r0, r1, Ab in blocks("W^T A"):
        R += oracle.product_WtA(Ab, W1r[r0:r1])
    H1 = oracle.hals_update_H(Hs, S, R)
    res1 = 0.0
    for r0, r1, Ab in blocks("residual"):
        res1 += oracle.objective_sq(Ab, W1[r0:r1], H1)
    e_ref = [np.sqrt(res0 / normA), np.sqrt(res1 / normA)]
    d_e = rel_diff(errs, e_ref)
    d_w = float(np.max(np.abs(Wg - W1)) / np.abs(W1).max())
    d_h = float(np.max(np.abs(Hg - H1)) / np.abs(H1).max())
    print("fullsize %s HALS: rel err gpu %s oracle %s; objective diff %.2e, "
          "max |dW|/max|W| %.2e, max |dH|/max|H| %.2e" % (fmt, errs, e_ref, d_e, d_w, d_h))
    assert d_e <= 1e-4
    assert d_w <= 1e-2 and d_h <= 1e-2


@pytest.mark.parametrize("algo,dt", [("mu", "f32"), ("hals", "f64"), ("hals", "f32")])
def test_unrolled_8192x4096_k64_T50_gradient_full_parity(algo, dt):
    """Differentiation workloads at full size: A = W0 H0 + |N(0, 0.01)| with
    planted rank 64 (8192 x 4096, float32 values), k = 64, 50 unrolled MU or
    HALS iterations, checkpoints every 10; loss <GW, W_T> + <GH, H_T>. The
    oracle's FP64 reference gradient runs on the same float32 inputs.

    MU (FP32) and HALS in FP64 are compared elementwise. The HALS map is
    piecewise smooth (the max(0, .) of every sweep entry), and over 50
    iterations FP32 rounding moves a few entries across a piece boundary (the
    final H has one clipped entry fewer in FP32 than in FP64 here); the
    gradient jumps there, so the FP32 HALS gradient is compared in the
    Frobenius norm, its forward pass elementwise."""
    import torch

    m, n, k, T, every = 8192, 4096, 64, 50, 10
    dev = torch.device("cuda:0")
    tdt = torch.float64 if dt == "f64" else torch.float32
    A = planted_dense(m, n, 64, sigma=0.01, seed=1609).astype(np.float32)
    W0, H0 = init_factors(m, n, k, seed=9154)
    W0 = W0.astype(np.float32)
    H0 = H0.astype(np.float32)
    from synth import uniform

    GW = (uniform((m, k), seed=11) - 0.5).astype(np.float32)
    GH = (uniform((k, n), seed=12) - 0.5).astype(np.float32)
    fwd, bwd = ((nmf.nmf_mu_unrolled_forward, nmf.nmf_mu_unrolled_backward) if algo == "mu"
                else (nmf.nmf_hals_unrolled_forward, nmf.nmf_hals_unrolled_backward))
    step("fullsize autograd %s %s: forward + backward on the GPU" % (algo, dt))

    def d(x):
        return torch.from_numpy(x).to(dev, tdt)

    Ad = d(A)
    W, H, ck = fwd(Ad, d(W0), d(H0), T, ckpt_every=every)
    gA, gW0, gH0 = bwd(Ad, ck, d(GW), d(GH), T, ckpt_every=every)
    torch.cuda.synchronize()
    step("fullsize autograd %s %s: oracle FP64 reference gradient" % (algo, dt))
    A64 = A.astype(np.float64)
    W064, H064 = W0.astype(np.float64), H0.astype(np.float64)
    G64 = (GW.astype(np.float64), GH.astype(np.float64))
    if algo == "mu":
        Wr, Hr, _ = oracle.mu_unrolled_forward(A64, W064, H064, T)
        rA, rW, rH = oracle.mu_unrolled_vjp(A64, W064, H064, T, *G64)
    else:
        Wr, Hr = oracle.hals_unrolled_forward(A64, W064, H064, T)
        rA, rW, rH = oracle.hals_unrolled_vjp(A64, W064, H064, T, *G64)
    got = [host(x).astype(np.float64) for x in (W, H, gA, gW0, gH0)]
    ref = [Wr, Hr, rA, rW, rH]
    mrel = [float(np.max(np.abs(a - b)) / np.abs(b).max()) for a, b in zip(got, ref)]
    frob = [float(np.linalg.norm(a - b) / np.linalg.norm(b)) for a, b in zip(got, ref)]
    print("fullsize autograd %s %s vs FP64 oracle (max / Frobenius relative): W_T %.2e/%.2e "
          "H_T %.2e/%.2e dA %.2e/%.2e dW0 %.2e/%.2e dH0 %.2e/%.2e; zeros in W_T, H_T: %d, %d "
          "(oracle %d, %d)" % ((algo, dt) + tuple(v for pair in zip(mrel, frob) for v in pair)
                               + (int((got[0] == 0).sum()), int((got[1] == 0).sum()),
                                  int((Wr == 0).sum()), int((Hr == 0).sum()))))
    if dt == "f64":
        assert max(mrel) <= 1e-10
    elif algo == "mu":
        assert max(mrel) <= 1e-3
    else:
        assert max(mrel[:2]) <= 1e-3
        assert max(frob[2:]) <= 1e-2
