"""Parity at the full workload sizes, in the launch configuration bench.py times.

Dense: A = W0 H0 + |N(0, 0.01)|, 65536 x 65536 float32 (17.2 GB, generated on
the GPU), k = 50, the first five HALS iterations through nmf_dense with the
default options (the transposed copy of A, the tuned product kernels). The
oracle runs the same iterations in FP64 from a host copy of A streamed in row
blocks: P = A H^T block by block, the HALS W step, W^T W, R = W^T A block by
block, the H step, and the relative error at every iteration.

Sparse: Erdos-Renyi 2^20 x 2^20, density 1e-4 (~1.1e8 stored entries), k = 50,
ABPP, iterations 1 to 3. At each one the oracle evaluates the relative error
of the GPU's factors over the whole matrix and solves sampled right-hand sides
of the W and H steps exactly from the GPU's own previous factors (the NNLS
solution is unique, so sampled rows are a complete check of those rows).
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


def _trace_relerr(normA_sq, P, W, Q):
    """||A - W H||_F / ||A||_F from ||A||^2 - 2 <A H^T, W> + <W^T W, H H^T>
    (P = A H^T, Q = H H^T), all in FP64. The identity is pinned against the
    direct residual by test_oracle_nmf.py::test_objective_direct_vs_trace_identity;
    with FP64 operands its rounding (about 1e-16 ||A||^2) is far below the
    1e-5 bar at the relative errors of these runs (0.03 and above)."""
    f2 = normA_sq - 2.0 * float(np.sum(P * W)) + float(np.sum(oracle.gram_fixed_W(W) * Q))
    return float(np.sqrt(max(f2, 0.0) / normA_sq))


T_DENSE = 5


def test_dense_65536_hals_T5_trajectory_full_parity():
    """The dense FP32 workload at full size for its first T = 5 iterations:
    e_t of the GPU run (nmf_dense, iters = 5, the bench's launch shapes)
    against the FP64 oracle's own trajectory from the same (W_0, H_0), every
    iteration within 1e-5; W_5 and H_5 elementwise. (With the products'
    reductions split into slabs of 8192 terms the GPU stays under 3.0e-7
    per iteration here; float32 BLAS products on the host move the same
    trajectory by up to 2.2e-6.)"""
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
    step("fullsize dense: %d HALS iterations on the GPU" % T_DENSE)
    errs, st = nmf.nmf_dense(A, W, H, algo="hals", iters=T_DENSE, objective=True)
    torch.cuda.synchronize()
    Wg, Hg = host(W).astype(np.float64), host(H).astype(np.float64)
    step("fullsize dense: host copy of A")
    Ah = host(A)
    del A
    torch.cuda.empty_cache()

    def blocks(what, t):
        step("fullsize dense oracle: iteration %d, %s" % (t, what))
        for r0 in range(0, m, ROWS):
            r1 = min(m, r0 + ROWS)
            yield r0, r1, torch.from_numpy(Ah[r0:r1]).double().numpy()

    Wo = W0n.astype(np.float64)
    Ho = H0n.astype(np.float64)
    normA_sq = 0.0
    e_ref = []
    for t in range(1, T_DENSE + 1):
        Q = oracle.gram_fixed_H(Ho)
        P = np.empty((m, k))
        for r0, r1, Ab in blocks("A H^T", t):
            P[r0:r1] = oracle.product_AHt(Ab, Ho)
            if t == 1:
                normA_sq += float(np.sum(Ab * Ab))
        e_ref.append(_trace_relerr(normA_sq, P, Wo, Q))      # e_{t-1}
        Wo, Ho = oracle.hals_update_W(Wo, Ho, Q, P)
        S = oracle.gram_fixed_W(Wo)
        R = np.zeros((k, n))
        for r0, r1, Ab in blocks("W^T A", t):
            R += oracle.product_WtA(Ab, Wo[r0:r1])
        Ho = oracle.hals_update_H(Ho, S, R)
    res = 0.0
    for r0, r1, Ab in blocks("direct residual", T_DENSE):
        res += oracle.objective_sq(Ab, Wo[r0:r1], Ho)
    e_ref.append(float(np.sqrt(res / normA_sq)))             # e_T, direct form
    e_ref = np.array(e_ref)
    per_it = np.abs(np.array(errs) - e_ref) / e_ref
    d_w = float(np.max(np.abs(Wg - Wo)) / np.abs(Wo).max())
    d_h = float(np.max(np.abs(Hg - Ho)) / np.abs(Ho).max())
    print("fullsize dense HALS T=%d: e_t gpu %s\n  oracle %s\n  per-iteration rel diff %s; "
          "max |dW|/max|W| %.2e, max |dH|/max|H| %.2e"
          % (T_DENSE, ["%.8f" % e for e in errs], ["%.8f" % e for e in e_ref],
             ["%.1e" % d for d in per_it], d_w, d_h), flush=True)
    assert per_it.max() <= 1e-5
    assert d_w <= 1e-3 and d_h <= 1e-3
    np.testing.assert_allclose(np.linalg.norm(Wg, axis=0), 1.0, rtol=1e-5)


def _csr_full():
    csr = erdos_renyi_csr(1 << 20, 1 << 20, 1e-4, seed=1609)
    return csr


def test_csr_2e20_abpp_t1_to_t3_full_parity():
    """The sparse workload at full size, one ABPP iteration at a time for
    t = 1..3 (a call with iters = 1 resumes exactly where the last one
    stopped). At each t, from the GPU's own previous factors:
    - e_t of the call against the oracle's FP64 relative error of the GPU's
      (W_t, H_t) over the whole matrix, within 1e-5;
    - sampled rows of W_t against the oracle's exact NNLS from H_{t-1}
      (Q = H_{t-1} H_{t-1}^T and those rows of A H_{t-1}^T), and sampled
      columns of H_t against the oracle's exact NNLS from W_t (S = W_t^T W_t
      and those columns of W_t^T A). The NNLS solution is unique, so the
      sampled rows and columns are a complete check of those entries."""
    import torch

    dev = torch.device("cuda:0")
    k = 50
    step("fullsize csr: generate ER 2^20 x 2^20, d = 1e-4")
    csr = _csr_full()
    m, n = csr.m, csr.n
    assert abs(csr.nnz / (m * float(n)) - 1e-4) < 2e-6
    A = scipy.sparse.csr_matrix((csr.vals.astype(np.float64), csr.colidx, csr.rowptr), shape=(m, n))
    normA_sq = float(np.sum(A.data * A.data))
    W0n, H0n = init_factors(m, n, k, seed=9154)
    rp = torch.from_numpy(csr.rowptr).to(dev)
    ci = torch.from_numpy(csr.colidx).to(dev)
    cv = torch.from_numpy(csr.vals.astype(np.float32)).to(dev)
    W = torch.from_numpy(W0n.astype(np.float32)).to(dev)
    H = torch.from_numpy(H0n.astype(np.float32)).to(dev)
    rng = np.random.default_rng(5)
    step("fullsize csr: column slices for the H checks")
    cols = np.sort(rng.choice(n, 1500, replace=False))
    A_cols = A[:, cols].tocsr()
    Hprev = H0n.astype(np.float32).astype(np.float64)
    for t in range(1, 4):
        step("fullsize csr: ABPP iteration %d on the GPU" % t)
        errs, st = nmf.nmf_csr(rp, ci, cv, n, W, H, algo="abpp", iters=1, objective=True)
        torch.cuda.synchronize()
        Wt = host(W).astype(np.float64)
        Ht = host(H).astype(np.float64)
        assert (Wt >= 0).all() and (Ht >= 0).all()

        step("fullsize csr: oracle relative error of (W_%d, H_%d)" % (t, t))
        e_ref = _trace_relerr(normA_sq, oracle.product_AHt(A, Ht), Wt, oracle.gram_fixed_H(Ht))
        d_e = abs(errs[1] - e_ref) / e_ref

        step("fullsize csr: oracle NNLS on sampled rows and columns, t = %d" % t)
        rows = np.sort(rng.choice(m, 1500, replace=False))
        W_ref = oracle.abpp_update_W(oracle.gram_fixed_H(Hprev), oracle.product_AHt(A[rows], Hprev))
        dW = float(np.max(np.abs(Wt[rows] - W_ref)) / np.abs(W_ref).max())
        H_ref = oracle.abpp_update_H(oracle.gram_fixed_W(Wt), oracle.product_WtA(A_cols, Wt))
        dH = float(np.max(np.abs(Ht[:, cols] - H_ref)) / np.abs(H_ref).max())
        print("fullsize csr ABPP t=%d: e_t gpu %.9f oracle %.9f (rel diff %.2e); sampled "
              "max |dW|/max|W| %.2e, max |dH|/max|H| %.2e; pivots %d"
              % (t, errs[1], e_ref, d_e, dW, dH, st["bpp_pivots"]))
        assert d_e <= 1e-5
        assert dW <= 1e-3 and dH <= 1e-3
        Hprev = Ht


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
