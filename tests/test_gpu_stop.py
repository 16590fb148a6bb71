"""Stationarity and tolerance stops (Section 6.2): the projected-gradient
kernel against the oracle's definition, and nmf_dense / nmf_csr with
stop = "pgrad" / "relerr" against oracle.run_until (same stopping iteration,
same metric values)."""
import numpy as np
import pytest
import scipy.sparse

import oracle
import paper_1609_09154_amd as nmf
from synth import csr_from_dense, erdos_renyi_csr, init_factors, planted_dense, uniform
from tests.gpu_util import host, rel_diff, step, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dt,tol", [(np.float64, 1e-12), (np.float32, 1e-5)])
@pytest.mark.parametrize("rows,k", [(1, 1), (1000, 5), (777, 50), (300, 100), (129, 128)])
def test_projected_gradient_kernel(dt, tol, rows, k):
    X = uniform((rows, k), seed=rows + k)
    X[X < 0.3] = 0.0                       # entries at the bound
    P = uniform((rows, k), seed=rows + k + 1) * k
    B = uniform((k, 2 * k + 3), seed=k + 2)
    G = B @ B.T
    X, P, G = X.astype(dt), P.astype(dt), G.astype(dt)
    step("pgrad kernel %s rows=%d k=%d" % (np.dtype(dt).name, rows, k))
    got = nmf.nmf_projected_gradient_sq(to_dev(X, dt), to_dev(P, dt), to_dev(G, dt))
    X64, G64 = X.astype(np.float64), G.astype(np.float64)
    ref = oracle.projected_gradient_sq(X64, X64 @ G64 - P.astype(np.float64))
    assert abs(got - ref) <= tol * ref


def _robust(ratios, tol, margin):
    """True if no ratio sits within `margin` (relative) of the threshold."""
    r = np.array(ratios[1:])
    return not np.any(np.abs(r - tol) <= margin * tol)


@pytest.mark.parametrize("algo,stop,tol", [("hals", "pgrad", 2e-2), ("mu", "relerr", 1e-2),
                                           ("abpp", "pgrad", 1e-3), ("mu", "pgrad", 0.1)])
def test_dense_fp64_stop_matches_oracle(algo, stop, tol):
    m, n, k = 200, 150, 6
    A = planted_dense(m, n, k, seed=61)
    W0, H0 = init_factors(m, n, k, seed=62)
    cap = 300
    _, _, e_ref, r_ref, t_ref = oracle.run_until(A, k, algo, cap, W0, H0, stop, tol)
    assert t_ref < cap
    dt = np.float64
    W, H = to_dev(W0, dt), to_dev(H0, dt)
    step("stop fp64 %s %s" % (algo, stop))
    errs, st = nmf.nmf_dense(to_dev(A, dt), W, H, algo=algo, iters=cap, objective=True,
                             stop=stop, tol=tol)
    print("%s %s: oracle stops at %d, gpu at %d; ratio oracle %.6e gpu %.6e" %
          (algo, stop, t_ref, st["iters_done"], r_ref[-1], st["pgrad_ratio"]))
    if stop == "pgrad":
        metric = r_ref
    else:
        metric = [1.0] + [(e_ref[s - 1] - e_ref[s]) / e_ref[s - 1] for s in range(1, len(e_ref))]
    if _robust(metric, tol, 1e-6):
        assert st["iters_done"] == t_ref
    assert len(errs) == st["iters_done"] + 1
    n_cmp = min(len(errs), len(e_ref))
    assert rel_diff(errs[:n_cmp], e_ref[:n_cmp]) <= 1e-9
    if stop == "pgrad":
        assert abs(st["pgrad_ratio"] - r_ref[st["iters_done"]]) <= 1e-8 * r_ref[st["iters_done"]]
    else:
        assert np.isnan(st["pgrad_ratio"])


def test_dense_fp32_pgrad_ratio_matches_oracle():
    m, n, k = 1500, 1100, 20
    A = planted_dense(m, n, k, seed=71).astype(np.float32)
    W0, H0 = init_factors(m, n, k, seed=72)
    W0, H0 = W0.astype(np.float32), H0.astype(np.float32)
    step("stop fp32 hals pgrad")
    W, H = to_dev(W0, np.float32), to_dev(H0, np.float32)
    errs, st = nmf.nmf_dense(to_dev(A, np.float32), W, H, algo="hals", iters=60, objective=True,
                             stop="pgrad", tol=0.1)
    t = st["iters_done"]
    assert t < 60 and st["pgrad_ratio"] <= 0.1
    A64 = A.astype(np.float64)
    Wr, Hr, _ = oracle.run(A64, k, "hals", t, W0, H0, track_error=False)
    ratio = oracle.projected_gradient_norm(A64, Wr, Hr) / oracle.projected_gradient_norm(
        A64, W0.astype(np.float64), H0.astype(np.float64))
    print("fp32 hals: stop at %d, ratio gpu %.6e oracle %.6e" % (t, st["pgrad_ratio"], ratio))
    assert abs(st["pgrad_ratio"] - ratio) <= 1e-3 * ratio


def test_csr_pgrad_stop():
    csr = erdos_renyi_csr(3000, 2600, 0.03, seed=81)
    A = scipy.sparse.csr_matrix((csr.vals.astype(np.float64), csr.colidx, csr.rowptr),
                                shape=(csr.m, csr.n))
    k = 10
    W0, H0 = init_factors(csr.m, csr.n, k, seed=82)
    W0, H0 = W0.astype(np.float32), H0.astype(np.float32)
    import torch

    dev = torch.device("cuda:0")
    rp = torch.from_numpy(csr.rowptr).to(dev)
    ci = torch.from_numpy(csr.colidx).to(dev)
    cv = torch.from_numpy(csr.vals.astype(np.float32)).to(dev)
    W, H = to_dev(W0, np.float32), to_dev(H0, np.float32)
    step("stop csr hals pgrad")
    errs, st = nmf.nmf_csr(rp, ci, cv, csr.n, W, H, algo="hals", iters=60, objective=True,
                           stop="pgrad", tol=0.05)
    t = st["iters_done"]
    Wr, Hr, _ = oracle.run(A, k, "hals", t, W0, H0, track_error=False)
    ratio = oracle.projected_gradient_norm(A, Wr, Hr) / oracle.projected_gradient_norm(
        A, W0.astype(np.float64), H0.astype(np.float64))
    print("csr hals: stop at %d, ratio gpu %.6e oracle %.6e" % (t, st["pgrad_ratio"], ratio))
    assert t < 60 and st["pgrad_ratio"] <= 0.05
    assert abs(st["pgrad_ratio"] - ratio) <= 1e-3 * ratio
