"""Sparse A with power-law row lengths and column popularity (the web-crawl
stand-in, synth.powerlaw_csr_torch): rows and columns far longer than the
SpMM's chunk length (4096 stored entries), so the chunked long-row path and
the sorted transpose are exercised on both A and A^T. Parity: the CSR
transpose bit for bit (it is unique), the products within the gamma_K bound
of the oracle's exact products, and full runs per iteration against the
oracle as for Erdos-Renyi data."""
import numpy as np
import pytest
import scipy.sparse

import oracle
import paper_1609_09154_amd as nmf
from synth import init_factors, powerlaw_csr_torch
from tests.gpu_util import U32, assert_gemm_bound, host, rel_diff, step, to_dev, torch_dev

pytestmark = pytest.mark.gpu

LONG = 4096   # the SpMM's chunk length: rows above it take the chunked path


def powerlaw(m, n, nnz, seed):
    """Host arrays of a power-law CSR matrix and its scipy form."""
    rp, ci, cv = powerlaw_csr_torch(m, n, nnz, seed=seed)
    rp, ci, cv = rp.numpy(), ci.numpy(), cv.numpy()
    return rp, ci, cv, scipy.sparse.csr_matrix((cv.astype(np.float64), ci, rp), shape=(m, n))


def boundary_matrix():
    """Rows of exactly LONG, LONG + 1, 0, 2 LONG and 3 LONG + 1 stored
    entries (and a few short rows), columns drawn without repeats."""
    n = 15000
    lengths = [LONG, LONG + 1, 0, 2 * LONG, 3 * LONG + 1, 7, 1, 300]
    rng = np.random.default_rng(11)
    cols = [np.sort(rng.choice(n, size=L, replace=False)) for L in lengths]
    rp = np.zeros(len(lengths) + 1, dtype=np.int64)
    rp[1:] = np.cumsum(lengths)
    ci = np.concatenate(cols).astype(np.int32)
    cv = rng.random(ci.size).astype(np.float32)
    return rp, ci, cv, scipy.sparse.csr_matrix((cv.astype(np.float64), ci, rp),
                                               shape=(len(lengths), n))


def dev(rp, ci, cv):
    return (to_dev(rp, np.int64), to_dev(ci, np.int32), to_dev(cv, np.float32))


CASES = [("powerlaw", (30000, 20000, 1500000, 2)), ("boundary", None)]


def get_case(name, args):
    if name == "boundary":
        return boundary_matrix()
    return powerlaw(*args)


@pytest.mark.parametrize("name,args", CASES)
def test_transpose_bit_exact(name, args):
    rp, ci, cv, S = get_case(name, args)
    m, n = S.shape
    step("powerlaw transpose %s %dx%d nnz=%d" % (name, m, n, ci.size))
    rpt, cit, cvt = nmf.nmf_csr_transpose(*dev(rp, ci, cv), n)
    T = scipy.sparse.csr_matrix((cv, ci, rp), shape=(m, n)).T.tocsr()
    T.sort_indices()
    np.testing.assert_array_equal(host(rpt), T.indptr.astype(np.int64))
    np.testing.assert_array_equal(host(cit), T.indices.astype(np.int32))
    np.testing.assert_array_equal(host(cvt), T.data.astype(np.float32))


@pytest.mark.parametrize("name,args", CASES)
@pytest.mark.parametrize("k", [50, 16, 100])
def test_spmm_long_rows(name, args, k):
    rp, ci, cv, S = get_case(name, args)
    m, n = S.shape
    lengths = np.diff(rp)
    assert lengths.max() > LONG        # the chunked path runs
    F = np.random.default_rng(k).random((n, k)).astype(np.float32)
    step("powerlaw spmm %s k=%d" % (name, k))
    P = host(nmf.nmf_csr_AF(*dev(rp, ci, cv), n, to_dev(F, np.float32)))
    ref = oracle.product_AHt(S, F.T.astype(np.float64))
    assert_gemm_bound(P, ref, ref, int(lengths.max()), U32, what="spmm A F")
    # A^T through the library's own transpose: long columns become long rows
    rpt, cit, cvt = nmf.nmf_csr_transpose(*dev(rp, ci, cv), n)
    G = np.random.default_rng(k + 1).random((m, k)).astype(np.float32)
    R = host(nmf.nmf_csr_AF(rpt, cit, cvt, m, to_dev(G, np.float32)))
    refR = oracle.product_WtA(S, G.astype(np.float64)).T
    assert_gemm_bound(R, refR, refR, int(np.diff(host(rpt)).max()), U32, what="spmm A^T F")


@pytest.mark.parametrize("algo,iters", [("hals", 6), ("mu", 6)])
def test_powerlaw_runs(algo, iters):
    m, n, k = 30000, 20000, 50
    rp, ci, cv, S = powerlaw(m, n, 1500000, 2)
    W0, H0 = init_factors(m, n, k, seed=88)
    W0, H0 = W0.astype(np.float32), H0.astype(np.float32)
    Wd, Hd = to_dev(W0, np.float32), to_dev(H0, np.float32)
    step("powerlaw %s %dx%d k=%d" % (algo, m, n, k))
    errs, _ = nmf.nmf_csr(*dev(rp, ci, cv), n, Wd, Hd, algo=algo, iters=iters, objective=True)
    _, _, er = oracle.run(S, k, algo, iters, W0.astype(np.float64), H0.astype(np.float64))
    d = rel_diff(errs, er)
    print("powerlaw %s max rel objective diff %.3e; e_T %.6f" % (algo, d, errs[-1]))
    assert d <= 1e-5, (errs, er)


def test_powerlaw_abpp_run():
    m, n, k = 4000, 3000, 20
    rp, ci, cv, S = powerlaw(m, n, 150000, 3)
    W0, H0 = init_factors(m, n, k, seed=89)
    W0, H0 = W0.astype(np.float32), H0.astype(np.float32)
    Wd, Hd = to_dev(W0, np.float32), to_dev(H0, np.float32)
    step("powerlaw abpp %dx%d k=%d" % (m, n, k))
    errs, _ = nmf.nmf_csr(*dev(rp, ci, cv), n, Wd, Hd, algo="abpp", iters=4, objective=True)
    _, _, er = oracle.run(S, k, "abpp", 4, W0.astype(np.float64), H0.astype(np.float64))
    d = rel_diff(errs, er)
    print("powerlaw abpp max rel objective diff %.3e" % d)
    # float32 storage moves this trajectory by about 6e-9
    # (test_parity_bars_cpu.py::test_powerlaw_abpp_case_stays_below_the_stated_tolerance)
    assert d <= 1e-5, (errs, er)


def test_generator_on_device_matches_its_recipe():
    """The generator's output on the GPU: a valid CSR (sorted distinct
    columns per row), heavy tails in both directions, the requested size
    within the duplicate loss."""
    import torch

    m, n, nnz = 200000, 150000, 2000000
    step("powerlaw generator on device")
    rp, ci, cv = powerlaw_csr_torch(m, n, nnz, seed=5, device=torch_dev())
    rp, ci = rp.cpu(), ci.cpu()
    assert int(rp[-1]) == ci.numel() and 0.95 * nnz <= ci.numel() <= nnz
    lengths = rp[1:] - rp[:-1]
    cnt = torch.bincount(ci.long(), minlength=n)
    assert int(lengths.max()) > 50 * float(lengths.double().mean())
    assert int(cnt.max()) > 50 * float(cnt.double().mean())
    inner = (ci[1:].long() - ci[:-1].long()) > 0
    starts = torch.zeros(ci.numel(), dtype=torch.bool)
    starts[rp[1:-1][rp[1:-1] < ci.numel()]] = True
    assert bool((inner | starts[1:]).all())
