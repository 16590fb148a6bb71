"""Per-step parity: each exported phase of Algorithm 1 on the GPU against the
FP64 oracle, on the same seeded inputs, over shapes that span several tiles,
ragged tails, k not a multiple of the 16-wide MFMA tile, and the degenerate
sizes (one row, k = 1)."""
import numpy as np
import pytest

import oracle
import paper_1609_09154_amd as nmf
from synth import uniform
from tests.gpu_util import U32, U64, assert_gemm_bound, host, rel_diff, step, to_dev

pytestmark = pytest.mark.gpu

DT = {"f32": (np.float32, U32), "f64": (np.float64, U64)}

GRAM_SHAPES = [(1, 1), (37, 7), (1000, 10), (4099, 50), (2500, 64), (777, 100), (300, 128), (5, 16),
               (40000, 50), (3000001, 50)]  # the last two: 1024 slabs, and the tall-factor slabs
PROD_SHAPES = [(1, 1, 1), (37, 53, 7), (300, 1000, 10), (1000, 777, 50), (513, 4099, 64),
               (257, 300, 100), (64, 64, 16), (1030, 2051, 33)]


@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("rows,k", GRAM_SHAPES)
def test_gram(dt, rows, k):
    npdt, u = DT[dt]
    X = uniform((rows, k), seed=rows * 131 + k).astype(npdt)
    step("gram %s rows=%d k=%d" % (dt, rows, k))
    G = host(nmf.nmf_gram(to_dev(X, npdt)))
    Xd = X.astype(np.float64)
    ref = oracle.gram_fixed_W(Xd)
    assert_gemm_bound(G, ref, np.abs(Xd).T @ np.abs(Xd), rows, u, what="gram")
    # H H^T of Algorithm 1 is the same call on H^T
    np.testing.assert_allclose(ref, oracle.gram_fixed_H(Xd.T), rtol=1e-14)


@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("m,n,k", PROD_SHAPES)
def test_dense_AHt(dt, m, n, k):
    npdt, u = DT[dt]
    A = uniform((m, n), seed=m + 7 * n).astype(npdt)
    H = uniform((k, n), seed=k + 11 * n).astype(npdt)
    step("dense A H^T %s %dx%d k=%d" % (dt, m, n, k))
    P = host(nmf.nmf_dense_AF(to_dev(A, npdt), to_dev(H.T, npdt)))
    ref = oracle.product_AHt(A.astype(np.float64), H.astype(np.float64))
    assert_gemm_bound(P, ref, ref, n, u, what="A H^T")  # nonnegative: |A||B| = AB


@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("m,n,k", PROD_SHAPES)
def test_dense_WtA(dt, m, n, k):
    npdt, u = DT[dt]
    A = uniform((m, n), seed=3 * m + n).astype(npdt)
    W = uniform((m, k), seed=k + 5 * m).astype(npdt)
    step("dense W^T A %s %dx%d k=%d" % (dt, m, n, k))
    R = host(nmf.nmf_dense_AtF(to_dev(A, npdt), to_dev(W, npdt)))
    ref = oracle.product_WtA(A.astype(np.float64), W.astype(np.float64)).T
    assert_gemm_bound(R, ref, ref, m, u, what="W^T A")


def _update_inputs(rows, k, n, seed, npdt):
    """G = H H^T and P = A H^T from U(0,1) data, rounded to the GPU type; the
    oracle uses the rounded values so both sides see identical inputs."""
    H = uniform((k, n), seed=seed)
    A = uniform((rows, n), seed=seed + 1)
    G = (H @ H.T).astype(npdt)
    P = (A @ H.T).astype(npdt)
    X = uniform((rows, k), seed=seed + 2).astype(npdt)
    return G, P, X


@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("rows,k", [(1, 1), (333, 10), (1000, 50), (257, 64), (130, 100)])
def test_update_mu(dt, rows, k):
    npdt, u = DT[dt]
    G, P, X = _update_inputs(rows, k, 3 * k + 5, rows + k, npdt)
    Xd = to_dev(X, npdt)
    step("update mu %s rows=%d k=%d" % (dt, rows, k))
    nmf.nmf_update("mu", to_dev(G, npdt), to_dev(P, npdt), Xd)
    ref = oracle.mu_update_W(X.astype(np.float64), G.astype(np.float64), P.astype(np.float64))
    # x p / (x G): a k-term sum, one product and one division
    assert rel_diff(host(Xd), ref) <= 4 * gamma_like(k, u)


def gamma_like(K, u):
    return (K + 4) * u


@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("m,n,k", [(1, 5, 1), (400, 300, 10), (1000, 700, 50), (300, 200, 64),
                                   (150, 120, 100), (700, 500, 72), (333, 301, 96),
                                   (20000, 300, 128)])
def test_update_hals_with_normalisation(dt, m, n, k):
    """W sweep (nmf_update) + normalisation (nmf_hals_normalize) against the
    oracle's HALS W step, which normalises column by column."""
    npdt, u = DT[dt]
    A = uniform((m, n), seed=m + n + k)
    H0 = uniform((k, n), seed=2 * k + 1)
    W0 = uniform((m, k), seed=3 * k + 2)
    Q = (H0 @ H0.T).astype(npdt)
    P = (A @ H0.T).astype(npdt)
    W0 = W0.astype(npdt)
    H0 = H0.astype(npdt)
    Wd, Htd = to_dev(W0, npdt), to_dev(H0.T, npdt)
    step("update hals %s %dx%d k=%d" % (dt, m, n, k))
    nmf.nmf_update("hals", to_dev(Q, npdt), to_dev(P, npdt), Wd)
    S, norms = nmf.nmf_hals_normalize(Wd, Htd)
    Wr, Hr = oracle.hals_update_W(W0.astype(np.float64), H0.astype(np.float64),
                                  Q.astype(np.float64), P.astype(np.float64))
    tol = 50 * k * u if dt == "f32" else 1e-10
    Wg, Hg = host(Wd), host(Htd).T
    scale_w = np.abs(Wr).max()
    assert np.max(np.abs(Wg - Wr)) <= tol * max(scale_w, 1.0)
    np.testing.assert_allclose(Hg, Hr, rtol=tol, atol=tol * np.abs(Hr).max())
    np.testing.assert_allclose(host(S), Wr.T @ Wr, rtol=0, atol=tol * 10)
    # the H-side sweep is the same kernel on H^T
    Sd = Wr.T @ Wr
    R = (Wr.T @ A).astype(npdt)
    Hd2 = to_dev(Hr.T.astype(npdt), npdt)
    nmf.nmf_update("hals", to_dev(Sd.astype(npdt), npdt), to_dev(R.T, npdt), Hd2)
    Href = oracle.hals_update_H(Hr.astype(npdt).astype(np.float64), Sd.astype(npdt).astype(np.float64),
                                R.astype(np.float64))
    np.testing.assert_allclose(host(Hd2).T, Href, rtol=tol, atol=tol * np.abs(Href).max())


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("rows,k", [(1, 1), (500, 10), (700, 50), (300, 64), (257, 33)])
def test_update_abpp(dt, rows, k):
    """Exact NNLS: the solution is unique, so the GPU (any pivot path) and the
    oracle must agree up to the conditioning of G."""
    npdt, u = DT[dt]
    G, P, X = _update_inputs(rows, k, 4 * k + 7, 17 * rows + k, npdt)
    Xd = to_dev(X, npdt)
    step("update abpp %s rows=%d k=%d" % (dt, rows, k))
    piv = nmf.nmf_update("abpp", to_dev(G, npdt), to_dev(P, npdt), Xd)
    Gd, Pd = G.astype(np.float64), P.astype(np.float64)
    ref = oracle.abpp_update_W(Gd, Pd)
    got = host(Xd).astype(np.float64)
    cond = np.linalg.cond(Gd)
    tol = 1e-9 if dt == "f64" else min(1e-2, 50 * cond * u)
    assert np.max(np.abs(got - ref)) <= tol * max(np.abs(ref).max(), 1e-30), (cond, piv)
    assert (got >= 0).all()
    assert piv >= rows  # at least one passive-set solve per row (x = 0 is infeasible here)


@pytest.mark.parametrize("dt,rows,k", [("f32", 200003, 20), ("f64", 200003, 20),
                                       ("f32", 70001, 50)])
def test_update_abpp_many_rows(dt, rows, k):
    """More right-hand sides than the solver holds at once (65,536: 4096
    workgroups of four wavefronts, four right-hand sides each), so 16-lane
    rows go on to further right-hand sides; a ragged count; every row checked
    against the oracle."""
    npdt, u = DT[dt]
    G, P, X = _update_inputs(rows, k, 4 * k + 7, rows + 3 * k, npdt)
    Xd = to_dev(X, npdt)
    step("update abpp many rows %s rows=%d k=%d" % (dt, rows, k))
    piv = nmf.nmf_update("abpp", to_dev(G, npdt), to_dev(P, npdt), Xd)
    ref = oracle.abpp_update_W(G.astype(np.float64), P.astype(np.float64))
    got = host(Xd).astype(np.float64)
    cond = np.linalg.cond(G.astype(np.float64))
    tol = 1e-9 if dt == "f64" else min(1e-2, 50 * cond * u)
    assert np.max(np.abs(got - ref)) <= tol * np.abs(ref).max(), cond
    assert piv >= rows


@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("k,zero", [(10, (3,)), (50, (0, 17, 49)), (40, tuple(range(20, 40)))])
def test_update_abpp_zero_factor_rows(dt, k, zero):
    """A zero row of the fixed factor H makes the Gram's row and column and
    P's column zero (the NNLS is not unique there): those indices stay at 0
    (read off the paper's problem with x_i = y_i = 0 feasible), from a warm
    start that is positive everywhere; the rest matches the oracle. With
    k = 40 and half the indices dead, the active form's inverse Gram covers
    only the live block; the warm start holds every live index, so the
    first solve takes the active form."""
    npdt, u = DT[dt]
    rows, n = 900, 4 * k + 7
    H = uniform((k, n), seed=k)
    H[list(zero)] = 0.0
    A = uniform((rows, n), seed=k + 1)
    G = (H @ H.T).astype(npdt)
    P = (A @ H.T).astype(npdt)
    X = np.ones((rows, k), dtype=npdt)
    Xd = to_dev(X, npdt)
    step("update abpp zero factor rows %s k=%d" % (dt, k))
    nmf.nmf_update("abpp", to_dev(G, npdt), to_dev(P, npdt), Xd)
    got = host(Xd).astype(np.float64)
    ref = oracle.abpp_update_W(G.astype(np.float64), P.astype(np.float64))
    live = [i for i in range(k) if i not in zero]
    cond = np.linalg.cond(G.astype(np.float64)[np.ix_(live, live)])
    tol = 1e-9 if dt == "f64" else min(1e-2, 50 * cond * u)
    assert not np.any(got[:, list(zero)])
    assert np.max(np.abs(got - ref)) <= tol * np.abs(ref).max(), cond


@pytest.mark.parametrize("start", ["zeros", "ones"])
def test_update_abpp_singular_gram_solves_or_reports(start):
    """k = 50 from a fixed factor with n = 30 columns: G = H H^T has rank 30.
    The NNLS still has solutions, but not a unique one. The call either
    returns one, checked by Section 4.3's optimality conditions (x >= 0,
    y = G x - p >= 0, x_i y_i = 0), or reports the singular system
    (NMF_ENUMERIC) or the pivot cap (NMF_ENOTCONV)."""
    k, n, rows = 50, 30, 400
    H = uniform((k, n), seed=5)
    A = uniform((rows, n), seed=6)
    G = H @ H.T
    P = A @ H.T
    X = np.zeros((rows, k)) if start == "zeros" else np.ones((rows, k))
    Xd = to_dev(X, np.float64)
    step("update abpp singular gram start=%s" % start)
    try:
        nmf.nmf_update("abpp", to_dev(G, np.float64), to_dev(P, np.float64), Xd)
    except nmf.NMFError as e:
        print("abpp singular gram start=%s: status %d" % (start, e.status))
        assert e.status in (4, 5)
        return
    x = host(Xd)
    y = x @ G - P
    tol = 1e-8 * np.abs(P).max()
    print("abpp singular gram start=%s: solved, max |y| on the support %.3e, min y off it %.3e"
          % (start, np.abs(y[x > 0]).max(initial=0.0), y[x == 0].min(initial=0.0)))
    assert (x >= 0).all()
    assert np.abs(y[x > 0]).max(initial=0.0) <= tol
    assert y[x == 0].min(initial=0.0) >= -tol


@pytest.mark.parametrize("start", ["zeros", "ones", "random"])
@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("k", [10, 33, 50, 64])
def test_update_abpp_planted(dt, k, start):
    """Instances whose unique solution is known by construction (optimality
    conditions planted at a point with every support size 0..k), from three
    starting supports: the empty set, the full set and a random one. Covers
    both solved systems (the passive set when |F| <= 32, the active set
    otherwise)."""
    from synth import planted_nnls

    npdt, u = DT[dt]
    rows = 600
    G, P, XS = planted_nnls(rows, k, seed=40 + k)
    if start == "zeros":
        X0 = np.zeros((rows, k))
    elif start == "ones":
        X0 = np.ones((rows, k))
    else:
        X0 = (uniform((rows, k), seed=k) > 0.5).astype(np.float64)
    Xd = to_dev(X0.astype(npdt), npdt)
    step("update abpp planted %s k=%d start=%s" % (dt, k, start))
    nmf.nmf_update("abpp", to_dev(G.astype(npdt), npdt), to_dev(P.astype(npdt), npdt), Xd)
    got = host(Xd).astype(np.float64)
    cond = np.linalg.cond(G)
    tol = 1e-9 if dt == "f64" else min(1e-2, 50 * cond * u)
    err = np.max(np.abs(got - XS)) / np.abs(XS).max()
    assert err <= tol, (err, tol, cond)
    assert ((got > 0) == (XS > 0)).all()


@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (300, 200, 10), (1000, 1500, 50), (129, 4100, 64)])
def test_dense_relerr(dt, m, n, k):
    npdt, u = DT[dt]
    A = uniform((m, n), seed=m * n + 1).astype(npdt)
    W = uniform((m, k), seed=m + 2).astype(npdt) / k
    H = uniform((k, n), seed=n + 3).astype(npdt)
    step("dense relerr %s %dx%d k=%d" % (dt, m, n, k))
    got = nmf.nmf_dense_relerr(to_dev(A, npdt), to_dev(W, npdt), to_dev(H.T, npdt))
    ref = oracle.relative_error(A.astype(np.float64), W.astype(np.float64), H.astype(np.float64))
    tol = 1e-12 if dt == "f64" else 20 * k * u / max(ref, 1e-3)
    assert abs(got - ref) <= tol * ref


def test_context_follows_stream_changes_in_order():
    """One context used on two streams in turn: nmf_set_stream makes the new
    stream wait for the work already enqueued on the old one, so a call on
    the second stream cannot overwrite the shared workspace while the first
    stream's update still reads it. Results equal those of the same calls on
    one stream."""
    import torch

    dev = torch.device("cuda:0")
    rows, k = 200003, 50
    X0 = to_dev(uniform((rows, k), seed=71), np.float32)
    P = to_dev(uniform((rows, k), seed=72) * 30.0, np.float32)
    F = uniform((3 * k, k), seed=73)
    G = to_dev(F.T @ F, np.float32)
    Y = to_dev(uniform((4099, k), seed=74), np.float32)
    ctx = nmf.Context(0)
    step("stream switch: reference on one stream")
    Xa = X0.clone()
    nmf.nmf_update("abpp", G, P, Xa, ctx=ctx)
    Ga = nmf.nmf_gram(Y, ctx=ctx)
    torch.cuda.synchronize()
    step("stream switch: the same calls on two streams")
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    Xb = X0.clone()
    torch.cuda.synchronize()
    with torch.cuda.stream(s1):
        nmf.nmf_update("hals", G, P, Xb, ctx=ctx)     # enqueued, not waited for
    with torch.cuda.stream(s2):
        Gb = nmf.nmf_gram(Y, ctx=ctx)
    torch.cuda.synchronize()
    Xc = X0.clone()
    nmf.nmf_update("hals", G, P, Xc, ctx=ctx)
    torch.cuda.synchronize()
    assert torch.equal(Gb, Ga)
    assert torch.equal(Xb, Xc)
    assert torch.isfinite(Xa).all()
    ctx.close()
