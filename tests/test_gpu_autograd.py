"""Differentiation through T unrolled MU iterations (the forward map of
Algorithm 1 with Eq. (3)): the library's adjoint against central finite
differences of its own forward pass (FP64), against the oracle's reference
gradient (FP64 and FP32), invariance to the checkpoint interval, and the
torch.autograd layer."""
import numpy as np
import pytest

import oracle
import paper_1609_09154_amd as nmf
from synth import init_factors, planted_dense, uniform
from tests.gpu_util import host, step, to_dev

pytestmark = pytest.mark.gpu


def _problem(m, n, k, seed, k_true=None):
    A = planted_dense(m, n, k_true or k, seed=seed)
    W0, H0 = init_factors(m, n, k, seed=seed + 1)
    GW = uniform((m, k), seed=seed + 2) - 0.5
    GH = uniform((k, n), seed=seed + 3) - 0.5
    return A, W0, H0, GW, GH


def _maxrel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("dt", [np.float64, np.float32])
@pytest.mark.parametrize("m,n,k", [(300, 208, 12), (1000, 700, 64)])
def test_forward_is_nmf_dense_mu(dt, m, n, k):
    """The unrolled forward pass is the MU iteration of the driver, kernel for
    kernel (the products, the Grams summed from the updates' row-block
    shares, the updates): both give the same factors bit for bit."""
    iters = 6
    A, W0, H0, _, _ = _problem(m, n, k, seed=4)
    Ad = to_dev(A, dt)
    step("mu unrolled forward vs nmf_dense %s %dx%d k=%d" % (np.dtype(dt).name, m, n, k))
    W, H, _ = nmf.nmf_mu_unrolled_forward(Ad, to_dev(W0, dt), to_dev(H0, dt), iters,
                                          want_ckpt=False)
    Wd, Hd = to_dev(W0, dt), to_dev(H0, dt)
    nmf.nmf_dense(Ad, Wd, Hd, algo="mu", iters=iters, objective=False)
    assert np.array_equal(host(W), host(Wd)) and np.array_equal(host(H), host(Hd))


@pytest.mark.parametrize("iters,every", [(10, 10), (12, 5)])
def test_fd_check_fp64_256x128_k8(iters, every):
    """Directional finite differences of the library's own FP64 forward
    pass against the library's FP64 gradient (loss <GW, W_T> + <GH, H_T>)."""
    m, n, k = 256, 128, 8
    A, W0, H0, GW, GH = _problem(m, n, k, seed=400 + iters)
    dt = np.float64
    Ad, W0d, H0d = to_dev(A, dt), to_dev(W0, dt), to_dev(H0, dt)
    step("autograd fd fp64 T=%d every=%d" % (iters, every))
    _, _, ck = nmf.nmf_mu_unrolled_forward(Ad, W0d, H0d, iters, ckpt_every=every)
    gA, gW0, gH0 = nmf.nmf_mu_unrolled_backward(Ad, ck, to_dev(GW, dt), to_dev(GH, dt), iters,
                                                ckpt_every=every)
    gA, gW0, gH0 = host(gA), host(gW0), host(gH0)

    def loss(dA, dW, dH, h):
        W, H, _ = nmf.nmf_mu_unrolled_forward(to_dev(A + h * dA, dt), to_dev(W0 + h * dW, dt),
                                              to_dev(H0 + h * dH, dt), iters, want_ckpt=False)
        return float(np.sum(GW * host(W)) + np.sum(GH * host(H)))

    rng = np.random.default_rng(iters)
    h = 1e-6
    for which in range(4):
        d = [rng.standard_normal(x.shape) for x in (A, W0, H0)]
        if which < 3:
            d = [x if i == which else np.zeros_like(x) for i, x in enumerate(d)]
        fd = (loss(*d, h) - loss(*d, -h)) / (2 * h)
        an = float(np.sum(gA * d[0]) + np.sum(gW0 * d[1]) + np.sum(gH0 * d[2]))
        print("direction %d: fd %.12e analytic %.12e" % (which, fd, an))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))


@pytest.mark.parametrize("dt,tol", [(np.float64, 1e-10), (np.float32, 5e-4)])
@pytest.mark.parametrize("m,n,k,iters,every", [(300, 200, 10, 12, 5), (257, 333, 33, 7, 3),
                                               (128, 96, 64, 4, 10)])
def test_gradient_matches_oracle(dt, tol, m, n, k, iters, every):
    A, W0, H0, GW, GH = _problem(m, n, k, seed=m + k)
    A32 = A.astype(dt)
    W0c, H0c = W0.astype(dt), H0.astype(dt)
    step("autograd vs oracle %s %dx%d k=%d T=%d" % (np.dtype(dt).name, m, n, k, iters))
    Ad = to_dev(A32, dt)
    W, H, ck = nmf.nmf_mu_unrolled_forward(Ad, to_dev(W0c, dt), to_dev(H0c, dt), iters,
                                           ckpt_every=every)
    gA, gW0, gH0 = nmf.nmf_mu_unrolled_backward(Ad, ck, to_dev(GW.astype(dt), dt),
                                                to_dev(GH.astype(dt), dt), iters,
                                                ckpt_every=every)
    A64 = A32.astype(np.float64)
    Wr, Hr, _ = oracle.mu_unrolled_forward(A64, W0c.astype(np.float64), H0c.astype(np.float64),
                                           iters)
    rA, rW, rH = oracle.mu_unrolled_vjp(A64, W0c.astype(np.float64), H0c.astype(np.float64),
                                        iters, GW.astype(dt).astype(np.float64),
                                        GH.astype(dt).astype(np.float64))
    errs = [_maxrel(host(W).astype(np.float64), Wr), _maxrel(host(H).astype(np.float64), Hr),
            _maxrel(host(gA).astype(np.float64), rA), _maxrel(host(gW0).astype(np.float64), rW),
            _maxrel(host(gH0).astype(np.float64), rH)]
    print("W_T %.2e H_T %.2e dA %.2e dW0 %.2e dH0 %.2e" % tuple(errs))
    assert max(errs) <= tol


def test_checkpoint_interval_does_not_change_the_gradient():
    """Recomputed segments repeat the forward pass bit for bit, so every
    checkpoint interval gives the same gradients of W_0 and H_0, bit for bit.
    dL/dA sums one term per iteration, added to dL/dA one checkpoint segment
    at a time (the segment's terms in one float32 matrix-core sum): the
    grouping follows the interval, so dL/dA agrees to float32 rounding."""
    m, n, k, iters = 200, 150, 16, 9
    A, W0, H0, GW, GH = _problem(m, n, k, seed=77)
    dt = np.float32
    Ad, W0d, H0d = to_dev(A, dt), to_dev(W0, dt), to_dev(H0, dt)
    outs = []
    for every in (1, 2, 4, 9, 20):
        step("autograd ckpt every=%d" % every)
        _, _, ck = nmf.nmf_mu_unrolled_forward(Ad, W0d, H0d, iters, ckpt_every=every)
        g = nmf.nmf_mu_unrolled_backward(Ad, ck, to_dev(GW, dt), to_dev(GH, dt), iters,
                                         ckpt_every=every)
        outs.append([host(x) for x in g])
    for o in outs[1:]:
        gA, gW0, gH0 = o
        assert np.array_equal(gW0, outs[0][1]) and np.array_equal(gH0, outs[0][2])
        ref = outs[0][0]
        np.testing.assert_allclose(gA, ref, rtol=0, atol=1e-5 * float(np.abs(ref).max()))


def test_zero_iterations_is_the_identity():
    m, n, k = 40, 30, 5
    A, W0, H0, GW, GH = _problem(m, n, k, seed=5)
    dt = np.float64
    Ad = to_dev(A, dt)
    W, H, ck = nmf.nmf_mu_unrolled_forward(Ad, to_dev(W0, dt), to_dev(H0, dt), 0)
    gA, gW0, gH0 = nmf.nmf_mu_unrolled_backward(Ad, ck, to_dev(GW, dt), to_dev(GH, dt), 0)
    assert np.array_equal(host(W), W0) and np.array_equal(host(H), H0)
    assert np.array_equal(host(gW0), GW) and np.array_equal(host(gH0), GH)
    assert not np.any(host(gA))


def test_torch_autograd_layer_gradcheck():
    """torch.autograd.gradcheck (finite differences in FP64) on the layer,
    with the fitting loss ||A - W_T H_T||^2 through torch."""
    import torch

    m, n, k, iters = 24, 16, 3, 4
    A, W0, H0, _, _ = _problem(m, n, k, seed=9)
    dev = torch.device("cuda:0")
    At = torch.tensor(A, device=dev, requires_grad=True)
    Wt = torch.tensor(W0, device=dev, requires_grad=True)
    Ht = torch.tensor(H0, device=dev, requires_grad=True)

    def f(A_, W_, H_):
        W, H = nmf.mu_unrolled(A_, W_, H_, iters, 1e-16, 2)
        return ((A_ - W @ H) ** 2).sum()

    step("autograd gradcheck")
    assert torch.autograd.gradcheck(f, (At, Wt, Ht), eps=1e-6, atol=1e-7, rtol=1e-5)
