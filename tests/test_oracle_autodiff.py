"""Pins for the oracle's reference gradient of T unrolled MU iterations:
central finite differences in FP64, and torch's reverse-mode autograd on
the same forward formula (a separate implementation of the chain rule)."""
import numpy as np
import pytest

import oracle
from synth import init_factors, planted_dense, uniform


def _problem(m, n, k, seed):
    A = planted_dense(m, n, k, seed=seed)
    W0, H0 = init_factors(m, n, k, seed=seed + 1)
    GW = uniform((m, k), seed=seed + 2) - 0.5
    GH = uniform((k, n), seed=seed + 3) - 0.5
    return A, W0, H0, GW, GH


def _loss(A, W0, H0, T, GW, GH):
    W, H, _ = oracle.mu_unrolled_forward(A, W0, H0, T)
    return float(np.sum(GW * W) + np.sum(GH * H))


@pytest.mark.parametrize("T", [1, 2, 5])
def test_vjp_matches_central_differences(T):
    m, n, k = 7, 6, 3
    A, W0, H0, GW, GH = _problem(m, n, k, seed=100 + T)
    gA, gW, gH = oracle.mu_unrolled_vjp(A, W0, H0, T, GW, GH)
    rng = np.random.default_rng(T)
    h = 1e-6
    for _ in range(5):
        dA = rng.standard_normal(A.shape)
        dW = rng.standard_normal(W0.shape)
        dH = rng.standard_normal(H0.shape)
        fd = (_loss(A + h * dA, W0 + h * dW, H0 + h * dH, T, GW, GH)
              - _loss(A - h * dA, W0 - h * dW, H0 - h * dH, T, GW, GH)) / (2 * h)
        an = np.sum(gA * dA) + np.sum(gW * dW) + np.sum(gH * dH)
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)
    # each input on its own (a wrong term in one of them cannot cancel)
    for which in range(3):
        d = [np.zeros_like(A), np.zeros_like(W0), np.zeros_like(H0)]
        d[which] = rng.standard_normal(d[which].shape)
        fd = (_loss(A + h * d[0], W0 + h * d[1], H0 + h * d[2], T, GW, GH)
              - _loss(A - h * d[0], W0 - h * d[1], H0 - h * d[2], T, GW, GH)) / (2 * h)
        an = [np.sum(gA * d[0]), np.sum(gW * d[1]), np.sum(gH * d[2])][which]
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (which, fd, an)


def test_vjp_matches_torch_autograd():
    torch = pytest.importorskip("torch")
    m, n, k, T = 20, 15, 4, 6
    A, W0, H0, GW, GH = _problem(m, n, k, seed=7)
    gA, gW, gH = oracle.mu_unrolled_vjp(A, W0, H0, T, GW, GH)
    At = torch.tensor(A, requires_grad=True)
    Wt = torch.tensor(W0, requires_grad=True)
    Ht = torch.tensor(H0, requires_grad=True)
    W, H = Wt, Ht
    eps = oracle.MU_EPS
    for _ in range(T):
        W = W * (At @ H.T) / (W @ (H @ H.T) + eps)
        H = H * (W.T @ At) / ((W.T @ W) @ H + eps)
    L = (torch.tensor(GW) * W).sum() + (torch.tensor(GH) * H).sum()
    L.backward()
    for mine, ref in ((gA, At.grad), (gW, Wt.grad), (gH, Ht.grad)):
        ref = ref.numpy()
        assert np.max(np.abs(mine - ref)) <= 1e-10 * np.abs(ref).max()


def test_vjp_of_the_objective():
    """L = ||A - W_T H_T||_F^2 (the loss a fitting layer would use)."""
    m, n, k, T = 9, 8, 3, 3
    A, W0, H0, _, _ = _problem(m, n, k, seed=31)
    W, H, _ = oracle.mu_unrolled_forward(A, W0, H0, T)
    Rz = A - W @ H
    gA_direct = 2 * Rz
    gA, gW, gH = oracle.mu_unrolled_vjp(A, W0, H0, T, -2 * Rz @ H.T, -2 * W.T @ Rz)
    gA = gA + gA_direct

    def L(A_, W_, H_):
        Wt, Htt, _ = oracle.mu_unrolled_forward(A_, W_, H_, T)
        return float(np.sum((A_ - Wt @ Htt) ** 2))

    rng = np.random.default_rng(0)
    h = 1e-6
    for _ in range(3):
        dA, dW, dH = (rng.standard_normal(x.shape) for x in (A, W0, H0))
        fd = (L(A + h * dA, W0 + h * dW, H0 + h * dH) - L(A - h * dA, W0 - h * dW, H0 - h * dH)) / (2 * h)
        an = np.sum(gA * dA) + np.sum(gW * dW) + np.sum(gH * dH)
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))
