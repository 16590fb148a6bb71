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


# --- HALS ------------------------------------------------------------------

def _hals_loss(A, W0, H0, T, GW, GH):
    W, H = oracle.hals_unrolled_forward(A, W0, H0, T)
    return float(np.sum(GW * W) + np.sum(GH * H))


@pytest.mark.parametrize("T", [1, 2, 4])
def test_hals_vjp_matches_central_differences(T):
    m, n, k = 9, 7, 3
    A, W0, H0, GW, GH = _problem(m, n, k, seed=200 + T)
    gA, gW, gH = oracle.hals_unrolled_vjp(A, W0, H0, T, GW, GH)
    rng = np.random.default_rng(T)
    h = 1e-6
    for which in range(4):
        d = [rng.standard_normal(A.shape), rng.standard_normal(W0.shape),
             rng.standard_normal(H0.shape)]
        if which < 3:   # each input on its own, then all together
            d = [x if i == which else np.zeros_like(x) for i, x in enumerate(d)]
        fd = (_hals_loss(A + h * d[0], W0 + h * d[1], H0 + h * d[2], T, GW, GH)
              - _hals_loss(A - h * d[0], W0 - h * d[1], H0 - h * d[2], T, GW, GH)) / (2 * h)
        an = np.sum(gA * d[0]) + np.sum(gW * d[1]) + np.sum(gH * d[2])
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (which, fd, an)


def _torch_hals(At, Wt, Ht, T):
    """HALS in the paper's order, written from Eq. (5) with the readings of
    the GPU path (exact block minimiser, normalisation of w_i right after its
    update, compensated in h_i), every product recomputed from the current
    factors; torch's autograd differentiates it."""
    import torch

    k = Wt.shape[1]
    Wc = [Wt[:, i] for i in range(k)]
    Hc = [Ht[i, :] for i in range(k)]
    for _ in range(T):
        for i in range(k):
            Hm = torch.stack(Hc)
            q = Hm @ Hc[i]
            p = At @ Hc[i]
            Wm = torch.stack(Wc, dim=1)
            w = torch.relu(Wc[i] + (p - Wm @ q) / q[i])
            s = torch.linalg.norm(w)
            Wc[i] = w / s
            Hc[i] = Hc[i] * s
        Wm = torch.stack(Wc, dim=1)
        S = Wm.T @ Wm
        R = Wm.T @ At
        for i in range(k):
            Hm = torch.stack(Hc)
            Hc[i] = torch.relu(Hc[i] + (R[i] - S[i] @ Hm) / S[i, i])
    return torch.stack(Wc, dim=1), torch.stack(Hc)


def test_hals_vjp_matches_torch_autograd():
    torch = pytest.importorskip("torch")
    m, n, k, T = 20, 15, 4, 5
    A, W0, H0, GW, GH = _problem(m, n, k, seed=17)
    gA, gW, gH = oracle.hals_unrolled_vjp(A, W0, H0, T, GW, GH)
    At = torch.tensor(A, requires_grad=True)
    Wt = torch.tensor(W0, requires_grad=True)
    Ht = torch.tensor(H0, requires_grad=True)
    W, H = _torch_hals(At, Wt, Ht, T)
    Wo, Ho = oracle.hals_unrolled_forward(A, W0, H0, T)
    assert np.max(np.abs(W.detach().numpy() - Wo)) <= 1e-12
    assert np.max(np.abs(H.detach().numpy() - Ho)) <= 1e-10 * np.abs(Ho).max()
    L = (torch.tensor(GW) * W).sum() + (torch.tensor(GH) * H).sum()
    L.backward()
    for mine, ref in ((gA, At.grad), (gW, Wt.grad), (gH, Ht.grad)):
        ref = ref.numpy()
        assert np.max(np.abs(mine - ref)) <= 1e-9 * np.abs(ref).max()


def test_hals_vjp_sees_clipped_entries():
    """A case where the sweep clips entries to zero: the gradient still
    matches central differences (the clipped entries carry none)."""
    m, n, k, T = 10, 8, 4, 2
    A, W0, H0, GW, GH = _problem(m, n, k, seed=5)
    A = A * (uniform(A.shape, seed=6) > 0.5)          # a sparse A clips entries
    W, H = oracle.hals_unrolled_forward(A, W0, H0, T)
    assert np.sum(W == 0) + np.sum(H == 0) > 0
    gA, gW, gH = oracle.hals_unrolled_vjp(A, W0, H0, T, GW, GH)
    rng = np.random.default_rng(9)
    h = 1e-7
    for _ in range(3):
        d = [rng.standard_normal(x.shape) for x in (A, W0, H0)]
        fd = (_hals_loss(A + h * d[0], W0 + h * d[1], H0 + h * d[2], T, GW, GH)
              - _hals_loss(A - h * d[0], W0 - h * d[1], H0 - h * d[2], T, GW, GH)) / (2 * h)
        an = np.sum(gA * d[0]) + np.sum(gW * d[1]) + np.sum(gH * d[2])
        assert abs(fd - an) <= 1e-5 * max(1.0, abs(an)), (fd, an)


def test_hals_vjp_of_the_objective():
    m, n, k, T = 9, 8, 3, 3
    A, W0, H0, _, _ = _problem(m, n, k, seed=41)
    W, H = oracle.hals_unrolled_forward(A, W0, H0, T)
    Rz = A - W @ H
    gA, gW, gH = oracle.hals_unrolled_vjp(A, W0, H0, T, -2 * Rz @ H.T, -2 * W.T @ Rz)
    gA = gA + 2 * Rz

    def L(A_, W_, H_):
        Wt, Htt = oracle.hals_unrolled_forward(A_, W_, H_, T)
        return float(np.sum((A_ - Wt @ Htt) ** 2))

    rng = np.random.default_rng(1)
    h = 1e-6
    for _ in range(3):
        dA, dW, dH = (rng.standard_normal(x.shape) for x in (A, W0, H0))
        fd = (L(A + h * dA, W0 + h * dW, H0 + h * dH) - L(A - h * dA, W0 - h * dW, H0 - h * dH)) / (2 * h)
        an = np.sum(gA * dA) + np.sum(gW * dW) + np.sum(gH * dH)
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))
