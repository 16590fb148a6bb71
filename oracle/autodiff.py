"""FP64 reference gradient of T unrolled multiplicative-update iterations.

Test infrastructure only (see the package docstring). The forward map is
Algorithm 1 with the MU rule of Section 4.1, Eq. (3), T times:

    W_{t+1} = W_t * P_t / D_t,    P_t = A H_t^T,       D_t = W_t Q_t + eps,
                                  Q_t = H_t H_t^T
    H_{t+1} = H_t * R_t / E_t,    R_t = W_{t+1}^T A,   E_t = S_t H_t + eps,
                                  S_t = W_{t+1}^T W_{t+1}

(* and / elementwise). ``mu_unrolled_vjp`` returns the gradient of a scalar
loss L(W_T, H_T) with respect to A, W_0 and H_0, given dL/dW_T and dL/dH_T,
by running the iterations backwards. For one multiplicative step
Y = X * N / (X G + eps) with N = num and G symmetric, the chain rule gives,
with gY = dL/dY and D = X G + eps:

    dL/dN = gY * X / D
    dL/dD = -gY * Y / D
    dL/dX = gY * N / D + (dL/dD) G
    dL/dG = X^T (dL/dD)

and then the products and Grams that formed N and G pass the gradients on
to A and to the other factor. Everything is written out on the k x n / m x k
matrices in the paper's orientation; no automatic differentiation is used.
"""
from __future__ import annotations

import numpy as np

from .nmf import MU_EPS


def _f64(X):
    return np.asarray(X, dtype=np.float64)


def mu_unrolled_forward(A, W0, H0, T: int, eps: float = MU_EPS):
    """T MU iterations from (W0, H0); returns (W_T, H_T, states) with
    states[t] = (W_t, H_t) for t = 0..T."""
    A = _f64(A)
    W = _f64(W0).copy()
    H = _f64(H0).copy()
    states = [(W, H)]
    for _ in range(T):
        P = A @ H.T
        D = W @ (H @ H.T) + eps
        W = W * P / D
        R = W.T @ A
        E = (W.T @ W) @ H + eps
        H = H * R / E
        states.append((W, H))
    return W, H, states


def mu_unrolled_vjp(A, W0, H0, T: int, gW_T, gH_T, eps: float = MU_EPS):
    """(dL/dA, dL/dW0, dL/dH0) for the loss whose gradients at (W_T, H_T)
    are gW_T (m x k) and gH_T (k x n)."""
    A = _f64(A)
    _, _, states = mu_unrolled_forward(A, W0, H0, T, eps)
    gA = np.zeros_like(A)
    gW = _f64(gW_T).copy()
    gH = _f64(gH_T).copy()
    for t in range(T - 1, -1, -1):
        W, H = states[t]          # inputs of iteration t
        Wn, Hn = states[t + 1]    # outputs of iteration t
        # H step: Hn = H * R / E, R = Wn^T A, E = S H + eps, S = Wn^T Wn.
        R = Wn.T @ A
        S = Wn.T @ Wn
        E = S @ H + eps
        gR = gH * H / E
        gE = -gH * Hn / E
        gH_prev = gH * R / E + S.T @ gE      # E = S H: dL/dH += S^T dL/dE
        gS = gE @ H.T                        # dL/dS = dL/dE H^T
        gA += Wn @ gR                        # R = Wn^T A
        gW = gW + A @ gR.T + Wn @ (gS + gS.T)
        # W step: Wn = W * P / D, P = A H^T, D = W Q + eps, Q = H H^T.
        P = A @ H.T
        Q = H @ H.T
        D = W @ Q + eps
        gP = gW * W / D
        gD = -gW * Wn / D
        gW_prev = gW * P / D + gD @ Q.T      # D = W Q: dL/dW += dL/dD Q^T
        gQ = W.T @ gD                        # dL/dQ = W^T dL/dD
        gA += gP @ H                         # P = A H^T: dL/dA += dL/dP H
        gH_prev = gH_prev + gP.T @ A + (gQ + gQ.T) @ H
        gW, gH = gW_prev, gH_prev
    return gA, gW, gH
