"""FP64 reference gradients of T unrolled MU or HALS iterations.

Test infrastructure only (see the package docstring). The MU forward map is
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

from .nmf import MU_EPS, hals_update_H, hals_update_W


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


# --- HALS (Section 4.2, Eq. (5), readings R2/R3) ---------------------------
#
# One HALS iteration of Algorithm 1, written as a map with explicit
# intermediate values. Column i of the W sweep (i = 1..k in order, newest
# values) sets
#
#     w_i' = max(0, (p_i - sum_{j != i} w_j Q_ji) / Q_ii),   P = A H^T, Q = H H^T
#
# (the update w_i + (p_i - W q_i)/Q_ii written without the w_i terms, which
# cancel), skipped when Q_ii = 0. The columns are then normalised,
# W_n = W' diag(1/s), s_i = ||w_i'||, with H_c = diag(s) H compensating
# (R3: the same map as normalising each column inside the sweep). The H
# sweep is the same rule on the rows of H_c with S = W_n^T W_n and
# R = W_n^T A. The reverse of one sweep column i, with g the gradient with
# respect to the sweep's current values and M = [w_i' > 0]:
#
#     d = M * g_i / Q_ii          (gradient of the numerator; dL/dp_i = d)
#     g_j -= Q_ji d, dL/dQ_ji -= <w_j, d>   for j != i (w_j: value at that time)
#     dL/dQ_ii -= <w_i', d>                 (N / Q_ii = w_i' where M holds)
#     g_i = 0                               (w_i' does not depend on the old w_i)


def _sweep(X, P, G):
    """The HALS sweep on the rows of X (rows x k) with product P (rows x k)
    and Gram G (k x k): column i = 0..k-1 in order."""
    X = X.copy()
    k = G.shape[0]
    for i in range(k):
        if G[i, i] > 0:
            num = P[:, i] - sum(X[:, j] * G[j, i] for j in range(k) if j != i)
            X[:, i] = np.maximum(0.0, num / G[i, i])
    return X


def _sweep_vjp(X_old, X_new, G, gX_new):
    """Reverse of _sweep: (dL/dX_old, dL/dP, dL/dG) from dL/dX_new."""
    g = np.array(gX_new, dtype=np.float64, copy=True)
    k = G.shape[0]
    gP = np.zeros_like(g)
    gG = np.zeros((k, k))
    for i in reversed(range(k)):
        if not G[i, i] > 0:
            continue                      # column skipped: the identity
        d = np.where(X_new[:, i] > 0, g[:, i] / G[i, i], 0.0)
        gP[:, i] = d
        for j in range(k):
            if j == i:
                continue
            xj = X_new[:, j] if j < i else X_old[:, j]   # value when column i ran
            g[:, j] -= G[j, i] * d
            gG[j, i] -= xj @ d
        gG[i, i] -= X_new[:, i] @ d
        g[:, i] = 0.0
    return g, gP, gG


def _hals_states(A, W, H):
    """One HALS iteration from (W, H) with its intermediate values."""
    Q = H @ H.T
    P = A @ H.T
    Wp = _sweep(W, P, Q)
    s = np.linalg.norm(Wp, axis=0)
    pos = s > 0
    Wn = Wp.copy()
    Wn[:, pos] /= s[pos]
    Hc = H.copy()
    Hc[pos, :] *= s[pos, None]
    S = Wn.T @ Wn
    R = Wn.T @ A
    Hn = _sweep(Hc.T, R.T, S).T
    return dict(W=W, H=H, Q=Q, Wp=Wp, s=s, pos=pos, Wn=Wn, Hc=Hc, S=S, Hn=Hn)


def hals_unrolled_forward(A, W0, H0, T: int):
    """T HALS iterations from (W0, H0) with Algorithm 1's HALS steps as the
    oracle takes them (hals_update_W then hals_update_H, normalisation inside
    the sweep). Returns (W_T, H_T)."""
    A = _f64(A)
    W = _f64(W0).copy()
    H = _f64(H0).copy()
    for _ in range(T):
        Q = H @ H.T
        P = A @ H.T
        W, H = hals_update_W(W, H, Q, P)
        H = hals_update_H(H, W.T @ W, W.T @ A)
    return W, H


def hals_unrolled_vjp(A, W0, H0, T: int, gW_T, gH_T):
    """(dL/dA, dL/dW0, dL/dH0) of T HALS iterations for the loss whose
    gradients at (W_T, H_T) are gW_T (m x k) and gH_T (k x n); the map is
    piecewise smooth (the max and the skipped columns), and the gradient is
    that of the piece the forward pass is on."""
    A = _f64(A)
    W = _f64(W0).copy()
    H = _f64(H0).copy()
    states = []
    for _ in range(T):
        st = _hals_states(A, W, H)
        states.append(st)
        W, H = st["Wn"], st["Hn"]
    gA = np.zeros_like(A)
    gW = _f64(gW_T).copy()
    gH = _f64(gH_T).copy()
    for st in reversed(states):
        Wn, Hc, s, pos = st["Wn"], st["Hc"], st["s"], st["pos"]
        # H sweep on the rows of Hc^T with R^T = A^T Wn and S = Wn^T Wn
        gHc_t, gR_t, gS = _sweep_vjp(Hc.T, st["Hn"].T, st["S"], gH.T)
        gA += Wn @ gR_t.T
        gWn = gW + A @ gR_t + Wn @ (gS + gS.T)
        # normalisation: Wn = Wp / s, Hc = s H (columns with s > 0)
        gHc = gHc_t.T
        gs = np.zeros_like(s)
        gs[pos] = (-np.sum(gWn[:, pos] * Wn[:, pos], axis=0) / s[pos]
                   + np.sum(gHc[pos, :] * st["H"][pos, :], axis=1))
        gWp = gWn.copy()
        gWp[:, pos] = gWn[:, pos] / s[pos] + gs[pos] * Wn[:, pos]
        gH_prev = gHc.copy()
        gH_prev[pos, :] = s[pos, None] * gHc[pos, :]
        # W sweep with P = A H^T and Q = H H^T
        gW_prev, gP, gQ = _sweep_vjp(st["W"], st["Wp"], st["Q"], gWp)
        gA += gP @ st["H"]
        gH_prev += gP.T @ A + (gQ + gQ.T) @ st["H"]
        gW, gH = gW_prev, gH_prev
    return gA, gW, gH
