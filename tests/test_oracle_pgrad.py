"""Pins for the projected gradient and the tolerance stop (Section 6.2)."""
import numpy as np

import oracle
from synth import init_factors, planted_dense, uniform


def test_gradients_match_finite_differences():
    m, n, k = 9, 7, 3
    A = planted_dense(m, n, k, seed=3)
    W, H = init_factors(m, n, k, seed=4)
    gW, gH = oracle.gradients(A, W, H)
    f = lambda W_, H_: 0.5 * np.sum((A - W_ @ H_) ** 2)
    h = 1e-6
    rng = np.random.default_rng(1)
    for _ in range(3):
        dW = rng.standard_normal(W.shape)
        dH = rng.standard_normal(H.shape)
        fd = (f(W + h * dW, H + h * dH) - f(W - h * dW, H - h * dH)) / (2 * h)
        assert abs(fd - np.sum(gW * dW) - np.sum(gH * dH)) <= 1e-6 * abs(fd)


def test_projection_rule():
    X = np.array([[0.0, 0.0, 1.0, 2.0]])
    G = np.array([[3.0, -2.0, 5.0, -1.0]])
    # bound entries keep only the negative part: (0, -2, 5, -1)
    assert oracle.projected_gradient_sq(X, G) == 4.0 + 25.0 + 1.0


def test_exact_half_step_is_stationary_in_that_factor():
    """After an exact NNLS update of W for fixed H (ABPP), the projected
    gradient in W vanishes: the KKT conditions of Eq. (7) hold."""
    m, n, k = 40, 30, 5
    A = planted_dense(m, n, k, seed=8)
    _, H = init_factors(m, n, k, seed=9)
    W = oracle.abpp_update_W(oracle.gram_fixed_H(H), oracle.product_AHt(A, H))
    gW, _ = oracle.gradients(A, W, H)
    assert np.sqrt(oracle.projected_gradient_sq(W, gW)) <= 1e-10 * np.abs(gW).max()
    assert (W == 0).any()  # some entries sit at the bound


def test_run_until_stops_where_the_metric_crosses():
    m, n, k = 80, 60, 4
    A = planted_dense(m, n, k, seed=10)
    W0, H0 = init_factors(m, n, k, seed=11)
    _, _, errs, ratios, t = oracle.run_until(A, k, "hals", 200, W0, H0, "pgrad", 1e-2)
    assert t < 200 and ratios[t] <= 1e-2 and min(ratios[1:t]) > 1e-2
    _, _, errs, _, t = oracle.run_until(A, k, "mu", 500, W0, H0, "relerr", 1e-3)
    assert t < 500 and errs[t - 1] - errs[t] < 1e-3 * errs[t - 1]
    assert all(errs[s - 1] - errs[s] >= 1e-3 * errs[s - 1] for s in range(1, t))
