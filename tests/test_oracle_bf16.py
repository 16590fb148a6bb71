"""Pins for the oracle's bfloat16 rounding and its reduced-precision
product variant (the precision extension of the dense products)."""
import numpy as np
import pytest

import oracle
from synth import init_factors, planted_dense, uniform


def test_round_bf16_hand_cases():
    one = 1.0
    ulp = 2.0 ** -7          # spacing of bfloat16 values in [1, 2)
    cases = [
        (one, one),
        (one + ulp / 2, one),                      # tie, even neighbour below
        (one + 3 * ulp / 2, one + 2 * ulp),        # tie, even neighbour above
        (one + ulp / 2 + 2.0 ** -20, one + ulp),   # just above the tie
        (one + ulp / 2 - 2.0 ** -20, one),         # just below the tie
        (-(one + 3 * ulp / 2), -(one + 2 * ulp)),  # sign is kept
        (0.0, 0.0),
        (3.0, 3.0),
        (2.0 ** -130, 2.0 ** -130),                # float32 subnormal, 7 bits enough
    ]
    for x, want in cases:
        assert oracle.round_bf16(np.array([x]))[0] == want, x


def test_round_bf16_matches_torch_conversion():
    """torch's float32 -> bfloat16 conversion rounds to nearest even: an
    independent implementation of the same rounding."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(3)
    x = (rng.standard_normal(200000) * np.exp(rng.uniform(-20, 20, 200000))).astype(np.float32)
    # exact ties: float32 values whose low 16 bits are 0x8000
    ties = (rng.integers(0x00800000, 0x7f000000, 5000, dtype=np.uint64) & ~np.uint64(0xFFFF)) \
        | np.uint64(0x8000)
    x = np.concatenate([x, ties.astype(np.uint32).view(np.float32)])
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy().astype(np.float64)
    got = oracle.round_bf16(x)
    assert np.array_equal(got, want)


def test_round_bf16_error_bound():
    x = uniform((100000,), seed=11) * 1e3 + 1e-3
    r = oracle.round_bf16(x)
    assert np.all(np.abs(r - x) <= 2.0 ** -8 * np.abs(x))


@pytest.mark.parametrize("algo", ["mu", "hals"])
def test_bf16_products_only_round_the_product_operand(algo):
    """With an initial H whose entries are bfloat16 values, the first product
    A H^T is the same in both variants, so the first W update must agree
    exactly; later products differ by the rounding of W and H only."""
    m, n, k = 60, 40, 5
    A = planted_dense(m, n, k, seed=5)
    W0, H0 = init_factors(m, n, k, seed=6)
    H0 = oracle.round_bf16(H0)
    Wa, _, _ = oracle.run(A, k, algo, 1, W0, H0, track_error=False)
    Wb, _, _ = oracle.run(A, k, algo, 1, W0, H0, track_error=False, bf16_products=True)
    # the W step saw identical inputs; the H step of iteration 1 rounds W
    Q = oracle.gram_fixed_H(H0)
    P = oracle.product_AHt(A, H0)
    W1 = oracle.mu_update_W(W0, Q, P) if algo == "mu" else oracle.hals_update_W(W0, H0, Q, P)[0]
    assert np.array_equal(Wa, W1) and np.array_equal(Wb, W1)
    _, Ha, ea = oracle.run(A, k, algo, 3, W0, H0)
    _, Hb, eb = oracle.run(A, k, algo, 3, W0, H0, bf16_products=True)
    assert not np.array_equal(Ha, Hb)
    # bfloat16 operands move the error by a small relative amount only
    assert np.max(np.abs(np.array(ea) - np.array(eb)) / np.array(ea)) < 1e-2


def test_hals_k100_trajectory_is_sensitive_to_gram_rounding():
    """The bf16 run test's HALS case (k = 100 on a 500 x 400 planted matrix,
    4 iterations) keeps many entries at the projection boundary, so its
    objective trajectory is ill-conditioned: perturbing only the oracle's
    Grams by relative amounts of 2^-24 (half a float32 ulp, symmetric noise)
    moves the trajectory by more than 1e-4 in some draws. The GPU run, which
    rounds its Grams, products and factors to float32, is therefore held to
    5e-4 on that case (and to 1e-4 at the first iteration)."""
    from oracle import nmf as on

    m, n, k, iters = 500, 400, 100, 4
    A64 = oracle.round_bf16(planted_dense(m, n, k, seed=31).astype(np.float32).astype(np.float64))
    W0, H0 = init_factors(m, n, k, seed=32)
    W0 = W0.astype(np.float32).astype(np.float64)
    H0 = H0.astype(np.float32).astype(np.float64)
    _, _, base = oracle.run(A64, k, "hals", iters, W0, H0, bf16_products=True)
    rng = np.random.default_rng(0)
    fH, fW = on.gram_fixed_H, on.gram_fixed_W

    def noisy(f):
        def g(X):
            G = f(X)
            E = rng.standard_normal(G.shape) * 2.0 ** -24
            return G * (1 + (E + E.T) / 2)
        return g

    spread = []
    try:
        on.gram_fixed_H, on.gram_fixed_W = noisy(fH), noisy(fW)
        for _ in range(6):
            _, _, e = oracle.run(A64, k, "hals", iters, W0, H0, bf16_products=True)
            spread.append(max(abs(a - b) / b for a, b in zip(e, base)))
    finally:
        on.gram_fixed_H, on.gram_fixed_W = fH, fW
    assert max(spread) > 1e-4          # a 1e-4 bar would sit inside the rounding spread
    assert max(spread) < 5e-4          # the bar used on the GPU is above it
