"""Pins for the oracle's FP8 E4M3 rounding, its per-column scale rule and its
FP8 product variant (the precision extension of the dense products)."""
import numpy as np
import pytest

import oracle
from synth import init_factors, planted_dense, uniform


def e4m3_values():
    """All finite non-negative E4M3 values from the format's definition:
    f 2^-9 for exponent field 0, (8 + f) 2^(e - 10) otherwise, the all-ones
    pattern excluded (NaN)."""
    vals = []
    for e in range(16):
        for f in range(8):
            if e == 15 and f == 7:
                continue
            vals.append(f * 2.0 ** -9 if e == 0 else (8 + f) * 2.0 ** (e - 10))
    return np.array(vals)


def test_e4m3_grid_is_fixed_and_ties_go_even():
    v = e4m3_values()
    assert v.max() == oracle.FP8_E4M3_MAX and len(v) == 127
    # every representable value rounds to itself, with either sign
    assert np.array_equal(oracle.round_fp8_e4m3(v), v)
    assert np.array_equal(oracle.round_fp8_e4m3(-v), -v)
    # midpoints go to the neighbour whose code (index on the grid) is even;
    # points just off the midpoint go to the nearer neighbour
    lo, hi = v[:-1], v[1:]
    mid = (lo + hi) / 2
    even = np.where(np.arange(len(lo)) % 2 == 0, lo, hi)
    assert np.array_equal(oracle.round_fp8_e4m3(mid), even)
    d = (hi - lo) * 1e-3
    assert np.array_equal(oracle.round_fp8_e4m3(mid - d), lo)
    assert np.array_equal(oracle.round_fp8_e4m3(mid + d), hi)


def test_round_fp8_saturates():
    x = np.array([448.0, 450.0, 463.9, 464.0, 1e6, -1e6])
    assert np.array_equal(oracle.round_fp8_e4m3(x), [448, 448, 448, 448, 448, -448])


def test_round_fp8_matches_torch_conversion():
    """torch's float32 -> float8_e4m3fn conversion rounds to nearest even:
    an independent implementation of the same rounding (inputs kept below
    464, where torch would produce NaN instead of saturating)."""
    torch = pytest.importorskip("torch")
    if not hasattr(torch, "float8_e4m3fn"):
        pytest.skip("no float8_e4m3fn in this torch")
    rng = np.random.default_rng(5)
    x = rng.uniform(0, 1, 300000) * np.exp2(rng.uniform(-14, 9, 300000))
    x = np.concatenate([x, -x[:1000], [0.0]])
    x = x[np.abs(x) < 464].astype(np.float32)
    v = e4m3_values()
    x = np.concatenate([x, ((v[:-1] + v[1:]) / 2).astype(np.float32)])
    want = torch.from_numpy(x).to(torch.float8_e4m3fn).to(torch.float32).numpy()
    assert np.array_equal(oracle.round_fp8_e4m3(x), want.astype(np.float64))


def test_round_fp8_error_bound():
    # normal range: relative error at most half a spacing, 2^-4
    x = uniform((100000,), seed=13) * 400 + 2.0 ** -6
    r = oracle.round_fp8_e4m3(x)
    assert np.all(np.abs(r - x) <= 2.0 ** -4 * np.abs(x))
    # subnormal range: absolute error at most 2^-10
    y = uniform((10000,), seed=14) * 2.0 ** -6
    assert np.all(np.abs(oracle.round_fp8_e4m3(y) - y) <= 2.0 ** -10)


def test_fp8_column_scales_rule():
    rng = np.random.default_rng(7)
    X = rng.uniform(0, 1, (50, 9)) * np.exp2(rng.uniform(-20, 20, 9))
    X[:, 3] = 0.0
    X[0, 4] = 448.0 * 2.0 ** -5     # max exactly 448 times a power of two
    X[1:, 4] = 0.0
    X[0, 5] = 448.0 * 2.0 ** 3 * (1 + 2.0 ** -20)   # just past: next power
    X[1:, 5] = 0.0
    s = oracle.fp8_column_scales(X, 1)
    mx = np.abs(X).max(axis=0)
    p = np.log2(s)
    assert np.array_equal(p, np.round(p))           # powers of two
    assert s[3] == 1.0
    assert s[4] == 2.0 ** -5 and s[5] == 2.0 ** 4
    nz = mx > 0
    assert np.all(mx[nz] / s[nz] <= 448.0)
    assert np.all(mx[nz] / s[nz] > 224.0)           # the smallest such power
    # the same rule along the other axis
    assert np.array_equal(oracle.fp8_column_scales(X.T, 0), s)


def test_round_fp8_scaled_is_exact_on_e4m3_columns():
    """A column whose entries are E4M3 values times a power of two, with its
    largest entry in (224, 448] after the scale, passes unchanged."""
    v = e4m3_values()
    rng = np.random.default_rng(8)
    X = rng.choice(v[v > 0], size=(40, 6))
    X[0, :] = 448.0
    X = X * np.exp2(np.arange(6) * 3 - 9)
    assert np.array_equal(oracle.round_fp8_scaled(X, 1), X)
    assert np.array_equal(oracle.round_fp8_scaled(X.T, 0), X.T)


def test_round_fp8_scaled_relative_error():
    """Every entry within 2^-4 relative of its value once scaled into the
    normal range, or within half the subnormal spacing times the scale."""
    X = uniform((300, 8), seed=15) * np.exp2(np.arange(8) * 4 - 16)
    R = oracle.round_fp8_scaled(X, 1)
    s = oracle.fp8_column_scales(X, 1)
    bound = np.maximum(2.0 ** -4 * np.abs(X), 2.0 ** -10 * s)
    assert np.all(np.abs(R - X) <= bound)


@pytest.mark.parametrize("algo", ["mu", "hals"])
def test_fp8_products_only_round_the_product_operand(algo):
    """The FP8 variant changes the two large products and nothing else: with
    an H that passes the scaled rounding unchanged, the first W update is the
    unrounded one; later the rounding of W and H moves the error by a few
    per cent at most."""
    m, n, k = 60, 40, 5
    A = oracle.round_fp8_e4m3(planted_dense(m, n, k, seed=5))
    W0, H0 = init_factors(m, n, k, seed=6)
    H0 = oracle.round_fp8_scaled(H0, 0)
    assert np.array_equal(oracle.round_fp8_scaled(H0, 0), H0)
    Wa, _, _ = oracle.run(A, k, algo, 1, W0, H0, track_error=False)
    Wb, _, _ = oracle.run(A, k, algo, 1, W0, H0, track_error=False, fp8_products=True)
    Q = oracle.gram_fixed_H(H0)
    P = oracle.product_AHt(A, H0)
    W1 = oracle.mu_update_W(W0, Q, P) if algo == "mu" else oracle.hals_update_W(W0, H0, Q, P)[0]
    assert np.array_equal(Wa, W1) and np.array_equal(Wb, W1)
    _, Ha, ea = oracle.run(A, k, algo, 3, W0, H0)
    _, Hb, eb = oracle.run(A, k, algo, 3, W0, H0, fp8_products=True)
    assert not np.array_equal(Ha, Hb)
    assert np.max(np.abs(np.array(ea) - np.array(eb)) / np.array(ea)) < 5e-2


def test_fp8_and_bf16_variants_are_exclusive():
    A = uniform((10, 8), seed=1)
    W0, H0 = init_factors(10, 8, 2, seed=2)
    with pytest.raises(ValueError):
        oracle.run(A, 2, "mu", 1, W0, H0, bf16_products=True, fp8_products=True)
