"""Precision extension: dense A stored in FP8 E4M3, the two large products on
the FP8 matrix cores (factor operand scaled per rank column by a power of
two and rounded to E4M3, float accumulation), everything else float32.

Parity is against the oracle's fp8_products variant on the same E4M3 values
of A (the oracle scales and rounds the factor operand with its own code and
multiplies exactly in float64), so what remains is float32 accumulation. The
error of the reduced-precision method itself, against the plain FP64 oracle,
is printed beside it.
"""
import numpy as np
import pytest

import oracle
import paper_1609_09154_amd as nmf
from synth import init_factors, planted_dense, uniform
from tests.gpu_util import U32, gamma, host, rel_diff, step, to_dev, torch_dev

pytestmark = pytest.mark.gpu


def fp8_dev(A32):
    """A on the device as float8_e4m3fn (converted on the host) and the
    float64 values that tensor holds (the oracle's input)."""
    import torch

    A8 = torch.from_numpy(np.ascontiguousarray(A32, dtype=np.float32)).to(torch.float8_e4m3fn)
    return A8.to(torch_dev()), A8.float().numpy().astype(np.float64)


# n is the row pitch of A: a multiple of 16. The shapes cover M and K tails
# (K not a multiple of 128), one column tile up to the full 128 columns, and
# factor columns whose magnitudes differ by many binades.
SHAPES = [(1, 16, 1), (300, 1008, 10), (777, 528, 50), (256, 4096, 100), (130, 2000, 128),
          (64, 80, 16), (2049, 144, 33)]


# Accumulation model of the FP8 matrix-core product, measured through
# nmf_dense_AF with designed exact inputs: the products of each group of 8
# consecutive K values are summed on a grid of 2^(E - 13), E the exponent of
# the group's largest |product| (1 + 2^-13 is kept, 1 + 2^-14 dropped;
# 2^16 + 2^3 kept, 2^16 + 2^2 dropped); group sums and the running float32
# accumulator are then added with float32 rounding (2^16 + 2^-7 exact across
# groups and across K steps). Whether the grid step truncates or rounds was
# not resolved, so the bound below charges each term a whole grid step.
FP8_GROUP = 8
FP8_GROUP_BITS = 13


def fp8_product_bound(X, Y, row_block=16):
    """Elementwise bound on |computed - exact| for D = X Y (X r x K, Y K x c,
    float64 values of the E4M3 operands, Y's column scales included):
    sum over groups of 8 |max product| 2^-13, plus gamma_K float32 for the
    accumulation of the group sums."""
    r, K = X.shape
    G = -(-K // FP8_GROUP)
    pad = G * FP8_GROUP - K
    Xp = np.pad(np.abs(X), ((0, 0), (0, pad))).reshape(r, G, FP8_GROUP)
    Yp = np.pad(np.abs(Y), ((0, pad), (0, 0))).reshape(G, FP8_GROUP, -1)
    out = np.empty((r, Y.shape[1]))
    for i in range(0, r, row_block):
        prod = Xp[i:i + row_block, :, :, None] * Yp[None]       # rows, G, 8, c
        gmax = prod.max(axis=2)                                  # rows, G, c
        out[i:i + row_block] = FP8_GROUP * 2.0 ** -FP8_GROUP_BITS * gmax.sum(axis=1)
    return out + gamma(G + 2, U32) * (np.abs(X) @ np.abs(Y))


def spread_factor(rows, k, seed):
    """U(0, 1) columns scaled by 2^(-12 .. 12): each column needs its own
    power-of-two scale to stay inside the E4M3 range."""
    F = uniform((rows, k), seed=seed)
    return (F * np.exp2(np.linspace(-12, 12, k))).astype(np.float32)


def assert_within(got, ref, bound, what):
    err = np.abs(got.astype(np.float64) - ref)
    worst = float(np.max(err / (bound + 1e-300))) if err.size else 0.0
    print("%s: worst error / bound %.3g" % (what, worst))
    assert worst <= 1.0, "%s: error exceeds the FP8 accumulation bound by %.3g" % (what, worst)


@pytest.mark.parametrize("m,n,k", SHAPES)
def test_fp8_AF(m, n, k):
    A32 = uniform((m, n), seed=m + n).astype(np.float32)
    F = spread_factor(n, k, k + 7)
    A8, A64 = fp8_dev(A32)
    step("fp8 A F %dx%d k=%d" % (m, n, k))
    P = host(nmf.nmf_dense_AF(A8, to_dev(F, np.float32)))
    Fr = oracle.round_fp8_scaled(F, 1)
    ref = oracle.product_AHt(A64, Fr.T)
    assert_within(P, ref, fp8_product_bound(A64, Fr), "fp8 A F")
    # precision of the method: the factor's rounding, at most 2^-4 per normal
    # entry (the scale keeps every column's largest entries normal)
    exact = A64 @ F.astype(np.float64)
    print("fp8 A F %dx%d k=%d: max rel diff to the unrounded product %.3e"
          % (m, n, k, rel_diff(P, exact)))
    assert rel_diff(P, exact) <= 2.0 ** -4 + 1e-6


@pytest.mark.parametrize("m,n,k", SHAPES)
def test_fp8_AtF(m, n, k):
    A32 = uniform((m, n), seed=3 * m + n).astype(np.float32)
    F = spread_factor(m, k, k + 9)
    A8, A64 = fp8_dev(A32)
    step("fp8 A^T F %dx%d k=%d" % (m, n, k))
    R = host(nmf.nmf_dense_AtF(A8, to_dev(F, np.float32)))
    Fr = oracle.round_fp8_scaled(F, 1)
    ref = oracle.product_WtA(A64, Fr).T
    assert_within(R, ref, fp8_product_bound(A64.T, Fr), "fp8 A^T F")


def unit_binade_e4m3(shape, seed):
    """Random E4M3 values in [1, 2): 1 + f/8."""
    rng = np.random.default_rng(seed)
    return 1.0 + rng.integers(0, 8, size=shape) / 8.0


@pytest.mark.parametrize("m,n,k", SHAPES)
def test_fp8_products_bit_exact_on_unit_binade(m, n, k):
    """A and F with E4M3 values in [1, 2): every product is a multiple of a
    common power of two well inside each group's 13-bit grid and every
    partial sum fits float32's 24 bits (K <= 4096), so the hardware sum is
    exact and both products must equal the oracle bit for bit (F's column
    scale 2^-7 or 2^-8 is a power of two)."""
    A64 = unit_binade_e4m3((m, n), m + 5 * n)
    A8, A64b = fp8_dev(A64.astype(np.float32))
    assert np.array_equal(A64, A64b)
    F = unit_binade_e4m3((n, k), k + 1).astype(np.float32)
    G = unit_binade_e4m3((m, k), k + 2).astype(np.float32)
    step("fp8 bit-exact %dx%d k=%d" % (m, n, k))
    P = host(nmf.nmf_dense_AF(A8, to_dev(F, np.float32)))
    R = host(nmf.nmf_dense_AtF(A8, to_dev(G, np.float32)))
    assert np.array_equal(oracle.round_fp8_scaled(F, 1), F)
    refP = oracle.product_AHt(A64, F.T.astype(np.float64))
    refR = oracle.product_WtA(A64, G.astype(np.float64)).T
    assert np.array_equal(P.astype(np.float64), refP)
    assert np.array_equal(R.astype(np.float64), refR)


def test_fp8_zero_and_single_column_factor():
    """An all-zero rank column takes scale 1 and gives a zero output column;
    a column with one nonzero entry is reproduced exactly when that entry
    is representable."""
    m, n, k = 200, 512, 3
    A32 = uniform((m, n), seed=41).astype(np.float32)
    A8, A64 = fp8_dev(A32)
    F = np.zeros((n, k), dtype=np.float32)
    F[7, 1] = 3.0 * 2.0 ** 20
    F[:, 2] = uniform((n,), seed=42).astype(np.float32)
    step("fp8 A F zero column")
    P = host(nmf.nmf_dense_AF(A8, to_dev(F, np.float32)))
    assert np.all(P[:, 0] == 0.0)
    assert np.array_equal(P[:, 1], (A64[:, 7] * 3.0 * 2.0 ** 20).astype(np.float32))


def test_fp8_rejects_unaligned_row_pitch():
    import torch

    A = torch.zeros((16, 24), dtype=torch.float8_e4m3fn, device=torch_dev())
    F = torch.zeros((24, 4), dtype=torch.float32, device=torch_dev())
    with pytest.raises(nmf.NMFError):
        nmf.nmf_dense_AF(A, F)


def test_fp8_relerr_matches_oracle():
    m, n, k = 333, 272, 12
    A32 = planted_dense(m, n, k, seed=21).astype(np.float32)
    A8, A64 = fp8_dev(A32)
    W, H = init_factors(m, n, k, seed=22)
    W32, H32 = W.astype(np.float32), H.astype(np.float32)
    step("fp8 relerr")
    got = nmf.nmf_dense_relerr(A8, to_dev(W32, np.float32), to_dev(H32.T, np.float32))
    ref = oracle.relative_error(A64, W32.astype(np.float64), H32.astype(np.float64))
    assert abs(got - ref) <= 1e-5 * ref


def test_fp8_check_input():
    """check_input decodes every stored byte: all non-negative finite E4M3
    codes pass, the NaN pattern and a negative value are flagged."""
    import torch

    m, n, k = 64, 160, 4
    codes = np.arange(m * n) % 0x7f           # every non-negative finite code
    A8 = torch.from_numpy(codes.astype(np.uint8).reshape(m, n)).view(torch.float8_e4m3fn)
    W0, H0 = init_factors(m, n, k, seed=3)
    W = to_dev(W0.astype(np.float32), np.float32)
    H = to_dev(H0.astype(np.float32), np.float32)
    step("fp8 check_input")
    nmf.nmf_dense(A8.to(torch_dev()), W, H, algo="mu", iters=1, objective=False,
                  check_input=True)
    # the NaN pattern and a negative value are flagged
    for bad in (0x7f, 0xb8):
        c = codes.astype(np.uint8).reshape(m, n).copy()
        c[5, 9] = bad
        Ab = torch.from_numpy(c).view(torch.float8_e4m3fn).to(torch_dev())
        with pytest.raises(nmf.NMFError):
            nmf.nmf_dense(Ab, W, H, algo="mu", iters=1, objective=False, check_input=True)


def nnls_kkt_excess(X, Gram, Prod, bound):
    """Largest violation, relative to bound, of the KKT conditions of
    min_{X >= 0} 1/2 tr(X Gram X^T) - tr(X Prod^T) for the computed X:
    g = X Gram - Prod must vanish where X > 0 and be >= 0 where X = 0."""
    g = X @ Gram - Prod
    viol = np.where(X > 0, np.abs(g), np.maximum(-g, 0.0))
    return float(np.max(viol / bound))


def abpp_step_kkt(A64, W, H, W1, H1):
    """ABPP solves each half-step exactly, so each half-step of the GPU is
    checked on its own against the oracle's exact FP8 products of the same
    inputs: W1 for (H H^T, A q(H)^T), H1 for (W1^T W1, q(W1)^T A), q the
    scaled E4M3 rounding. The allowance is the FP8 product bound plus float32
    slack for the Gram (accumulated in double, stored in float) and for
    storing the solution in float32 (k u |X| |Gram| each)."""
    k = W.shape[1]
    Hq = oracle.round_fp8_scaled(H, 0)
    Q = H @ H.T
    slackW = 4 * k * U32 * (np.abs(W1) @ np.abs(Q))
    bW = fp8_product_bound(A64, Hq.T) + slackW + 1e-300
    eW = nnls_kkt_excess(W1, Q, A64 @ Hq.T, bW)
    Wq = oracle.round_fp8_scaled(W1, 1)
    S = W1.T @ W1
    Ht1 = H1.T
    slackH = 4 * k * U32 * (np.abs(Ht1) @ np.abs(S))
    bH = fp8_product_bound(A64.T, Wq) + slackH + 1e-300
    eH = nnls_kkt_excess(Ht1, S, A64.T @ Wq, bH)
    return max(eW, eH)


@pytest.mark.parametrize("algo,k,iters", [("hals", 16, 10), ("mu", 16, 10), ("abpp", 10, 6),
                                          ("hals", 100, 4)])
def test_fp8_runs_match_oracle(algo, k, iters):
    """Step parity: every iteration, started from the GPU's own current
    factors, against one oracle iteration (fp8_products) from the same
    factors. Rounding the factor operand to a 3-bit fraction is
    discontinuous, so two long runs drift apart through rare rounding flips
    as soon as the stored factors differ in float32's last bits; one step
    from identical factors leaves float accumulation and the FP8 group
    accumulation as the only differences.

    MU and HALS: the relative error after the step may differ by at most
    2^-10 (absolute), the worst-case relative error of an FP8 product of
    nonnegative operands (8 terms of a group, each within 2^-13 of the
    group's largest): neither update applies an inverse of the Gram, so a
    product perturbation moves W H, and the residual, by an amount of that
    order relative to ||A||. ABPP applies one, so its steps are checked
    through the KKT conditions instead (abpp_step_kkt). The plain FP64
    trajectory and one GPU run of all iterations are printed beside it."""
    import torch

    m, n = 500, 400
    A32 = planted_dense(m, n, k, seed=31).astype(np.float32)
    A8, A64 = fp8_dev(A32)
    W0, H0 = init_factors(m, n, k, seed=32)
    W0, H0 = W0.astype(np.float32), H0.astype(np.float32)
    step("fp8 run %s k=%d" % (algo, k))
    Wd, Hd = to_dev(W0, np.float32), to_dev(H0, np.float32)
    e_full, _ = nmf.nmf_dense(A8, Wd, Hd, algo=algo, iters=iters, objective=True)
    W, H = W0, H0
    e_chain = [e_full[0]]
    worst = 0.0   # largest step check relative to its allowance
    for t in range(iters):
        Wd, Hd = to_dev(W, np.float32), to_dev(H, np.float32)
        e, _ = nmf.nmf_dense(A8, Wd, Hd, algo=algo, iters=1, objective=True)
        torch.cuda.synchronize()
        W1, H1 = host(Wd).astype(np.float64), host(Hd).astype(np.float64)
        if algo == "abpp":
            r = abpp_step_kkt(A64, W.astype(np.float64), H.astype(np.float64), W1, H1)
        else:
            _, _, e_q = oracle.run(A64, k, algo, 1, W.astype(np.float64), H.astype(np.float64),
                                   fp8_products=True)
            r = abs(e[1] - e_q[1]) / 2.0 ** -10
        print("  step %d: check / allowance %.3g" % (t, r))
        worst = max(worst, r)
        e_chain.append(e[1])
        W, H = host(Wd), host(Hd)
    _, _, e_x = oracle.run(A64, k, algo, iters, W0, H0)
    print("fp8 %s k=%d: rel err per GPU step %s\n  one GPU run %s\n  oracle(fp64) %s\n"
          "  worst step check / allowance %.2e; chained steps vs one run %.2e; "
          "fp8 vs fp64 at the end %.2e"
          % (algo, k, e_chain, e_full, e_x, worst, rel_diff(e_chain, e_full),
             (e_chain[-1] - e_x[-1]) / e_x[-1]))
    assert worst <= 1.0
