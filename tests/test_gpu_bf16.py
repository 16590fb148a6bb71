"""Precision extension: dense A stored in bfloat16, the two large products on
the BF16 matrix cores (factor operand rounded to bfloat16, float
accumulation), everything else float32.

Parity is against the oracle's bf16_products variant on the same bfloat16
values of A (the oracle rounds the factor operand with its own rounding and
multiplies exactly in float64), so what remains is float32 accumulation. The
error of the reduced-precision method itself, against the plain FP64 oracle,
is printed beside it.
"""
import numpy as np
import pytest

import oracle
import paper_1609_09154_amd as nmf
from synth import init_factors, planted_dense, uniform
from tests import parity_bars
from tests.gpu_util import U32, assert_gemm_bound, host, rel_diff, step, to_dev, torch_dev

pytestmark = pytest.mark.gpu


def bf16_dev(A32):
    """A on the device as bfloat16 and, on the host, the float64 values that
    tensor holds (the oracle's input)."""
    import torch

    Ab = torch.from_numpy(np.ascontiguousarray(A32, dtype=np.float32)).to(torch_dev())
    Ab = Ab.to(torch.bfloat16)
    return Ab, Ab.float().cpu().numpy().astype(np.float64)


# n is the row pitch of A: a multiple of 8. The shapes cover M and K tails
# (K = n not a multiple of 64), one column tile up to the full 128 columns.
SHAPES = [(1, 8, 1), (300, 1000, 10), (777, 520, 50), (256, 4096, 100), (130, 2000, 128),
          (64, 72, 16), (2049, 136, 33)]


@pytest.mark.parametrize("m,n,k", SHAPES)
def test_bf16_AF(m, n, k):
    A32 = uniform((m, n), seed=m + n).astype(np.float32)
    F = uniform((n, k), seed=k + 7).astype(np.float32)
    Ab, A64 = bf16_dev(A32)
    step("bf16 A F %dx%d k=%d" % (m, n, k))
    P = host(nmf.nmf_dense_AF(Ab, to_dev(F, np.float32)))
    Fr = oracle.round_bf16(F)
    ref = oracle.product_AHt(A64, Fr.T)
    assert_gemm_bound(P, ref, np.abs(A64) @ np.abs(Fr), n, U32, what="bf16 A F")
    # precision of the method: the factor's rounding, at most 2^-8 per entry
    exact = A64 @ F.astype(np.float64)
    assert rel_diff(P, exact) <= 2.0 ** -8 + 1e-6


@pytest.mark.parametrize("m,n,k", SHAPES)
def test_bf16_AtF(m, n, k):
    A32 = uniform((m, n), seed=3 * m + n).astype(np.float32)
    F = uniform((m, k), seed=k + 9).astype(np.float32)
    Ab, A64 = bf16_dev(A32)
    step("bf16 A^T F %dx%d k=%d" % (m, n, k))
    R = host(nmf.nmf_dense_AtF(Ab, to_dev(F, np.float32)))
    Fr = oracle.round_bf16(F)
    ref = oracle.product_WtA(A64, Fr).T
    assert_gemm_bound(R, ref, np.abs(A64).T @ np.abs(Fr), m, U32, what="bf16 A^T F")


def test_bf16_rejects_unaligned_row_pitch():
    import torch

    A = torch.zeros((16, 12), dtype=torch.bfloat16, device=torch_dev())
    F = torch.zeros((12, 4), dtype=torch.float32, device=torch_dev())
    with pytest.raises(nmf.NMFError):
        nmf.nmf_dense_AF(A, F)


def test_bf16_relerr_matches_oracle():
    m, n, k = 333, 264, 12
    A32 = planted_dense(m, n, k, seed=21).astype(np.float32)
    Ab, A64 = bf16_dev(A32)
    W, H = init_factors(m, n, k, seed=22)
    W32, H32 = W.astype(np.float32), H.astype(np.float32)
    step("bf16 relerr")
    got = nmf.nmf_dense_relerr(Ab, to_dev(W32, np.float32), to_dev(H32.T, np.float32))
    ref = oracle.relative_error(A64, W32.astype(np.float64), H32.astype(np.float64))
    assert abs(got - ref) <= 1e-5 * ref


@pytest.mark.parametrize("algo,k,iters", [("hals", 16, 10), ("mu", 16, 10), ("abpp", 10, 6),
                                          ("hals", 100, 4)])
def test_bf16_runs_match_oracle(algo, k, iters):
    import torch

    m, n = 500, 400
    A32 = planted_dense(m, n, k, seed=31).astype(np.float32)
    Ab, A64 = bf16_dev(A32)
    W0, H0 = init_factors(m, n, k, seed=32)
    W0, H0 = W0.astype(np.float32), H0.astype(np.float32)
    W = to_dev(W0, np.float32)
    H = to_dev(H0, np.float32)
    step("bf16 run %s k=%d" % (algo, k))
    errs, _ = nmf.nmf_dense(Ab, W, H, algo=algo, iters=iters, objective=True)
    torch.cuda.synchronize()
    _, _, e_b = oracle.run(A64, k, algo, iters, W0, H0, bf16_products=True)
    _, _, e_x = oracle.run(A64, k, algo, iters, W0, H0)
    d_b = rel_diff(errs, e_b)
    d_x = rel_diff(errs, e_x)
    d_bx = rel_diff(e_b, e_x)
    print("bf16 %s k=%d: rel err gpu %s\n  oracle(bf16 products) %s\n  oracle(fp64) %s\n"
          "  max diff %.2e vs bf16 variant, %.2e vs fp64 (bf16 variant vs fp64: %.2e)"
          % (algo, k, errs, e_b, e_x, d_b, d_x, d_bx))
    # the first iteration starts from identical factors: float accumulation only
    assert rel_diff(errs[:2], e_b[:2]) <= 1e-4
    # Two cases are held to bars derived from what float32 arithmetic alone
    # does to their trajectories (tests/parity_bars.py, produced by
    # test_parity_bars_cpu.py): ABPP, whose exact solves carry every
    # float32-level change of a factor into whole bfloat16 steps of the next
    # product's operand, and HALS at k = 100, with many entries at the
    # projection boundary. The others are held to 1e-4.
    if algo == "abpp":
        c = parity_bars.ABPP_BF16_CASE
        assert (m, n, k, iters) == (c["m"], c["n"], c["k"], c["iters"])
        bar = parity_bars.ABPP_BF16_BAR
    elif k == 100:
        c = parity_bars.HALS_BF16_K100_CASE
        assert (m, n, k, iters) == (c["m"], c["n"], c["k"], c["iters"])
        bar = parity_bars.HALS_BF16_K100_BAR
    else:
        bar = 1e-4
    assert d_b <= bar
