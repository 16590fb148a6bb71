"""Plain FP64 CPU oracle for alternating-updating NMF.

TEST INFRASTRUCTURE ONLY. Nothing in the GPU library imports, links or runs
anything in this package; only the test suite, the smoke check and the
benchmark's CPU-baseline leg may call it. It shares no code with the GPU
path: the two see the same input arrays (from ``synth``) and nothing else.

Everything here follows the paper's definitions in the paper's order, in
float64, with library primitives (matmul, a dense linear solve) as the only
building blocks:

* Algorithm 1 (AU-NMF): update W from (H H^T, A H^T), then H from
  (W^T W, W^T A), for a fixed number of iterations (Section 6.1.3 uses the
  iteration count as the stopping rule).
* Section 4.1, Eq. (3): multiplicative update (MU).
* Section 4.2, Eqs. (4)-(5): HALS, a 2k-block coordinate descent.
* Section 4.3, Eqs. (6)-(7): ANLS with block principal pivoting (BPP).
* Section 6.2: relative error ||A - W H||_F / ||A||_F after each full
  iteration.

Readings where the paper is silent or inconsistent are stated next to the
code that takes them (MU's zero-denominator guard, HALS's divisor and
normalisation, BPP's pivoting rule and the degenerate-Gram tie-break).
"""
from .nmf import (  # noqa: F401
    gram_fixed_H, gram_fixed_W, product_AHt, product_WtA,
    mu_update_W, mu_update_H, hals_update_W, hals_update_H,
    abpp_update_W, abpp_update_H, relative_error, objective_sq, run,
    round_bf16, round_fp8_e4m3, fp8_column_scales, round_fp8_scaled, FP8_E4M3_MAX,
    MU_EPS, gradients, projected_gradient_sq, projected_gradient_norm, run_until,
)
from .bpp import bpp_nnls, passive_solve  # noqa: F401
from .autodiff import (mu_unrolled_forward, mu_unrolled_vjp, hals_unrolled_forward,  # noqa: F401
                       hals_unrolled_vjp)
