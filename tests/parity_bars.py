"""Parity bars looser than the stated tolerances (1e-5 per iteration on the
relative error for FP32 runs, 1e-4 for runs with BF16 products), with the
cases they apply to. Each value here is produced by a CPU test in
tests/test_parity_bars_cpu.py: float32 arithmetic alone (tests/fp32_model.py,
sums accumulated term by term in float32 in several orders of the terms,
factors, products and Grams stored in float32) moves the FP64 oracle's
trajectory on that case by more than the stated tolerance, and the bar is
set above the largest such move and no more than twice it."""

# Dense FP32 ABPP, 1500 x 1100, k = 50 on a planted rank-50 matrix (seed
# 151), 5 iterations: the fit reaches the noise level (e_T = 0.0133), and
# ABPP's exact solves amplify the rounding of A H^T, W^T A and the Grams by
# their conditioning. float32 arithmetic moves this trajectory by 8.9e-6 to
# 7.9e-5 depending on the summation order.
ABPP_F32_CASE = dict(m=1500, n=1100, k=50, k_true=50, seed=151, iters=5)
ABPP_F32_BAR = 1e-4

# HALS with BF16 products, 500 x 400, k = 100 on a planted rank-100 matrix
# (seeds 31, 32), 4 iterations: many entries sit at the projection boundary;
# float32 arithmetic moves the trajectory by about 2.5e-4.
HALS_BF16_K100_CASE = dict(m=500, n=400, k=100, seed=31, init_seed=32, iters=4)
HALS_BF16_K100_BAR = 5e-4

# ABPP with BF16 products, 500 x 400, k = 10 (seeds 31, 32), 6 iterations: a
# float32-level change of a factor moves the bfloat16 rounding of the next
# product's operand by whole bfloat16 steps, and the exact solves carry that
# forward; float32 arithmetic moves the trajectory by 2.6e-3 to 7.7e-3.
ABPP_BF16_CASE = dict(m=500, n=400, k=10, seed=31, init_seed=32, iters=6)
ABPP_BF16_BAR = 1e-2
