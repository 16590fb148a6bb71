"""Helpers shared by the GPU parity tests (inputs, tolerances, transfers)."""
import sys

import numpy as np

U32 = 2.0 ** -24   # unit roundoff, float32
U64 = 2.0 ** -53   # unit roundoff, float64


def step(name):
    """Print (and flush) what the next GPU step is, so a lost run names it."""
    print("[gpu-step] %s" % name, flush=True)
    sys.stdout.flush()


def torch_dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda:0")


def to_dev(x, dtype):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x, dtype=dtype)).to(torch_dev())


def host(t):
    return t.detach().cpu().numpy()


def gamma(K, u):
    """gamma_K = K u / (1 - K u): the textbook bound on the relative error of a
    K-term sum of products in floating point, any summation order."""
    return K * u / (1.0 - K * u)


def assert_gemm_bound(got, ref, absref, K, u, slack=1.0, what=""):
    """|got - ref| <= gamma_K |A||B| elementwise (ref, absref in FP64)."""
    bound = slack * gamma(K + 2, u) * absref + 1e-300
    err = np.abs(got.astype(np.float64) - ref)
    worst = float(np.max(err / bound)) if err.size else 0.0
    assert worst <= 1.0, "%s: error exceeds gamma_K bound by %.3g" % (what, worst)
    return worst


def rel_diff(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)))
