"""nmf_update_noalloc, the allocation-free form of nmf_update (fixed device
scratch instead of the context workspace), against nmf_update itself.

Both run the same kernels with the same launch shapes, so the updated
factor and the ABPP pivot count must be identical, bit for bit. Each case
makes two calls in a row on the one scratch array, the second with a
smaller input (fewer rows and a smaller rank), so a stale counter, inverse
Gram or padding column left by the first call would show in the second."""
import numpy as np
import pytest

import paper_1609_09154_amd as nmf
from paper_1609_09154_amd import _lib
from tests.gpu_util import step

pytestmark = pytest.mark.gpu


def _case(rows, k, dtype, seed):
    """G = F^T F of a random nonnegative F (SPD for 3k >= k rows), P >= 0 and a
    positive starting X, as the update sees them inside Algorithm 1."""
    import torch

    rng = np.random.default_rng(seed)
    F = rng.uniform(0.0, 1.0, size=(3 * k + 7, k))
    G = F.T @ F
    P = rng.uniform(0.0, 1.0, size=(rows, k)) * (3 * k + 7) / 4.0
    X = rng.uniform(0.0, 1.0, size=(rows, k))
    dev = torch.device("cuda:0")
    return [torch.from_numpy(a).to(dev, dtype).contiguous() for a in (G, P, X)]


@pytest.mark.parametrize("algo", ["mu", "hals", "abpp"])
@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_noalloc_update_matches_nmf_update(algo, dt):
    import torch

    dtype = torch.float32 if dt == "f32" else torch.float64
    # (rows, k): a large call first, then a smaller one on the same scratch
    for i, (rows, k) in enumerate([(20011, 50), (3001, 10)]):
        step("noalloc %s %s call %d: rows %d k %d" % (algo, dt, i, rows, k))
        G, P, X0 = _case(rows, k, dtype, seed=100 * i + 7)
        Xa = X0.clone()
        piv_a = nmf.nmf_update(algo, G, P, Xa)
        Xb = X0.clone()
        piv_b = nmf.nmf_update_noalloc(algo, G, P, Xb)
        torch.cuda.synchronize()
        assert torch.isfinite(Xb).all()
        assert (Xb >= 0).all()
        assert torch.equal(Xa, Xb), float((Xa - Xb).abs().max())
        assert piv_a == piv_b
        if algo == "abpp":
            assert piv_b >= rows


def test_noalloc_rejects_sizes_past_the_scratch():
    import torch

    dev = torch.device("cuda:0")
    k = 64
    rows = _lib.NMF_NOALLOC_SCRATCH_BYTES // (2 * k * 4) + 1
    G = torch.eye(k, device=dev)
    P = torch.zeros((rows, k), device=dev)
    X = torch.zeros((rows, k), device=dev)
    step("noalloc: oversized call must be rejected")
    with pytest.raises(nmf.NMFError) as ei:
        nmf.nmf_update_noalloc("mu", G, P, X)
    assert ei.value.status == _lib.NMF_EINVAL
    assert "scratch" in str(ei.value)
    # the entry point still works after the rejection
    G, P, X0 = _case(1000, 16, torch.float32, seed=3)
    Xa, Xb = X0.clone(), X0.clone()
    nmf.nmf_update("hals", G, P, Xa)
    nmf.nmf_update_noalloc("hals", G, P, Xb)
    torch.cuda.synchronize()
    assert torch.equal(Xa, Xb)
