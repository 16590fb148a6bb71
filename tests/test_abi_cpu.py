"""The C-ABI library loads, exports every function include/nmf.h declares,
and rejects bad arguments on the host before touching a device (checked on a
context bound to no device, so no GPU is needed)."""
import ctypes
import os
import re

import pytest

from paper_1609_09154_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nmf.h")

EINVAL, EDEVICE = _lib.NMF_EINVAL, _lib.NMF_EDEVICE


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nmf_[a-z_A-Z0-9]+)\s*\(", text)))


def test_header_and_binding_agree():
    names = declared_functions()
    assert len(names) >= 15
    assert set(names) == set(_lib.SIGNATURES), set(names) ^ set(_lib.SIGNATURES)


def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_status_strings_and_defaults():
    L = _lib.lib()
    assert L.nmf_status_str(0) == b"NMF_OK"
    assert L.nmf_status_str(5) == b"NMF_ENOTCONV"
    o = _lib.default_opts()
    assert o.algo == _lib.NMF_MU and o.iters == 0 and o.eps_mu == 1e-16
    assert o.max_pivots == 0 and o.objective == 0 and o.transpose_a == 0
    # the ctypes mirrors must be at least as large as the C structs they stand for
    assert o.tol == 0.0 and o.stop == 0
    assert ctypes.sizeof(_lib.NmfOpts) == 8 * 7 and ctypes.sizeof(_lib.NmfStats) == 8 * 16


@pytest.fixture
def hctx():
    L = _lib.lib()
    h = ctypes.c_void_p()
    assert L.nmf_create(ctypes.byref(h), -1, None) == 0
    yield h
    L.nmf_destroy(h)


P = ctypes.c_void_p(4096)  # never dereferenced: checks fail or the context has no device


def dense(h, m=10, n=8, lda=8, k=3, dtype=_lib.NMF_F32, opts=None, A=P, W=P, H=P, relerr=None):
    o = opts or _lib.default_opts(algo="hals", iters=2)
    return _lib.lib().nmf_dense(h, dtype, m, n, A, lda, k, ctypes.byref(o), W, H, relerr, None)


def test_valid_dense_call_reaches_device_stage(hctx):
    assert dense(hctx) == EDEVICE


@pytest.mark.parametrize("kw", [dict(m=0), dict(n=0), dict(k=0), dict(k=129), dict(lda=7),
                                dict(dtype=7), dict(A=None), dict(W=None), dict(H=None),
                                dict(m=1 << 41)])
def test_dense_argument_errors(hctx, kw):
    assert dense(hctx, **kw) == EINVAL
    assert _lib.lib().nmf_last_error(hctx)


@pytest.mark.parametrize("dtype,unit", [(_lib.NMF_BF16, 8), (_lib.NMF_FP8_E4M3, 16)])
def test_reduced_precision_A_checks(hctx, dtype, unit):
    # a row pitch of whole 16-byte units and an aligned A reach the device stage
    assert dense(hctx, n=8, lda=2 * unit, dtype=dtype) == EDEVICE
    assert dense(hctx, n=8, lda=unit + unit // 2, dtype=dtype) == EINVAL
    assert dense(hctx, n=8, lda=2 * unit, dtype=dtype, A=ctypes.c_void_p(4096 + 8)) == EINVAL
    o = _lib.default_opts(algo="hals", iters=2, transpose_a=-1)
    assert dense(hctx, n=8, lda=2 * unit, dtype=dtype, opts=o) == EINVAL
    L = _lib.lib()
    assert L.nmf_dense_AF(hctx, dtype, 10, 8, P, unit + 1, 3, P, 3, P) == EINVAL
    assert L.nmf_dense_AF(hctx, dtype, 10, 8, P, 2 * unit, 3, P, 3, P) == EDEVICE


def test_dense_bad_options(hctx):
    assert dense(hctx, opts=_lib.default_opts(algo=3)) == EINVAL
    assert dense(hctx, opts=_lib.default_opts(iters=-1)) == EINVAL
    assert dense(hctx, opts=_lib.default_opts(objective=9)) == EINVAL
    assert dense(hctx, opts=_lib.default_opts(eps_mu=-1.0)) == EINVAL
    assert dense(hctx, k=65, opts=_lib.default_opts(algo="abpp")) == EINVAL
    # rel_err requested without an objective
    errs = (ctypes.c_double * 3)()
    assert dense(hctx, relerr=errs) == EINVAL


def test_null_context_and_opts():
    L = _lib.lib()
    assert L.nmf_dense(None, 1, 4, 4, P, 4, 2, None, P, P, None, None) == EINVAL
    h = ctypes.c_void_p()
    assert L.nmf_create(ctypes.byref(h), -1, None) == 0
    assert L.nmf_dense(h, 1, 4, 4, P, 4, 2, None, P, P, None, None) == EINVAL
    L.nmf_destroy(h)
    assert L.nmf_create(None, 0, None) == EINVAL


def test_csr_argument_errors(hctx):
    L = _lib.lib()
    o = _lib.default_opts(algo="abpp", iters=1)
    ok = L.nmf_csr(hctx, 10, 10, 5, P, P, P, 3, ctypes.byref(o), P, P, None, None)
    assert ok == EDEVICE
    assert L.nmf_csr(hctx, 10, 10, -1, P, P, P, 3, ctypes.byref(o), P, P, None, None) == EINVAL
    assert L.nmf_csr(hctx, 10, 10, 5, None, P, P, 3, ctypes.byref(o), P, P, None, None) == EINVAL
    assert L.nmf_csr(hctx, 10, 10, 5, P, None, P, 3, ctypes.byref(o), P, P, None, None) == EINVAL
    assert L.nmf_csr(hctx, 10, 1 << 32, 5, P, P, P, 3, ctypes.byref(o), P, P, None, None) == EINVAL


def test_step_argument_errors(hctx):
    L = _lib.lib()
    assert L.nmf_gram(hctx, 1, 10, 3, P, 2, P) == EINVAL          # ldx < k
    assert L.nmf_gram(hctx, 1, 10, 3, P, 3, P) == EDEVICE
    assert L.nmf_dense_AF(hctx, 1, 10, 8, P, 8, 3, P, 2, P) == EINVAL
    assert L.nmf_dense_AtF(hctx, 1, 10, 8, P, 7, 3, P, 3, P) == EINVAL
    assert L.nmf_dense_AF(hctx, 1, 10, 8, P, 8, 3, P, 3, P) == EDEVICE
    o = _lib.default_opts()
    piv = ctypes.c_longlong()
    assert L.nmf_update(hctx, 9, 1, 10, 3, P, P, P, ctypes.byref(o), ctypes.byref(piv)) == EINVAL
    assert L.nmf_update(hctx, 2, 1, 10, 80, P, P, P, ctypes.byref(o), ctypes.byref(piv)) == EINVAL
    assert L.nmf_update(hctx, 1, 1, 10, 3, None, P, P, ctypes.byref(o), ctypes.byref(piv)) == EINVAL
    assert L.nmf_update(hctx, 1, 1, 10, 3, P, P, P, ctypes.byref(o), ctypes.byref(piv)) == EDEVICE
    # the allocation-free form: same checks, plus its fixed scratch size
    upd = L.nmf_update_noalloc
    assert upd(hctx, 9, 1, 10, 3, P, P, P, ctypes.byref(o), ctypes.byref(piv)) == EINVAL
    assert upd(hctx, 2, 1, 10, 80, P, P, P, ctypes.byref(o), ctypes.byref(piv)) == EINVAL
    assert upd(hctx, 1, 7, 10, 3, P, P, P, ctypes.byref(o), ctypes.byref(piv)) == EINVAL
    # float32, k = 64: 2 rows 64 4 + 64^2 (4 + 8) + at most 1024 bytes
    too_many = _lib.NMF_NOALLOC_SCRATCH_BYTES // (2 * 64 * 4) + 1
    assert upd(hctx, 1, 1, too_many, 64, P, P, P, ctypes.byref(o), ctypes.byref(piv)) == EINVAL
    assert b"scratch" in L.nmf_last_error(hctx)
    fits = (_lib.NMF_NOALLOC_SCRATCH_BYTES - 1024 - 64 * 64 * 12) // (2 * 64 * 4)
    assert upd(hctx, 1, 1, fits, 64, P, P, P, ctypes.byref(o), ctypes.byref(piv)) == EDEVICE
    assert upd(hctx, 1, 0, 32000, 128, P, P, P, ctypes.byref(o), ctypes.byref(piv)) == EDEVICE
    out = ctypes.c_double()
    assert L.nmf_dense_relerr(hctx, 1, 10, 8, P, 8, 3, P, P, None) == EINVAL
    assert L.nmf_dense_relerr(hctx, 1, 10, 8, P, 8, 3, P, P, ctypes.byref(out)) == EDEVICE
    assert L.nmf_csr_transpose(hctx, 10, 8, -2, P, P, P, P, P, P) == EINVAL
    assert L.nmf_hals_normalize(hctx, 1, 10, 8, 0, P, P, None, None) == EINVAL


def test_mu_unrolled_argument_errors(hctx):
    L = _lib.lib()
    assert L.nmf_mu_ckpt_elems(10, 8, 3, 25, 10) == 3 * (10 + 8) * 16
    assert L.nmf_mu_ckpt_elems(10, 8, 65, 5, 1) == -1
    assert L.nmf_mu_ckpt_elems(10, 8, 3, 5, 0) == -1
    assert L.nmf_mu_ckpt_elems(10, 8, 3, 0, 4) == 0
    fw = L.nmf_mu_unrolled_forward
    assert fw(hctx, 1, 10, 8, P, 8, 3, 5, 1e-16, 2, P, P, P) == EDEVICE
    assert fw(hctx, 1, 10, 8, P, 8, 65, 5, 1e-16, 2, P, P, P) == EINVAL   # k > 64
    assert fw(hctx, 2, 10, 8, P, 8, 3, 5, 1e-16, 2, P, P, P) == EINVAL    # BF16 A
    assert fw(hctx, 1, 10, 8, P, 8, 3, 5, 1e-16, 0, P, P, P) == EINVAL    # ckpt_every 0
    assert fw(hctx, 1, 10, 8, P, 8, 3, -1, 1e-16, 2, P, P, P) == EINVAL   # iters < 0
    assert fw(hctx, 1, 10, 8, P, 8, 3, 5, -1.0, 2, P, P, P) == EINVAL     # eps < 0
    assert fw(hctx, 1, 10, 8, P, 7, 3, 5, 1e-16, 2, P, P, P) == EINVAL    # lda < n
    assert fw(hctx, 1, 10, 8, P, 8, 3, 5, 1e-16, 2, None, P, P) == EINVAL
    bw = L.nmf_mu_unrolled_backward
    assert bw(hctx, 1, 10, 8, P, 8, 3, 5, 1e-16, 2, P, P, P, P, 8, P, P) == EDEVICE
    assert bw(hctx, 1, 10, 8, P, 8, 3, 5, 1e-16, 2, None, P, P, P, 8, P, P) == EINVAL
    assert bw(hctx, 1, 10, 8, P, 8, 3, 5, 1e-16, 2, P, P, P, P, 7, P, P) == EINVAL  # ldga
    assert bw(hctx, 1, 10, 8, P, 8, 3, 5, 1e-16, 2, P, P, P, None, 0, P, P) == EDEVICE


def test_hals_unrolled_argument_errors(hctx):
    L = _lib.lib()
    fw = L.nmf_hals_unrolled_forward
    assert fw(hctx, 1, 10, 8, P, 8, 3, 5, 2, P, P, P) == EDEVICE
    assert fw(hctx, 0, 10, 8, P, 8, 3, 5, 2, P, P, None) == EDEVICE    # no checkpoints
    assert fw(hctx, 1, 10, 8, P, 8, 65, 5, 2, P, P, P) == EINVAL      # k > 64
    assert fw(hctx, 2, 10, 8, P, 8, 3, 5, 2, P, P, P) == EINVAL       # BF16 A
    assert fw(hctx, 1, 10, 8, P, 8, 3, 5, 0, P, P, P) == EINVAL       # ckpt_every 0
    assert fw(hctx, 1, 10, 8, P, 8, 3, -1, 2, P, P, P) == EINVAL      # iters < 0
    assert fw(hctx, 1, 10, 8, P, 7, 3, 5, 2, P, P, P) == EINVAL       # lda < n
    assert fw(hctx, 1, 10, 8, None, 8, 3, 5, 2, P, P, P) == EINVAL
    assert fw(hctx, 1, 10, 8, P, 8, 3, 5, 2, P, None, P) == EINVAL
    bw = L.nmf_hals_unrolled_backward
    assert bw(hctx, 1, 10, 8, P, 8, 3, 5, 2, P, P, P, P, 8, P, P) == EDEVICE
    assert bw(hctx, 1, 10, 8, P, 8, 3, 5, 2, None, P, P, P, 8, P, P) == EINVAL
    assert bw(hctx, 1, 10, 8, P, 8, 3, 0, 2, None, P, P, P, 8, P, P) == EDEVICE  # T = 0
    assert bw(hctx, 1, 10, 8, P, 8, 3, 5, 2, P, P, P, P, 7, P, P) == EINVAL  # ldga
    assert bw(hctx, 1, 10, 8, P, 8, 3, 5, 2, P, P, None, P, 8, P, P) == EINVAL
    assert bw(hctx, 1, 10, 8, P, 8, 3, 5, 2, P, P, P, None, 0, P, P) == EDEVICE


def test_stop_options_and_pgrad_argument_errors(hctx):
    L = _lib.lib()
    assert dense(hctx, opts=_lib.default_opts(algo="hals", iters=2, stop=1, tol=0.1)) == EDEVICE
    assert dense(hctx, opts=_lib.default_opts(algo="hals", iters=2, stop=3)) == EINVAL
    assert dense(hctx, opts=_lib.default_opts(algo="hals", iters=2, stop=1, tol=-1.0)) == EINVAL
    # the relative-error test needs the objective
    assert dense(hctx, opts=_lib.default_opts(algo="hals", iters=2, stop=2, tol=0.1)) == EINVAL
    assert dense(hctx, opts=_lib.default_opts(algo="hals", iters=2, stop=2, tol=0.1,
                                              objective=1)) == EDEVICE
    out = ctypes.c_double()
    assert L.nmf_projected_gradient_sq(hctx, 1, 10, 3, P, P, P, ctypes.byref(out)) == EDEVICE
    assert L.nmf_projected_gradient_sq(hctx, 1, 10, 3, P, None, P, ctypes.byref(out)) == EINVAL
    assert L.nmf_projected_gradient_sq(hctx, 1, 10, 3, P, P, P, None) == EINVAL
