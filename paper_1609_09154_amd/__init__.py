"""Alternating-updating NMF (A ~= W H, W, H >= 0) on one MI355X (gfx950).

Python face of libnmf_mi355x.so. Each function here has the name of the C
entry point it calls (include/nmf.h) and only marshals arguments: torch
CUDA tensors give device pointers, the current torch stream gives the HIP
stream. Shapes follow the paper's notation: A is m x n, W is m x k, H is
k x n; the per-step calls use the row layout of the header (the fixed
factor as W, m x k, or as H^T, n x k).
"""
from __future__ import annotations

import ctypes

from . import _lib
from ._lib import (NMF_ABPP, NMF_BF16, NMF_F32, NMF_F64, NMF_FP8_E4M3, NMF_HALS, NMF_MU,  # noqa: F401
                   NMF_OBJ_DIRECT, NMF_OBJ_NONE, NMFError, NmfStats, default_opts)

__all__ = ["Context", "NMFError", "nmf_dense", "nmf_csr", "nmf_gram", "nmf_dense_AF",
           "nmf_mu_unrolled_forward", "nmf_mu_unrolled_backward", "mu_unrolled",
           "nmf_hals_unrolled_forward", "nmf_hals_unrolled_backward", "hals_unrolled",
           "nmf_projected_gradient_sq",
           "nmf_dense_AtF", "nmf_csr_AF", "nmf_csr_transpose", "nmf_update", "nmf_update_noalloc",
           "nmf_hals_normalize", "nmf_dense_relerr", "nmf_csr_relerr", "library_path"]


def library_path() -> str:
    return _lib.LIB_PATH


def _torch():
    import torch
    return torch


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.float32:
        return NMF_F32
    if t.dtype == torch.float64:
        return NMF_F64
    if t.dtype == torch.bfloat16:
        return NMF_BF16
    if t.dtype == getattr(torch, "float8_e4m3fn", None):
        return NMF_FP8_E4M3
    raise TypeError("only float32, float64, bfloat16 (A) and float8_e4m3fn (A) tensors are "
                    "supported, got %s" % t.dtype)


def _factor_dtype(A):
    """Element type of W, H and the products for a dense A: float32 when A
    is bfloat16 or float8_e4m3fn, A's own type otherwise."""
    torch = _torch()
    if A.dtype in (torch.bfloat16, getattr(torch, "float8_e4m3fn", None)):
        return torch.float32
    return A.dtype


def _dev(t, name, dtype=None, shape=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if dtype is not None and t.dtype != dtype:
        raise TypeError("%s must have dtype %s, got %s" % (name, dtype, t.dtype))
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """Owns an nmf_ctx (the library's workspace) on one device.

    The context follows torch's current stream at every call.
    """

    def __init__(self, device: int = 0):
        torch = _torch()
        self.device = device
        h = ctypes.c_void_p()
        with torch.cuda.device(device):
            st = torch.cuda.current_stream(device).cuda_stream
            rc = _lib.lib().nmf_create(ctypes.byref(h), device, ctypes.c_void_p(st))
        if rc != 0:
            raise NMFError(rc, "nmf_create failed")
        self.handle = h

    def _sync_stream(self):
        torch = _torch()
        st = torch.cuda.current_stream(self.device).cuda_stream
        _lib.lib().nmf_set_stream(self.handle, ctypes.c_void_p(st))

    def check(self, rc: int):
        if rc != 0:
            raise NMFError(rc, _lib.lib().nmf_last_error(self.handle).decode())

    def close(self):
        if getattr(self, "handle", None):
            _lib.lib().nmf_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_CTX = {}


def _ctx(ctx, device) -> Context:
    if ctx is not None:
        ctx._sync_stream()
        return ctx
    if device not in _CTX:
        _CTX[device] = Context(device)
    c = _CTX[device]
    c._sync_stream()
    return c


def _stop_opts(stop, tol):
    code = _lib.STOPS["iters" if stop is None else stop]
    return dict(stop=code, tol=float(tol))


def _errs(errs, stats):
    if errs is None:
        return None
    return list(errs)[: int(stats.iters_done) + 1]


def nmf_dense(A, W, H, algo="hals", iters=10, objective=True, eps_mu=1e-16, max_pivots=0,
              timers=False, check_input=False, transpose_a=True, stop=None, tol=0.0, ctx=None):
    """Algorithm 1 on dense A (m x n); W (m x k) and H (k x n) are updated in
    place. transpose_a=False keeps the library from holding a transposed
    copy of A. A may be bfloat16 or float8_e4m3fn (then W and H are float32,
    the products run on the BF16 or FP8 matrix cores). stop = "pgrad" or "relerr" adds the tolerance
    test of nmf_opts (iters is then the cap). Returns (rel_err list or None,
    stats dict); the list ends at the last iteration performed."""
    torch = _torch()
    m, n = A.shape
    k = W.shape[1]
    dt = _factor_dtype(A)
    pa = _dev(A, "A")
    pw = _dev(W, "W", dtype=dt, shape=(m, k))
    ph = _dev(H, "H", dtype=dt, shape=(k, n))
    c = _ctx(ctx, A.device.index or 0)
    o = default_opts(algo=algo, iters=iters, eps_mu=eps_mu, max_pivots=max_pivots,
                     objective=NMF_OBJ_DIRECT if objective else NMF_OBJ_NONE,
                     timers=1 if timers else 0, check_input=1 if check_input else 0,
                     transpose_a=0 if transpose_a else -1, **_stop_opts(stop, tol))
    errs = (ctypes.c_double * (iters + 1))() if objective else None
    stats = NmfStats()
    rc = _lib.lib().nmf_dense(c.handle, _dtype_code(A), m, n, pa, A.stride(0), k, ctypes.byref(o),
                            pw, ph, errs, ctypes.byref(stats))
    c.check(rc)
    del torch
    return _errs(errs, stats), stats.as_dict()


def nmf_csr(rowptr, colidx, vals, n, W, H, algo="abpp", iters=10, objective=True,
            eps_mu=1e-16, max_pivots=0, timers=False, check_input=False, stop=None, tol=0.0,
            ctx=None):
    """Algorithm 1 on CSR A (float32); W (m x k), H (k x n) float32, in place."""
    torch = _torch()
    m = rowptr.numel() - 1
    nnz = colidx.numel()
    k = W.shape[1]
    args = (_dev(rowptr, "rowptr", dtype=torch.int64), _dev(colidx, "colidx", dtype=torch.int32),
            _dev(vals, "vals", dtype=torch.float32))
    pw = _dev(W, "W", dtype=torch.float32, shape=(m, k))
    ph = _dev(H, "H", dtype=torch.float32, shape=(k, n))
    c = _ctx(ctx, W.device.index or 0)
    o = default_opts(algo=algo, iters=iters, eps_mu=eps_mu, max_pivots=max_pivots,
                     objective=NMF_OBJ_DIRECT if objective else NMF_OBJ_NONE,
                     timers=1 if timers else 0, check_input=1 if check_input else 0,
                     **_stop_opts(stop, tol))
    errs = (ctypes.c_double * (iters + 1))() if objective else None
    stats = NmfStats()
    rc = _lib.lib().nmf_csr(c.handle, m, n, nnz, *args, k, ctypes.byref(o), pw, ph, errs,
                          ctypes.byref(stats))
    c.check(rc)
    return _errs(errs, stats), stats.as_dict()


def nmf_gram(X, ctx=None):
    """G = X^T X for X rows x k."""
    torch = _torch()
    rows, k = X.shape
    G = torch.empty((k, k), dtype=X.dtype, device=X.device)
    c = _ctx(ctx, X.device.index or 0)
    c.check(_lib.lib().nmf_gram(c.handle, _dtype_code(X), rows, k, _dev(X, "X"), X.stride(0),
                              _dev(G, "G")))
    return G


def nmf_dense_AF(A, F, ctx=None):
    """P = A F for dense A (m x n) and F (n x k); A may be bfloat16 or
    float8_e4m3fn (F and P float32)."""
    torch = _torch()
    m, n = A.shape
    k = F.shape[1]
    _dev(F, "F", dtype=_factor_dtype(A), shape=(n, k))
    P = torch.empty((m, k), dtype=_factor_dtype(A), device=A.device)
    c = _ctx(ctx, A.device.index or 0)
    c.check(_lib.lib().nmf_dense_AF(c.handle, _dtype_code(A), m, n, _dev(A, "A"), A.stride(0), k,
                                  _dev(F, "F"), F.stride(0), _dev(P, "P")))
    return P


def nmf_dense_AtF(A, F, ctx=None):
    """R = A^T F for dense A (m x n) and F (m x k); A may be bfloat16 or
    float8_e4m3fn (F and R float32)."""
    torch = _torch()
    m, n = A.shape
    k = F.shape[1]
    _dev(F, "F", dtype=_factor_dtype(A), shape=(m, k))
    R = torch.empty((n, k), dtype=_factor_dtype(A), device=A.device)
    c = _ctx(ctx, A.device.index or 0)
    c.check(_lib.lib().nmf_dense_AtF(c.handle, _dtype_code(A), m, n, _dev(A, "A"), A.stride(0), k,
                                   _dev(F, "F"), F.stride(0), _dev(R, "R")))
    return R


def nmf_csr_AF(rowptr, colidx, vals, n, F, ctx=None):
    """P = A F for CSR A (m x n, float32) and F (n x k, float32)."""
    torch = _torch()
    m = rowptr.numel() - 1
    k = F.shape[1]
    _dev(F, "F", dtype=torch.float32, shape=(n, k))
    P = torch.empty((m, k), dtype=torch.float32, device=F.device)
    c = _ctx(ctx, F.device.index or 0)
    c.check(_lib.lib().nmf_csr_AF(c.handle, m, n, colidx.numel(),
                                _dev(rowptr, "rowptr", dtype=torch.int64),
                                _dev(colidx, "colidx", dtype=torch.int32),
                                _dev(vals, "vals", dtype=torch.float32), k, _dev(F, "F"),
                                _dev(P, "P")))
    return P


def nmf_csr_transpose(rowptr, colidx, vals, n, ctx=None):
    """CSR of A^T: returns (rowptr_t, colidx_t, vals_t)."""
    torch = _torch()
    m = rowptr.numel() - 1
    nnz = colidx.numel()
    dev = rowptr.device
    rpt = torch.empty(n + 1, dtype=torch.int64, device=dev)
    cit = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)[:nnz]
    cvt = torch.empty(max(nnz, 1), dtype=torch.float32, device=dev)[:nnz]
    c = _ctx(ctx, dev.index or 0)
    c.check(_lib.lib().nmf_csr_transpose(c.handle, m, n, nnz,
                                       _dev(rowptr, "rowptr", dtype=torch.int64),
                                       _dev(colidx, "colidx", dtype=torch.int32),
                                       _dev(vals, "vals", dtype=torch.float32),
                                       _dev(rpt, "rowptr_t"), _dev(cit, "colidx_t"),
                                       _dev(cvt, "vals_t")))
    return rpt, cit, cvt


def nmf_update(algo, G, P, X, eps_mu=1e-16, max_pivots=0, ctx=None):
    """In-place local update of X (rows x k) from the Gram G (k x k) and P
    (rows x k). Returns the number of BPP passive-set solves (ABPP) or 0."""
    rows, k = X.shape
    dt = X.dtype
    _dev(G, "G", dtype=dt, shape=(k, k))
    _dev(P, "P", dtype=dt, shape=(rows, k))
    c = _ctx(ctx, X.device.index or 0)
    o = default_opts(algo=algo, eps_mu=eps_mu, max_pivots=max_pivots)
    piv = ctypes.c_longlong(0)
    code = _lib.ALGOS[algo.lower()] if isinstance(algo, str) else int(algo)
    c.check(_lib.lib().nmf_update(c.handle, code, _dtype_code(X), rows, k, _dev(G, "G"),
                                _dev(P, "P"), _dev(X, "X"), ctypes.byref(o), ctypes.byref(piv)))
    return piv.value


def nmf_update_noalloc(algo, G, P, X, eps_mu=1e-16, max_pivots=0, ctx=None):
    """nmf_update on the library's fixed device scratch (no allocation);
    rejects sizes past NMF_NOALLOC_SCRATCH_BYTES with NMFError."""
    rows, k = X.shape
    dt = X.dtype
    _dev(G, "G", dtype=dt, shape=(k, k))
    _dev(P, "P", dtype=dt, shape=(rows, k))
    c = _ctx(ctx, X.device.index or 0)
    o = default_opts(algo=algo, eps_mu=eps_mu, max_pivots=max_pivots)
    piv = ctypes.c_longlong(0)
    code = _lib.ALGOS[algo.lower()] if isinstance(algo, str) else int(algo)
    c.check(_lib.lib().nmf_update_noalloc(c.handle, code, _dtype_code(X), rows, k, _dev(G, "G"),
                                          _dev(P, "P"), _dev(X, "X"), ctypes.byref(o),
                                          ctypes.byref(piv)))
    return piv.value


def nmf_hals_normalize(W, Ht, ctx=None):
    """HALS column normalisation of W (m x k) compensated in Ht (n x k), in
    place. Returns (S = W^T W of the normalised W, norms)."""
    torch = _torch()
    m, k = W.shape
    n = Ht.shape[0]
    _dev(Ht, "Ht", dtype=W.dtype, shape=(n, k))
    S = torch.empty((k, k), dtype=W.dtype, device=W.device)
    norms = torch.empty(k, dtype=W.dtype, device=W.device)
    c = _ctx(ctx, W.device.index or 0)
    c.check(_lib.lib().nmf_hals_normalize(c.handle, _dtype_code(W), m, n, k, _dev(W, "W"),
                                        _dev(Ht, "Ht"), _dev(S, "S"), _dev(norms, "norms")))
    return S, norms


def nmf_dense_relerr(A, W, Ht, ctx=None):
    """||A - W Ht^T||_F / ||A||_F for dense A."""
    m, n = A.shape
    k = W.shape[1]
    _dev(W, "W", dtype=_factor_dtype(A), shape=(m, k))
    _dev(Ht, "Ht", dtype=_factor_dtype(A), shape=(n, k))
    out = ctypes.c_double(0.0)
    c = _ctx(ctx, A.device.index or 0)
    c.check(_lib.lib().nmf_dense_relerr(c.handle, _dtype_code(A), m, n, _dev(A, "A"), A.stride(0),
                                      k, _dev(W, "W"), _dev(Ht, "Ht"), ctypes.byref(out)))
    return out.value


def nmf_projected_gradient_sq(X, P, G, ctx=None):
    """Sum of squares of the projected gradient in the factor whose rows are
    X (rows x k), given its product P (rows x k) and the Gram G (k x k) of
    the other factor."""
    rows, k = X.shape
    _dev(P, "P", dtype=X.dtype, shape=(rows, k))
    _dev(G, "G", dtype=X.dtype, shape=(k, k))
    out = ctypes.c_double(0.0)
    c = _ctx(ctx, X.device.index or 0)
    c.check(_lib.lib().nmf_projected_gradient_sq(c.handle, _dtype_code(X), rows, k, _dev(X, "X"),
                                               _dev(P, "P"), _dev(G, "G"), ctypes.byref(out)))
    return out.value


def nmf_csr_relerr(rowptr, colidx, vals, n, W, Ht, ctx=None):
    """||A - W Ht^T||_F / ||A||_F for CSR A (float32)."""
    torch = _torch()
    m = rowptr.numel() - 1
    k = W.shape[1]
    out = ctypes.c_double(0.0)
    c = _ctx(ctx, W.device.index or 0)
    c.check(_lib.lib().nmf_csr_relerr(c.handle, m, n, colidx.numel(),
                                    _dev(rowptr, "rowptr", dtype=torch.int64),
                                    _dev(colidx, "colidx", dtype=torch.int32),
                                    _dev(vals, "vals", dtype=torch.float32), k,
                                    _dev(W, "W", dtype=torch.float32, shape=(m, k)),
                                    _dev(Ht, "Ht", dtype=torch.float32, shape=(n, k)),
                                    ctypes.byref(out)))
    return out.value


# ---- differentiation through unrolled MU iterations ----------------------

def nmf_mu_unrolled_forward(A, W0, H0, iters, eps=1e-16, ckpt_every=10, want_ckpt=True,
                            ctx=None):
    """T = iters MU iterations from (W0, H0) (not modified). Returns
    (W_T, H_T, ckpt) where ckpt (or None) feeds nmf_mu_unrolled_backward."""
    torch = _torch()
    m, n = A.shape
    k = W0.shape[1]
    _dev(A, "A")
    _dev(W0, "W0", dtype=A.dtype, shape=(m, k))
    _dev(H0, "H0", dtype=A.dtype, shape=(k, n))
    W = W0.clone()
    H = H0.clone()
    ckpt = None
    if want_ckpt:
        ne = _lib.lib().nmf_mu_ckpt_elems(m, n, k, iters, ckpt_every)
        if ne < 0:
            raise ValueError("invalid sizes for the unrolled MU gradient")
        ckpt = torch.empty(max(ne, 1), dtype=A.dtype, device=A.device)
    c = _ctx(ctx, A.device.index or 0)
    c.check(_lib.lib().nmf_mu_unrolled_forward(
        c.handle, _dtype_code(A), m, n, _dev(A, "A"), A.stride(0), k, iters, float(eps),
        ckpt_every, _dev(W, "W"), _dev(H, "H"),
        _dev(ckpt, "ckpt") if ckpt is not None else None))
    return W, H, ckpt


def nmf_mu_unrolled_backward(A, ckpt, gW, gH, iters, eps=1e-16, ckpt_every=10, want_gA=True,
                             ctx=None):
    """(dL/dA or None, dL/dW0, dL/dH0) from dL/dW_T = gW and dL/dH_T = gH."""
    torch = _torch()
    m, n = A.shape
    k = gW.shape[1]
    _dev(gW, "gW", dtype=A.dtype, shape=(m, k))
    _dev(gH, "gH", dtype=A.dtype, shape=(k, n))
    gA = torch.empty((m, n), dtype=A.dtype, device=A.device) if want_gA else None
    gW0 = torch.empty((m, k), dtype=A.dtype, device=A.device)
    gH0 = torch.empty((k, n), dtype=A.dtype, device=A.device)
    c = _ctx(ctx, A.device.index or 0)
    c.check(_lib.lib().nmf_mu_unrolled_backward(
        c.handle, _dtype_code(A), m, n, _dev(A, "A"), A.stride(0), k, iters, float(eps),
        ckpt_every, _dev(ckpt, "ckpt"), _dev(gW, "gW"), _dev(gH, "gH"),
        _dev(gA, "gA") if gA is not None else None, n, _dev(gW0, "gW0"), _dev(gH0, "gH0")))
    return gA, gW0, gH0


def nmf_hals_unrolled_forward(A, W0, H0, iters, ckpt_every=10, want_ckpt=True, ctx=None):
    """T = iters HALS iterations from (W0, H0) (not modified), as nmf_dense
    runs them. Returns (W_T, H_T, ckpt) where ckpt (or None) feeds
    nmf_hals_unrolled_backward."""
    torch = _torch()
    m, n = A.shape
    k = W0.shape[1]
    _dev(A, "A")
    _dev(W0, "W0", dtype=A.dtype, shape=(m, k))
    _dev(H0, "H0", dtype=A.dtype, shape=(k, n))
    W = W0.clone()
    H = H0.clone()
    ckpt = None
    if want_ckpt:
        ne = _lib.lib().nmf_mu_ckpt_elems(m, n, k, iters, ckpt_every)
        if ne < 0:
            raise ValueError("invalid sizes for the unrolled HALS gradient")
        ckpt = torch.empty(max(ne, 1), dtype=A.dtype, device=A.device)
    c = _ctx(ctx, A.device.index or 0)
    c.check(_lib.lib().nmf_hals_unrolled_forward(
        c.handle, _dtype_code(A), m, n, _dev(A, "A"), A.stride(0), k, iters, ckpt_every,
        _dev(W, "W"), _dev(H, "H"), _dev(ckpt, "ckpt") if ckpt is not None else None))
    return W, H, ckpt


def nmf_hals_unrolled_backward(A, ckpt, gW, gH, iters, ckpt_every=10, want_gA=True, ctx=None):
    """(dL/dA or None, dL/dW0, dL/dH0) of the HALS map from dL/dW_T = gW and
    dL/dH_T = gH."""
    torch = _torch()
    m, n = A.shape
    k = gW.shape[1]
    _dev(gW, "gW", dtype=A.dtype, shape=(m, k))
    _dev(gH, "gH", dtype=A.dtype, shape=(k, n))
    gA = torch.empty((m, n), dtype=A.dtype, device=A.device) if want_gA else None
    gW0 = torch.empty((m, k), dtype=A.dtype, device=A.device)
    gH0 = torch.empty((k, n), dtype=A.dtype, device=A.device)
    c = _ctx(ctx, A.device.index or 0)
    c.check(_lib.lib().nmf_hals_unrolled_backward(
        c.handle, _dtype_code(A), m, n, _dev(A, "A"), A.stride(0), k, iters, ckpt_every,
        _dev(ckpt, "ckpt"), _dev(gW, "gW"), _dev(gH, "gH"),
        _dev(gA, "gA") if gA is not None else None, n, _dev(gW0, "gW0"), _dev(gH0, "gH0")))
    return gA, gW0, gH0


def _hals_unrolled_function():
    torch = _torch()

    class HALSUnrolled(torch.autograd.Function):
        """T unrolled HALS iterations as a differentiable layer: forward and
        backward both run in the library (checkpoints every ckpt_every
        iterations, segments recomputed in the backward pass)."""

        @staticmethod
        def forward(fctx, A, W0, H0, iters, ckpt_every):
            A, W0, H0 = A.contiguous(), W0.contiguous(), H0.contiguous()
            W, H, ckpt = nmf_hals_unrolled_forward(A, W0, H0, iters, ckpt_every)
            fctx.save_for_backward(A, ckpt)
            fctx.meta = (iters, ckpt_every, W0.shape, H0.shape)
            return W, H

        @staticmethod
        def backward(fctx, gW, gH):
            A, ckpt = fctx.saved_tensors
            iters, ckpt_every, ws, hs = fctx.meta
            gW = torch.zeros(ws, dtype=A.dtype, device=A.device) if gW is None else gW.contiguous()
            gH = torch.zeros(hs, dtype=A.dtype, device=A.device) if gH is None else gH.contiguous()
            gA, gW0, gH0 = nmf_hals_unrolled_backward(A, ckpt, gW, gH, iters, ckpt_every,
                                                      want_gA=fctx.needs_input_grad[0])
            return gA, gW0, gH0, None, None

    return HALSUnrolled


_HALS_FN = None


def hals_unrolled(A, W0, H0, iters, ckpt_every=10):
    """Differentiable (W_T, H_T) = T HALS iterations from (W0, H0) on dense A."""
    global _HALS_FN
    if _HALS_FN is None:
        _HALS_FN = _hals_unrolled_function()
    return _HALS_FN.apply(A, W0, H0, iters, ckpt_every)


def _mu_unrolled_function():
    torch = _torch()

    class MUUnrolled(torch.autograd.Function):
        """T unrolled MU iterations as a differentiable layer: forward and
        backward both run in the library (checkpoints every ckpt_every
        iterations, segments recomputed in the backward pass)."""

        @staticmethod
        def forward(fctx, A, W0, H0, iters, eps, ckpt_every):
            A, W0, H0 = A.contiguous(), W0.contiguous(), H0.contiguous()
            W, H, ckpt = nmf_mu_unrolled_forward(A, W0, H0, iters, eps, ckpt_every)
            fctx.save_for_backward(A, ckpt)
            fctx.meta = (iters, eps, ckpt_every, W0.shape, H0.shape)
            return W, H

        @staticmethod
        def backward(fctx, gW, gH):
            A, ckpt = fctx.saved_tensors
            iters, eps, ckpt_every, ws, hs = fctx.meta
            gW = torch.zeros(ws, dtype=A.dtype, device=A.device) if gW is None else gW.contiguous()
            gH = torch.zeros(hs, dtype=A.dtype, device=A.device) if gH is None else gH.contiguous()
            gA, gW0, gH0 = nmf_mu_unrolled_backward(A, ckpt, gW, gH, iters, eps, ckpt_every,
                                                    want_gA=fctx.needs_input_grad[0])
            return gA, gW0, gH0, None, None, None

    return MUUnrolled


_MU_FN = None


def mu_unrolled(A, W0, H0, iters, eps=1e-16, ckpt_every=10):
    """Differentiable (W_T, H_T) = T MU iterations from (W0, H0) on dense A."""
    global _MU_FN
    if _MU_FN is None:
        _MU_FN = _mu_unrolled_function()
    return _MU_FN.apply(A, W0, H0, iters, eps, ckpt_every)
