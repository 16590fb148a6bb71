"""ctypes binding of libnmf_mi355x.so (include/nmf.h).

Argument marshalling only: torch tensors supply device pointers and the HIP
stream, every computation happens in the library's HIP kernels. If the
library is missing, the first call raises ImportError; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnmf_mi355x.so")

NMF_OK, NMF_EINVAL, NMF_ENOMEM, NMF_EDEVICE, NMF_ENUMERIC, NMF_ENOTCONV = range(6)
NMF_MU, NMF_HALS, NMF_ABPP = 0, 1, 2
NMF_F64, NMF_F32, NMF_BF16, NMF_FP8_E4M3 = 0, 1, 2, 3
NMF_OBJ_NONE, NMF_OBJ_DIRECT = 0, 1
NMF_NOALLOC_SCRATCH_BYTES = 64 << 20
ALGOS = {"mu": NMF_MU, "hals": NMF_HALS, "abpp": NMF_ABPP}

# Every function the header declares, with its ctypes signature.
_i64 = ctypes.c_int64
_int = ctypes.c_int
_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)


STOPS = {"iters": 0, "pgrad": 1, "relerr": 2}


class NmfOpts(ctypes.Structure):
    _fields_ = [("algo", _int), ("iters", _int), ("eps_mu", ctypes.c_double),
                ("max_pivots", _int), ("objective", _int), ("timers", _int),
                ("check_input", _int), ("transpose_a", _int), ("tol", ctypes.c_double),
                ("stop", _int)]


class NmfStats(ctypes.Structure):
    _fields_ = [("ms_total", ctypes.c_double), ("ms_mm", ctypes.c_double),
                ("ms_luc", ctypes.c_double), ("ms_gram", ctypes.c_double),
                ("ms_obj", ctypes.c_double), ("ms_setup", ctypes.c_double),
                ("bpp_pivots", ctypes.c_longlong), ("ms_mm_aht", ctypes.c_double),
                ("ms_mm_wta", ctypes.c_double), ("iters_done", ctypes.c_longlong),
                ("pgrad_ratio", ctypes.c_double), ("bpp_solves", ctypes.c_longlong),
                ("bpp_flops", ctypes.c_double), ("bpp_size_mean", ctypes.c_double),
                ("bpp_size_max_mean", ctypes.c_double), ("bpp_size_class_mean", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


SIGNATURES = {
    "nmf_default_opts": (None, [ctypes.POINTER(NmfOpts)]),
    "nmf_create": (_int, [ctypes.POINTER(_vp), _int, _vp]),
    "nmf_destroy": (None, [_vp]),
    "nmf_set_stream": (_int, [_vp, _vp]),
    "nmf_status_str": (ctypes.c_char_p, [_int]),
    "nmf_last_error": (ctypes.c_char_p, [_vp]),
    "nmf_dense": (_int, [_vp, _int, _i64, _i64, _vp, _i64, _int, ctypes.POINTER(NmfOpts),
                         _vp, _vp, _dp, ctypes.POINTER(NmfStats)]),
    "nmf_csr": (_int, [_vp, _i64, _i64, _i64, _vp, _vp, _vp, _int, ctypes.POINTER(NmfOpts),
                       _vp, _vp, _dp, ctypes.POINTER(NmfStats)]),
    "nmf_gram": (_int, [_vp, _int, _i64, _int, _vp, _i64, _vp]),
    "nmf_dense_AF": (_int, [_vp, _int, _i64, _i64, _vp, _i64, _int, _vp, _i64, _vp]),
    "nmf_dense_AtF": (_int, [_vp, _int, _i64, _i64, _vp, _i64, _int, _vp, _i64, _vp]),
    "nmf_csr_AF": (_int, [_vp, _i64, _i64, _i64, _vp, _vp, _vp, _int, _vp, _vp]),
    "nmf_csr_transpose": (_int, [_vp, _i64, _i64, _i64, _vp, _vp, _vp, _vp, _vp, _vp]),
    "nmf_update": (_int, [_vp, _int, _int, _i64, _int, _vp, _vp, _vp, ctypes.POINTER(NmfOpts),
                          ctypes.POINTER(ctypes.c_longlong)]),
    "nmf_update_noalloc": (_int, [_vp, _int, _int, _i64, _int, _vp, _vp, _vp,
                                  ctypes.POINTER(NmfOpts), ctypes.POINTER(ctypes.c_longlong)]),
    "nmf_hals_normalize": (_int, [_vp, _int, _i64, _i64, _int, _vp, _vp, _vp, _vp]),
    "nmf_dense_relerr": (_int, [_vp, _int, _i64, _i64, _vp, _i64, _int, _vp, _vp, _dp]),
    "nmf_csr_relerr": (_int, [_vp, _i64, _i64, _i64, _vp, _vp, _vp, _int, _vp, _vp, _dp]),
    "nmf_projected_gradient_sq": (_int, [_vp, _int, _i64, _int, _vp, _vp, _vp, _dp]),
    "nmf_mu_ckpt_elems": (_i64, [_i64, _i64, _int, _int, _int]),
    "nmf_mu_unrolled_forward": (_int, [_vp, _int, _i64, _i64, _vp, _i64, _int, _int,
                                       ctypes.c_double, _int, _vp, _vp, _vp]),
    "nmf_mu_unrolled_backward": (_int, [_vp, _int, _i64, _i64, _vp, _i64, _int, _int,
                                        ctypes.c_double, _int, _vp, _vp, _vp, _vp, _i64, _vp,
                                        _vp]),
    "nmf_hals_unrolled_forward": (_int, [_vp, _int, _i64, _i64, _vp, _i64, _int, _int, _int,
                                         _vp, _vp, _vp]),
    "nmf_hals_unrolled_backward": (_int, [_vp, _int, _i64, _i64, _vp, _i64, _int, _int, _int,
                                          _vp, _vp, _vp, _vp, _i64, _vp, _vp]),
}


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError("HIP library %s is not built; run paper_1609_09154_amd.build.build()" % path)
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_LIB = None


def lib() -> ctypes.CDLL:
    """The loaded library (loaded on first use; raises if it is not built)."""
    global _LIB
    if _LIB is None:
        _LIB = load()
    return _LIB


class NMFError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        name = lib().nmf_status_str(status).decode()
        super().__init__("%s: %s" % (name, message))


def default_opts(**kw) -> NmfOpts:
    o = NmfOpts()
    lib().nmf_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if k == "algo" and isinstance(v, str):
            v = ALGOS[v.lower()]
        setattr(o, k, v)
    return o
