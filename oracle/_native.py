"""Build and load the oracle's plain-C vector core (``ftk_oracle.c``).

Test infrastructure only (see ``oracle/__init__``).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ftk_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# -ffp-contract=off: no fused multiply-add except the explicit fma() calls.
CFLAGS = ["-O2", "-fPIC", "-shared", "-fopenmp", "-mfma", "-ffp-contract=off", "-fno-fast-math"]


def build():
    cmd = ["gcc", *CFLAGS, "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)


_lib = None

_d = ctypes.c_double
_i = ctypes.c_int
_i64 = ctypes.c_int64
_u64 = ctypes.c_uint64
_p = ctypes.c_void_p


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        L.orc_dot_re.restype = _d
        L.orc_dot_re.argtypes = [_i64, _p, _p]
        L.orc_hv.restype = None
        L.orc_hv.argtypes = [_i, _i, _p, _p, _p, _d, _d, _p, _p, _p, _p]
        L.orc_hv_at.restype = None
        L.orc_hv_at.argtypes = [_i, _i, _p, _p, _p, _d, _d, _p, _p, _p, _i64, _p, _p]
        L.orc_lanczos.restype = _i
        L.orc_lanczos.argtypes = [_i, _i, _p, _p, _p, _d, _d, _p, _p, _p, _i, _d, _p, _p, _p, _p]
        L.orc_lanczos_combine.restype = _i
        L.orc_lanczos_combine.argtypes = [_i, _i, _p, _p, _p, _d, _d, _p, _p, _p, _i, _d, _p, _p, _p, _i, _p, _p]
        L.orc_combine.restype = None
        L.orc_combine.argtypes = [_i, _i, _i, _p, _p, _p]
        L.orc_apply_sq.restype = None
        L.orc_apply_sq.argtypes = [_i, _i, _p, _p, _p]
        L.orc_taylor_term.restype = None
        L.orc_taylor_term.argtypes = [_i, _i, _p, _p, _p, _d, _d, _p, _p, _p, _p, _p, _d, _d]
        L.orc_scale.restype = None
        L.orc_scale.argtypes = [_i64, _p, _d]
        L.orc_gaussian.restype = None
        L.orc_gaussian.argtypes = [_u64, _u64, _i, _p]
        L.orc_splitmix64.restype = _u64
        L.orc_splitmix64.argtypes = [_u64, _u64]
        L.orc_lanczos_bilinear.restype = _i
        L.orc_lanczos_bilinear.argtypes = [_i, _i, _p, _p, _p, _d, _d, _p, _p, _p, _p, _i, _d, _p, _p, _p, _p,
                                           _p]
        L.orc_num_threads.restype = _i
        L.orc_num_threads.argtypes = []
        _lib = L
    return _lib


def ptr(a):
    """Address of a C-contiguous numpy array."""
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


def cvec(n_sites):
    """A zeroed complex vector of dimension 2^N as an interleaved float64 array."""
    return np.zeros(2 << n_sites, dtype=np.float64)


def as_f64(v):
    """View a complex128 array as interleaved float64 (copy only if needed)."""
    v = np.ascontiguousarray(v)
    if v.dtype == np.complex128:
        return v.view(np.float64)
    return np.ascontiguousarray(v, dtype=np.float64)
