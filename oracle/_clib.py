"""Builds (on demand) and loads the plain-C FP64 loops of oracle/ct_oracle.c.
Test infrastructure only."""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ct_oracle.c")
_SO = os.path.join(_HERE, "libct_oracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle loops with gcc (-O3, OpenMP threads and simd lanes for AVX2
    machines, glibc's vector exp; IEEE double semantics: no fast-math, no FMA
    contraction)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-march=x86-64-v3", "-fno-math-errno",
                               "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               _SRC, "-o", tmp, "-lmvec", "-lm"])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        D = ctypes.POINTER(ctypes.c_double)
        I64 = ctypes.c_int64
        _lib.orc_lse.argtypes = [ctypes.c_int, I64, D, I64, D, D, ctypes.c_double, D, D]
        _lib.orc_lse.restype = None
        _lib.orc_svgd_phi.argtypes = [ctypes.c_int, I64, D, D, ctypes.c_double, D]
        _lib.orc_svgd_phi.restype = None
        _lib.orc_pair_count.argtypes = [ctypes.c_int, I64, D, ctypes.c_double,
                                        ctypes.POINTER(I64), ctypes.POINTER(I64)]
        _lib.orc_pair_count.restype = None
    return _lib


def dptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))
