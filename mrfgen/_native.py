"""Builds and loads the small C helper (EPG simulator) of the input generator."""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "epg.c")
_LIB = os.path.join(_HERE, "_epg.so")
_lib = None


def build(force=False):
    """Compile epg.c with gcc (OpenMP) into mrfgen/_epg.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = ctypes.CDLL(_LIB)
        f = _lib.mrfgen_epg_fisp
        dp = ctypes.POINTER(ctypes.c_double)
        f.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp, dp, dp, dp,
                      ctypes.c_double, ctypes.POINTER(ctypes.c_float)]
        f.restype = None
    return _lib


def epg_fisp(t1, t2, fa_deg, tr_ms, te_ms, n_states=24, b1=None):
    """Simulate FISP fingerprints; returns complex64 [n_atoms, L]."""
    t1 = np.ascontiguousarray(t1, np.float64)
    t2 = np.ascontiguousarray(t2, np.float64)
    fa = np.ascontiguousarray(fa_deg, np.float64)
    tr = np.ascontiguousarray(tr_ms, np.float64)
    n, L = t1.size, fa.size
    out = np.empty((n, L), np.complex64)
    dp = ctypes.POINTER(ctypes.c_double)
    b1p = None
    if b1 is not None:
        b1 = np.ascontiguousarray(b1, np.float64)
        b1p = b1.ctypes.data_as(dp)
    lib().mrfgen_epg_fisp(n, L, n_states, t1.ctypes.data_as(dp), t2.ctypes.data_as(dp), b1p,
                          fa.ctypes.data_as(dp), tr.ctypes.data_as(dp), float(te_ms),
                          out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
    return out
