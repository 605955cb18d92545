"""Builds and loads the C pulse-accumulation core of the RF generator."""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "simcore.c")
_LIB = os.path.join(_HERE, "libsimcore.so")
_lib = None


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-o", tmp, _SRC,
                               "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        # worker threads sleep rather than spin between calls, so a caller timing
        # other work right after a simulation does not share the CPUs with them
        os.environ.setdefault("OMP_WAIT_POLICY", "PASSIVE")
        _lib = ctypes.CDLL(_LIB)
        _lib.sim_accumulate.restype = None
        _lib.sim_accumulate.argtypes = [
            ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
            ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_void_p]
    return _lib


def accumulate(t: np.ndarray, amp: np.ndarray, n_samp: int, fs: float, f0: float,
               sigma: float, trunc: float) -> np.ndarray:
    """RF rows [n_rows][n_samp] from arrival times ``t`` [n_rows][n_scat]."""
    t = np.ascontiguousarray(t, dtype=np.float64)
    amp = np.ascontiguousarray(amp, dtype=np.float64)
    n_rows, n_scat = t.shape
    assert amp.shape == (n_scat,)
    out = np.zeros((n_rows, n_samp), dtype=np.float64)
    lib().sim_accumulate(n_rows, n_samp, n_scat, t.ctypes.data, amp.ctypes.data, fs, f0,
                         sigma, trunc, out.ctypes.data)
    return out
