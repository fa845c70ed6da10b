"""Build and load the oracle's C core (test infrastructure only)."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wigner_oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle core with gcc (plain C, OpenMP, FP64)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        cmd = ["gcc", "-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared",
               "-std=c11", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        L = ctypes.CDLL(_SO)
        dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
        ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
        L.oracle_delta_size.restype = ctypes.c_size_t
        L.oracle_delta_size.argtypes = [ctypes.c_int]
        L.oracle_delta_offset.restype = ctypes.c_size_t
        L.oracle_delta_offset.argtypes = [ctypes.c_int]
        L.oracle_delta_table.restype = None
        L.oracle_delta_table.argtypes = [ctypes.c_int, dp]
        L.oracle_delta_get.restype = ctypes.c_double
        L.oracle_delta_get.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.oracle_wigner_fourier.restype = None
        L.oracle_wigner_fourier.argtypes = [ctypes.c_int, ctypes.c_int, ip, ctypes.c_int, ip, dp, dp, dp]
        L.oracle_wigner_project.restype = None
        L.oracle_wigner_project.argtypes = [ctypes.c_int, ctypes.c_int, ip, ctypes.c_int, ip, dp, dp, dp]
        L.oracle_wigner_d_sum.restype = ctypes.c_double
        L.oracle_wigner_d_sum.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double]
        _lib = L
    return _lib
