"""Loader for the oracle's one C routine (test infrastructure only).

``build()`` compiles ``negacyclic.c`` with gcc into ``_oracle_native.so``
next to this file; ``lib()`` loads it.  Nothing here touches a GPU.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "negacyclic.c")
_SO = os.path.join(_HERE, "_oracle_native.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle C code (plain gcc, no GPU)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-mavx2", "-fPIC", "-shared",
                               "-o", tmp, _SRC])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        L = ctypes.CDLL(_SO)
        L.oracle_negacyclic_mac.argtypes = [ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_int64]
        L.oracle_negacyclic_mac.restype = None
        _lib = L
    return _lib


def negacyclic_mac(acc: np.ndarray, u: np.ndarray, K: np.ndarray) -> None:
    """acc += u * K in Z[X]/(X^N+1) mod 2^32 (in place).

    acc: uint32[N] (contiguous, modified), u: integer poly, K: uint32[N].
    """
    N = acc.shape[0]
    assert acc.dtype == np.uint32 and acc.flags.c_contiguous
    u32 = np.ascontiguousarray(u, dtype=np.int32)
    K32 = np.ascontiguousarray(K, dtype=np.uint32)
    assert u32.shape == (N,) and K32.shape == (N,)
    lib().oracle_negacyclic_mac(acc.ctypes.data, u32.ctypes.data,
                                K32.ctypes.data, N)
