"""Barabasi-Albert graphs through the small C generator in ``ba.c``.

The shared library is compiled in place with gcc the first time it is
needed (``build_ba()`` does it eagerly).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ba.c")
_LIB = os.path.join(_HERE, "libgraphgen_ba.so")
_lib = None


def build_ba() -> str:
    subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-o", _LIB, _SRC])
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build_ba()
        lib = ctypes.CDLL(_LIB)
        lib.graphgen_ba_edges.restype = ctypes.c_int64
        lib.graphgen_ba_edges.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64,
                                          ctypes.c_void_p, ctypes.c_void_p]
        _lib = lib
    return _lib


def barabasi_albert(n: int, m: int = 8, seed: int = 0):
    from . import from_edges
    cap = m * (m + 1) // 2 + (n - m - 1) * m
    src = np.empty(cap, dtype=np.int32)
    dst = np.empty(cap, dtype=np.int32)
    ne = _load().graphgen_ba_edges(n, m, seed, src.ctypes.data, dst.ctypes.data)
    if ne != cap:
        raise RuntimeError("Barabasi-Albert generator failed")
    return from_edges(n, src, dst, name=f"ba-{n}-m{m}-s{seed}")
