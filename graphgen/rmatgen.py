"""Large R-MAT graphs through the C generator in ``rmat.c`` (OpenMP).

Same construction as :func:`graphgen.rmat` (recursive quadrant choice with
probabilities a, b, c, d, random relabelling, symmetrised, deduplicated,
loop-free, isolated vertices kept), with its own splitmix64 streams, so the
two generators give different graphs of the same distribution.  Meant for
scales the numpy generator cannot hold (up to 2^26 nodes and 2^30 draws);
the shared library is compiled in place with gcc.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rmat.c")
_LIB = os.path.join(_HERE, "libgraphgen_rmat.so")
_lib = None


def build_rmat() -> str:
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", _LIB, _SRC])
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build_rmat()
        lib = ctypes.CDLL(_LIB)
        lib.graphgen_rmat_csr.restype = ctypes.c_int64
        lib.graphgen_rmat_csr.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                                          ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
        _lib = lib
    return _lib


def rmat_native(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19,
                c: float = 0.19, seed: int = 0, permute: bool = True):
    from . import CSR
    n = 1 << scale
    row_ptr = np.empty(n + 1, dtype=np.int64)
    col = np.empty(2 * edge_factor * n, dtype=np.int32)
    nnz = _load().graphgen_rmat_csr(scale, edge_factor, a, b, c, seed, 1 if permute else 0,
                                    row_ptr.ctypes.data, col.ctypes.data)
    if nnz < 0:
        raise RuntimeError("R-MAT generator failed (arguments or memory)")
    return CSR(n, row_ptr, col[:nnz], None, f"rmat-native-{scale}-ef{edge_factor}-s{seed}")
