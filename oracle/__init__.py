"""CPU oracle for the row/column-sampling Monte Carlo estimator of f(sA).

TEST INFRASTRUCTURE ONLY.  The test-suite, the smoke check and the benchmark's
CPU-baseline leg use it to check the GPU library; the library itself never
imports, links or calls anything here, and nothing here imports the library.

Two parts:

* ``mcmf_oracle.c`` (loaded through ctypes): the estimator written out step
  by step -- RandFunmAction (Section 3.4, Algorithm 3) and RandFunmDiag
  (Section 3.3, Eq. rand_funm_formula_diag) -- replaying the Philox walks, plus
  an exact-expectation mode that propagates the walk distribution instead of
  sampling it.
* :func:`dense_series` (numpy): the truncated power series
  sum_{k<=K} c_k (sA)^k by Horner's rule, for small dense checks.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mcmf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

FN_EXP = 0
FN_RESOLVENT = 1

_ERRORS = {1: "invalid argument", 2: "matrix is not symmetric", 3: "out of memory"}


class OracleError(RuntimeError):
    pass


def build() -> str:
    """Compile the oracle in place (gcc, no FMA contraction)."""
    subprocess.check_call(["gcc", "-std=gnu99", "-O2", "-ffp-contract=off", "-fno-fast-math",
                           "-Wall", "-shared", "-fPIC", "-o", _LIB, _SRC, "-lm"])
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    _lib = _open(_LIB)
    return _lib


def _swap_library(path: Optional[str]):
    """Use the oracle library at ``path`` (None: the default build) and return
    the previously active one.  The test-suite uses it to run the pins
    against deliberately broken copies of the oracle."""
    global _lib
    prev = _lib
    _lib = None if path is None else _open(path)
    return prev


def _open(path: str):
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i64, u64, u32, i32, f64, cint = (ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32,
                                     ctypes.c_int32, ctypes.c_double, ctypes.c_int)
    lib.oracle_philox4x32_10.argtypes = [P, P, P]
    lib.oracle_philox4x32_10.restype = None
    lib.oracle_philox4x64_10.argtypes = [P, P, P]
    lib.oracle_philox4x64_10.restype = None
    lib.oracle_uniform_index.argtypes = [u64, i64]
    lib.oracle_uniform_index.restype = i64
    lib.oracle_select_next.argtypes = [i64, P, P, P, i64, u64, u64]
    lib.oracle_select_next.restype = i64
    lib.oracle_set_alias.argtypes = [cint]
    lib.oracle_set_alias.restype = None
    lib.oracle_alias_table.argtypes = [i64, P, P, P, P, P]
    lib.oracle_alias_table.restype = cint
    lib.oracle_is_symmetric.argtypes = [i64, P, P, P]
    lib.oracle_is_symmetric.restype = cint
    lib.oracle_coeffs.argtypes = [cint, cint, P]
    lib.oracle_coeffs.restype = cint
    lib.oracle_action.argtypes = [i64, P, P, P, P, cint, f64, i64, u64, u32, f64, P, P, i64,
                                  cint, P, P, P, P, P]
    lib.oracle_action.restype = cint
    lib.oracle_diag.argtypes = [i64, P, P, P, P, cint, f64, i64, u64, u32, f64, P, i64, cint,
                                cint, P, P, P, P]
    lib.oracle_diag.restype = cint
    lib.oracle_allocation.argtypes = [i64, P, P, P, cint, P, i64, i64, cint, P]
    lib.oracle_allocation.restype = cint
    return lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def _csr_arrays(g):
    row_ptr = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    val = None if g.val is None else np.ascontiguousarray(g.val, dtype=np.float64)
    return row_ptr, col, val


def _check(rc: int):
    if rc != 0:
        raise OracleError(_ERRORS.get(rc, f"oracle error {rc}"))


# ---------------------------------------------------------------- primitives

def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _load().oracle_philox4x32_10(c.ctypes.data, k.ctypes.data, out.ctypes.data)
    return out


def philox4x64_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    _load().oracle_philox4x64_10(c.ctypes.data, k.ctypes.data, out.ctypes.data)
    return out


def uniform_index(u: int, deg: int) -> int:
    return int(_load().oracle_uniform_index(u, deg))


def select_next(g, row: int, u: int, u2: int = 0, sampler: str = "cdf") -> int:
    """Index in row ``row`` of the next state for random words u (and u2,
    the alias method's second word)."""
    row_ptr, col, val = _csr_arrays(g)
    with _sampler(sampler):
        return int(_load().oracle_select_next(g.n, _ptr(row_ptr), _ptr(col), _ptr(val), row, u, u2))


def alias_table(g):
    """The alias method's tables of a weighted graph: (prob float64[nnz],
    alias int64[nnz], alias given as an index inside the row)."""
    row_ptr, col, val = _csr_arrays(g)
    nnz = int(row_ptr[-1])
    prob = np.zeros(max(nnz, 1), dtype=np.float64)
    alias = np.zeros(max(nnz, 1), dtype=np.int64)
    _check(_load().oracle_alias_table(g.n, _ptr(row_ptr), _ptr(col), _ptr(val), _ptr(prob), _ptr(alias)))
    return prob[:nnz], alias[:nnz]


class _sampler:
    """Weighted rows sample by running sums ("cdf") or by alias tables
    ("alias") inside the block; unweighted rows are not affected."""

    def __init__(self, kind: str):
        if kind not in ("cdf", "alias"):
            raise OracleError(f"unknown sampler {kind!r}")
        self.on = kind == "alias"

    def __enter__(self):
        _load().oracle_set_alias(1 if self.on else 0)

    def __exit__(self, *exc):
        _load().oracle_set_alias(0)


def is_symmetric(g) -> bool:
    row_ptr, col, val = _csr_arrays(g)
    r = _load().oracle_is_symmetric(g.n, _ptr(row_ptr), _ptr(col), _ptr(val))
    if r < 0:
        raise OracleError("out of memory")
    return bool(r)


def coeffs(kind: int, K: int) -> np.ndarray:
    c = np.zeros(K + 1, dtype=np.float64)
    _check(_load().oracle_coeffs(kind, K, c.ctypes.data))
    return c


def _coeff_array(fn, K: int) -> np.ndarray:
    if isinstance(fn, (int, np.integer)):
        return coeffs(int(fn), K)
    c = np.ascontiguousarray(fn, dtype=np.float64)
    if c.size < K + 1:
        raise OracleError("need K+1 coefficients")
    return c


# ---------------------------------------------------------------- estimators

def _walks_array(walks, n):
    if walks is None:
        return None
    w = np.ascontiguousarray(walks, dtype=np.int64)
    if w.size != n:
        raise OracleError("walks must have length n")
    return w


def allocation(g, Ns: int, starts, symmetric: bool = True, min_one: bool = False):
    """Walks per start row with p_k proportional to ||C_k||_2 (Eq.
    initial_prob): N_k = round(Ns p_k), which may be 0 (Algorithms 2-3), or
    max(1, round(Ns p_k)) with ``min_one``; int64[n], 0 off the starts."""
    row_ptr, col, val = _csr_arrays(g)
    st = np.ascontiguousarray(starts, dtype=np.int32)
    out = np.zeros(max(g.n, 1), dtype=np.int64)
    _check(_load().oracle_allocation(g.n, _ptr(row_ptr), _ptr(col), _ptr(val), 1 if symmetric else 0,
                                     _ptr(st), st.size, int(Ns), 1 if min_one else 0, _ptr(out)))
    return out[:g.n]


def action(g, fn, v, N: int, K: int, scale: float = 1.0, seed: int = 0, request: int = 0,
           cutoff: float = 0.0, rows=None, expect: bool = False, want_q: bool = False,
           want_digest: bool = False, walks=None, sampler: str = "cdf"):
    """RandFunmAction.  Returns dict(y, q, digest, steps).

    ``fn``: FN_EXP, FN_RESOLVENT or an explicit coefficient array c_0..c_K.
    ``rows``: output rows (default all); walks start only where needed.
    ``expect``: exact expectation of the estimator instead of sampling.
    ``walks``: walks per start row (int64[n]) instead of N for every row; a
    row given 0 starts no walk.
    ``sampler``: "cdf" (running sums) or "alias" for weighted rows.
    """
    row_ptr, col, val = _csr_arrays(g)
    c = _coeff_array(fn, K)
    v = np.ascontiguousarray(v, dtype=np.float64)
    if v.size != g.n:
        raise OracleError("v must have length n")
    out_rows = None if rows is None else np.ascontiguousarray(rows, dtype=np.int32)
    n_out = g.n if out_rows is None else out_rows.size
    y = np.zeros(max(n_out, 1), dtype=np.float64)
    q = np.zeros(max(g.n, 1), dtype=np.float64) if want_q else None
    dig = np.zeros(max(g.n, 1), dtype=np.uint64) if want_digest else None
    steps = ctypes.c_uint64(0)
    with _sampler(sampler):
        _check(_load().oracle_action(g.n, _ptr(row_ptr), _ptr(col), _ptr(val), _ptr(c), K,
                                     float(scale), int(N), int(seed), int(request), float(cutoff),
                                     _ptr(v), _ptr(out_rows), 0 if out_rows is None else out_rows.size,
                                     1 if expect else 0, _ptr(y), _ptr(q), _ptr(dig),
                                     ctypes.addressof(steps), _ptr(_walks_array(walks, g.n))))
    return {"y": y[:n_out], "q": None if q is None else q[:g.n],
            "digest": None if dig is None else dig[:g.n], "steps": steps.value}


def diag(g, fn, N: int, K: int, scale: float = 1.0, seed: int = 0, request: int = 0,
         cutoff: float = 0.0, rows=None, expect: bool = False, assume_symmetric: bool = False,
         want_digest: bool = False, walks=None, sampler: str = "cdf"):
    """RandFunmDiag.  Returns dict(d, digest, steps).  ``walks``: walks per
    start row (int64[n]) instead of N for every row; a row given 0 starts no
    walk.  ``sampler``: "cdf" (running sums) or "alias" for weighted rows."""
    row_ptr, col, val = _csr_arrays(g)
    c = _coeff_array(fn, K)
    r = None if rows is None else np.ascontiguousarray(rows, dtype=np.int32)
    count = g.n if r is None else r.size
    d = np.zeros(max(count, 1), dtype=np.float64)
    dig = np.zeros(max(g.n, 1), dtype=np.uint64) if want_digest else None
    steps = ctypes.c_uint64(0)
    with _sampler(sampler):
        _check(_load().oracle_diag(g.n, _ptr(row_ptr), _ptr(col), _ptr(val), _ptr(c), K,
                                   float(scale), int(N), int(seed), int(request), float(cutoff),
                                   _ptr(r), 0 if r is None else r.size, 1 if assume_symmetric else 0,
                                   1 if expect else 0, _ptr(d), _ptr(dig), ctypes.addressof(steps),
                                   _ptr(_walks_array(walks, g.n))))
    return {"d": d[:count], "digest": None if dig is None else dig[:g.n], "steps": steps.value}


# ---------------------------------------------------------------- dense check

def dense_series(a: np.ndarray, c, scale: float = 1.0) -> np.ndarray:
    """sum_{k=0}^{K} c_k (scale*A)^k by Horner's rule (K = len(c)-1)."""
    b = scale * np.asarray(a, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    out = c[-1] * np.eye(b.shape[0])
    for ck in c[-2::-1]:
        out = b @ out + ck * np.eye(b.shape[0])
    return out
