"""ctypes binding of the C ABI declared in include/mcmf.h.

The functions here carry the C names and only marshal arguments: every step
of the computation runs in the HIP library ``libmcmf.so``.  Arrays may be
torch tensors (CUDA/HIP device or CPU) or numpy arrays; pointers are handed
to the library as they are, and the library tells host from device memory.

Importing this module fails with an ImportError if ``libmcmf.so`` has not
been built: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmcmf.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing; build it with `python -m paper_2308_01037_amd.build`")

# torch ships its own HIP runtime under the same soname; loading it first
# makes the library bind to that runtime, so torch's device pointers and
# streams are valid in both.
try:
    import torch  # noqa: F401
except ImportError:  # the library also works without torch
    torch = None

_lib = ctypes.CDLL(LIB_PATH)

# ---------------------------------------------------------------- constants

MCMF_OK = 0
MCMF_E_ARG = 1
MCMF_E_CSR = 2
MCMF_E_NOT_SYMMETRIC = 3
MCMF_E_NOMEM = 4
MCMF_E_DEVICE = 5
MCMF_E_UNSUPPORTED = 6

MCMF_FN_EXP = 0
MCMF_FN_RESOLVENT = 1
MCMF_FN_COEFFS = 2

MCMF_SYMMETRIC = 1
MCMF_VALIDATE = 2
MCMF_DIGRAPH = 4

MCMF_PRECISION_FP64 = 0
MCMF_PRECISION_FP32_WEIGHTS = 1

MCMF_ALLOC_PER_ROW = 0
MCMF_ALLOC_NORM = 1
MCMF_ALLOC_NORM_MIN1 = 2

MCMF_SAMPLER_EDGE = 0
MCMF_SAMPLER_ROW = 1
MCMF_SAMPLER_VALUE = 2
MCMF_SAMPLER_WIDE = 3
MCMF_SAMPLER_ALIAS = 4
MCMF_SAMPLER_AUTO = 5


class mcmf_fn(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("scale", ctypes.c_double),
                ("coeffs", ctypes.POINTER(ctypes.c_double)), ("n_coeffs", ctypes.c_int32)]


class mcmf_opts(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("request_id", ctypes.c_uint32),
                ("precision", ctypes.c_int32), ("weight_cutoff", ctypes.c_double),
                ("stream", ctypes.c_void_p), ("path_digest", ctypes.c_void_p),
                ("q_out", ctypes.c_void_p), ("walks_out", ctypes.c_void_p),
                ("allocation", ctypes.c_int32), ("reserved", ctypes.c_uint32 * 5)]


class mcmf_stats(ctypes.Structure):
    _fields_ = [("start_rows", ctypes.c_uint64), ("walks", ctypes.c_uint64),
                ("walk_steps", ctypes.c_uint64), ("gather_probes", ctypes.c_uint64),
                ("ms_setup", ctypes.c_double), ("ms_spmv", ctypes.c_double),
                ("ms_walk", ctypes.c_double), ("ms_gather", ctypes.c_double),
                ("ms_total", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class mcmf_tuning(ctypes.Structure):
    _fields_ = [("action_sampler", ctypes.c_int32), ("action_stream", ctypes.c_int32),
                ("diag_sampler", ctypes.c_int32), ("diag_stream", ctypes.c_int32),
                ("action_ms", ctypes.c_double * 4), ("diag_ms", ctypes.c_double * 4),
                ("sample_rows", ctypes.c_int64), ("hub_min_degree", ctypes.c_int32),
                ("hub_count", ctypes.c_int32), ("action_value_ms", ctypes.c_double * 2),
                ("walk_threads", ctypes.c_int32), ("gather_item", ctypes.c_int32),
                ("walk_threads_ms", ctypes.c_double * 3), ("gather_item_ms", ctypes.c_double * 4),
                ("hub_ms", ctypes.c_double * 2), ("wide_ms", ctypes.c_double),
                ("alias_ms", ctypes.c_double * 2), ("wide_hub_count", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {"action_sampler": self.action_sampler, "action_stream": self.action_stream,
                "diag_sampler": self.diag_sampler, "diag_stream": self.diag_stream,
                "action_ms": list(self.action_ms), "diag_ms": list(self.diag_ms),
                "sample_rows": self.sample_rows, "hub_min_degree": self.hub_min_degree,
                "hub_count": self.hub_count, "action_value_ms": list(self.action_value_ms),
                "walk_threads": self.walk_threads, "gather_item": self.gather_item,
                "walk_threads_ms": list(self.walk_threads_ms),
                "gather_item_ms": list(self.gather_item_ms), "hub_ms": list(self.hub_ms),
                "wide_ms": self.wide_ms, "alias_ms": list(self.alias_ms),
                "wide_hub_count": self.wide_hub_count}


MCMF_REQ_DIAG = 0
MCMF_REQ_ACTION = 1


class mcmf_request(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("K", ctypes.c_int32), ("graph", ctypes.c_void_p),
                ("fn", mcmf_fn), ("rows", ctypes.c_void_p), ("n_rows", ctypes.c_int64),
                ("v", ctypes.c_void_p), ("n_walks", ctypes.c_int64), ("seed", ctypes.c_uint64),
                ("request_id", ctypes.c_uint32), ("precision", ctypes.c_int32),
                ("weight_cutoff", ctypes.c_double), ("out", ctypes.c_void_p),
                ("path_digest", ctypes.c_void_p), ("status", ctypes.c_int),
                ("walk_steps", ctypes.c_uint64)]


class mcmf_batch_opts(ctypes.Structure):
    _fields_ = [("stream", ctypes.c_void_p), ("use_graph", ctypes.c_int32),
                ("reserved0", ctypes.c_int32), ("visit_chunk_bytes", ctypes.c_uint64),
                ("reserved", ctypes.c_uint32 * 4)]


class mcmf_server_opts(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("visit_chunk_bytes", ctypes.c_uint64),
                ("n_streams", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("device", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("max_batch_steps", ctypes.c_uint64), ("max_large_in_flight", ctypes.c_int32),
                ("reserved", ctypes.c_uint32 * 5)]


class mcmf_ticket_info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("batch_size", ctypes.c_int32),
                ("queue_ms", ctypes.c_double), ("run_ms", ctypes.c_double),
                ("est_bytes", ctypes.c_uint64), ("est_steps", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class mcmf_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("batches", ctypes.c_uint64), ("bytes_in_flight", ctypes.c_uint64),
                ("peak_bytes_in_flight", ctypes.c_uint64),
                ("peak_batches_in_flight", ctypes.c_uint64), ("largest_batch", ctypes.c_uint64),
                ("peak_large_in_flight", ctypes.c_uint64), ("reserved", ctypes.c_uint32 * 6)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "reserved"}


_P = ctypes.c_void_p
_lib.mcmf_graph_create.argtypes = [ctypes.c_int64, _P, _P, _P, ctypes.c_uint32, ctypes.POINTER(_P)]
_lib.mcmf_graph_create.restype = ctypes.c_int
_lib.mcmf_graph_destroy.argtypes = [_P]
_lib.mcmf_graph_destroy.restype = None
_lib.mcmf_graph_info.argtypes = [_P] + [ctypes.POINTER(ctypes.c_int64)] * 4
_lib.mcmf_graph_info.restype = ctypes.c_int
_lib.mcmf_diag.argtypes = [_P, ctypes.POINTER(mcmf_fn), _P, ctypes.c_int64, ctypes.c_int64,
                           ctypes.c_int32, ctypes.POINTER(mcmf_opts), _P, ctypes.POINTER(mcmf_stats)]
_lib.mcmf_diag.restype = ctypes.c_int
_lib.mcmf_action.argtypes = [_P, ctypes.POINTER(mcmf_fn), _P, ctypes.c_int64, ctypes.c_int32,
                             ctypes.POINTER(mcmf_opts), _P, ctypes.POINTER(mcmf_stats)]
_lib.mcmf_action.restype = ctypes.c_int
_lib.mcmf_action_noalloc.argtypes = [_P, ctypes.POINTER(mcmf_fn), _P, ctypes.c_int64, ctypes.c_int32,
                                     ctypes.POINTER(mcmf_opts), _P]
_lib.mcmf_action_noalloc.restype = ctypes.c_int
_lib.mcmf_batch.argtypes = [ctypes.POINTER(mcmf_request), ctypes.c_int64,
                            ctypes.POINTER(mcmf_batch_opts), ctypes.POINTER(mcmf_stats)]
_lib.mcmf_batch.restype = ctypes.c_int
_lib.mcmf_server_create.argtypes = [ctypes.POINTER(mcmf_server_opts), ctypes.POINTER(_P)]
_lib.mcmf_server_create.restype = ctypes.c_int
_lib.mcmf_server_submit.argtypes = [_P, ctypes.POINTER(mcmf_request), ctypes.POINTER(ctypes.c_uint64)]
_lib.mcmf_server_submit.restype = ctypes.c_int
_lib.mcmf_server_wait.argtypes = [_P, ctypes.c_uint64, ctypes.POINTER(mcmf_ticket_info)]
_lib.mcmf_server_wait.restype = ctypes.c_int
_lib.mcmf_server_query.argtypes = [_P, ctypes.POINTER(mcmf_server_stats)]
_lib.mcmf_server_query.restype = ctypes.c_int
_lib.mcmf_server_destroy.argtypes = [_P]
_lib.mcmf_server_destroy.restype = None
_lib.mcmf_graph_set_tuning.argtypes = [_P, ctypes.POINTER(mcmf_tuning)]
_lib.mcmf_graph_set_tuning.restype = ctypes.c_int
_lib.mcmf_graph_get_tuning.argtypes = [_P, ctypes.POINTER(mcmf_tuning)]
_lib.mcmf_graph_get_tuning.restype = ctypes.c_int
_lib.mcmf_tune.argtypes = [_P, ctypes.POINTER(mcmf_fn), ctypes.c_int64, ctypes.c_int32,
                           ctypes.POINTER(mcmf_tuning)]
_lib.mcmf_tune.restype = ctypes.c_int
_lib.mcmf_status_string.argtypes = [ctypes.c_int]
_lib.mcmf_status_string.restype = ctypes.c_char_p
_lib.mcmf_last_error.argtypes = []
_lib.mcmf_last_error.restype = ctypes.c_char_p

EXPORTED = ["mcmf_graph_create", "mcmf_graph_destroy", "mcmf_graph_info", "mcmf_diag",
            "mcmf_action", "mcmf_action_noalloc", "mcmf_batch", "mcmf_server_create",
            "mcmf_server_submit",
            "mcmf_server_wait", "mcmf_server_query", "mcmf_server_destroy",
            "mcmf_graph_set_tuning", "mcmf_graph_get_tuning", "mcmf_tune",
            "mcmf_status_string", "mcmf_last_error"]


class MCMFError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{mcmf_status_string(status)}: {message}")
        self.status = status


# ---------------------------------------------------------------- marshalling

def _addr(a) -> Optional[int]:
    """Raw address of a torch tensor or numpy array (None for None)."""
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        if not a.is_contiguous():
            raise ValueError("arrays must be contiguous")
        return a.data_ptr()
    if isinstance(a, np.ndarray):
        if not a.flags["C_CONTIGUOUS"]:
            raise ValueError("arrays must be contiguous")
        return a.ctypes.data
    if isinstance(a, int):
        return a
    raise TypeError(f"unsupported array type {type(a)!r}")


def _check_dtype(a, np_dtype, name):
    if a is None:
        return
    if hasattr(a, "dtype") and not isinstance(a, np.ndarray):
        import torch
        want = {np.int64: torch.int64, np.int32: torch.int32, np.float64: torch.float64,
                np.uint64: torch.uint64 if hasattr(torch, "uint64") else torch.int64}[np_dtype]
        if a.dtype != want and not (np_dtype is np.uint64 and a.dtype == torch.int64):
            raise TypeError(f"{name} must have dtype {want}, got {a.dtype}")
    elif isinstance(a, np.ndarray) and a.dtype != np_dtype:
        raise TypeError(f"{name} must have dtype {np.dtype(np_dtype)}, got {a.dtype}")


def _raise(status: int):
    if status != MCMF_OK:
        raise MCMFError(status, mcmf_last_error())


def make_fn(kind: int = MCMF_FN_EXP, scale: float = 1.0, coeffs=None):
    """An mcmf_fn; ``coeffs`` (host float64) is kept alive on the struct."""
    f = mcmf_fn()
    f.kind = kind
    f.scale = float(scale)
    if coeffs is not None:
        c = np.ascontiguousarray(coeffs, dtype=np.float64)
        f._keep = c
        f.coeffs = c.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        f.n_coeffs = c.size
    return f


def make_opts(seed: int = 0, request_id: int = 0, precision: int = MCMF_PRECISION_FP64,
              weight_cutoff: float = 0.0, stream=None, path_digest=None, q_out=None,
              allocation: int = MCMF_ALLOC_PER_ROW, walks_out=None):
    o = mcmf_opts()
    o.seed = seed
    o.request_id = request_id
    o.precision = precision
    o.weight_cutoff = weight_cutoff
    o.stream = stream
    _check_dtype(path_digest, np.uint64, "path_digest")
    _check_dtype(q_out, np.float64, "q_out")
    _check_dtype(walks_out, np.int32, "walks_out")
    o.path_digest = _addr(path_digest)
    o.q_out = _addr(q_out)
    o.walks_out = _addr(walks_out)
    o.allocation = allocation
    return o


# ---------------------------------------------------------------- C names

def mcmf_status_string(status: int) -> str:
    return _lib.mcmf_status_string(status).decode()


def mcmf_last_error() -> str:
    return _lib.mcmf_last_error().decode()


def mcmf_graph_create(n: int, row_ptr, col_idx, values=None, flags: int = MCMF_SYMMETRIC) -> int:
    """Returns the graph handle (an address); raises MCMFError on failure."""
    _check_dtype(row_ptr, np.int64, "row_ptr")
    _check_dtype(col_idx, np.int32, "col_idx")
    _check_dtype(values, np.float64, "values")
    out = _P()
    _raise(_lib.mcmf_graph_create(n, _addr(row_ptr), _addr(col_idx), _addr(values), flags,
                                  ctypes.byref(out)))
    return out.value


def mcmf_graph_destroy(g: int) -> None:
    _lib.mcmf_graph_destroy(g)


def mcmf_graph_info(g: int) -> dict:
    vals = [ctypes.c_int64() for _ in range(4)]
    _raise(_lib.mcmf_graph_info(g, *[ctypes.byref(v) for v in vals]))
    return dict(zip(("n", "nnz", "d_max", "active_rows"), (v.value for v in vals)))


_EMPTY_ROWS = ctypes.c_int32(0)


def mcmf_diag(g: int, f: mcmf_fn, rows, n_rows: int, n_walks: int, K: int,
              opts: Optional[mcmf_opts], out, stats: Optional[mcmf_stats] = None) -> None:
    _check_dtype(rows, np.int32, "rows")
    _check_dtype(out, np.float64, "out")
    rows_addr = _addr(rows)
    if rows is not None and not rows_addr:
        # An empty array may have no storage; NULL would mean "every row".
        rows_addr = ctypes.addressof(_EMPTY_ROWS)
    _raise(_lib.mcmf_diag(g, ctypes.byref(f), rows_addr, n_rows, n_walks, K,
                          ctypes.byref(opts) if opts is not None else None, _addr(out),
                          ctypes.byref(stats) if stats is not None else None))


def mcmf_action(g: int, f: mcmf_fn, v, n_walks: int, K: int, opts: Optional[mcmf_opts], out,
                stats: Optional[mcmf_stats] = None) -> None:
    _check_dtype(v, np.float64, "v")
    _check_dtype(out, np.float64, "out")
    _raise(_lib.mcmf_action(g, ctypes.byref(f), _addr(v), n_walks, K,
                            ctypes.byref(opts) if opts is not None else None, _addr(out),
                            ctypes.byref(stats) if stats is not None else None))


MCMF_NOALLOC_MAX_ROWS = 4192256


def mcmf_action_noalloc(g: int, f: mcmf_fn, v, n_walks: int, K: int, opts: Optional[mcmf_opts],
                        out) -> None:
    _check_dtype(v, np.float64, "v")
    _check_dtype(out, np.float64, "out")
    _raise(_lib.mcmf_action_noalloc(g, ctypes.byref(f), _addr(v), n_walks, K,
                                    ctypes.byref(opts) if opts is not None else None, _addr(out)))


def make_request(kind: int, graph: int, fn: mcmf_fn, K: int, n_walks: int, out, *, rows=None,
                 v=None, seed: int = 0, request_id: int = 0,
                 precision: int = MCMF_PRECISION_FP64, weight_cutoff: float = 0.0,
                 path_digest=None) -> mcmf_request:
    """An mcmf_request; the arrays it points to are kept alive on the struct."""
    _check_dtype(rows, np.int32, "rows")
    _check_dtype(v, np.float64, "v")
    _check_dtype(out, np.float64, "out")
    _check_dtype(path_digest, np.uint64, "path_digest")
    r = mcmf_request()
    r.kind = kind
    r.K = K
    r.graph = graph
    r.fn = fn
    rows_addr = _addr(rows)
    if rows is not None and not rows_addr:
        rows_addr = ctypes.addressof(_EMPTY_ROWS)
    r.rows = rows_addr
    r.n_rows = 0 if rows is None else len(rows)
    r.v = _addr(v)
    r.n_walks = n_walks
    r.seed = seed
    r.request_id = request_id
    r.precision = precision
    r.weight_cutoff = weight_cutoff
    r.out = _addr(out)
    r.path_digest = _addr(path_digest)
    r._keep = (fn, rows, v, out, path_digest)
    return r


def mcmf_batch(reqs, opts: Optional[mcmf_batch_opts] = None,
               stats: Optional[mcmf_stats] = None) -> None:
    """Runs a list of mcmf_request; writes each request's status and
    walk_steps back into the given structs."""
    reqs = list(reqs)
    arr = (mcmf_request * max(len(reqs), 1))()
    for i, r in enumerate(reqs):
        ctypes.memmove(ctypes.byref(arr, i * ctypes.sizeof(mcmf_request)), ctypes.byref(r),
                       ctypes.sizeof(mcmf_request))
    st = _lib.mcmf_batch(arr, len(reqs), ctypes.byref(opts) if opts is not None else None,
                         ctypes.byref(stats) if stats is not None else None)
    for i, r in enumerate(reqs):
        r.status = arr[i].status
        r.walk_steps = arr[i].walk_steps
    _raise(st)


def mcmf_graph_set_tuning(g: int, t: mcmf_tuning) -> None:
    _raise(_lib.mcmf_graph_set_tuning(g, ctypes.byref(t)))


def mcmf_graph_get_tuning(g: int) -> mcmf_tuning:
    t = mcmf_tuning()
    _raise(_lib.mcmf_graph_get_tuning(g, ctypes.byref(t)))
    return t


def mcmf_tune(g: int, f: mcmf_fn, n_walks: int, K: int) -> mcmf_tuning:
    t = mcmf_tuning()
    _raise(_lib.mcmf_tune(g, ctypes.byref(f), n_walks, K, ctypes.byref(t)))
    return t


def mcmf_server_create(opts: Optional[mcmf_server_opts] = None) -> int:
    out = _P()
    _raise(_lib.mcmf_server_create(ctypes.byref(opts) if opts is not None else None,
                                   ctypes.byref(out)))
    return out.value


def mcmf_server_submit(server: int, req: mcmf_request) -> int:
    """Queues req (which must stay alive until its wait); returns the ticket."""
    t = ctypes.c_uint64()
    _raise(_lib.mcmf_server_submit(server, ctypes.byref(req), ctypes.byref(t)))
    return t.value


def mcmf_server_wait(server: int, ticket: int, raise_on_error: bool = True) -> mcmf_ticket_info:
    info = mcmf_ticket_info()
    st = _lib.mcmf_server_wait(server, ticket, ctypes.byref(info))
    if raise_on_error:
        _raise(st)
    return info


def mcmf_server_query(server: int) -> dict:
    st = mcmf_server_stats()
    _raise(_lib.mcmf_server_query(server, ctypes.byref(st)))
    return st.as_dict()


def mcmf_server_destroy(server: int) -> None:
    _lib.mcmf_server_destroy(server)


# ---------------------------------------------------------------- convenience

class Graph:
    """Owns a graph handle.  ``Graph.from_csr(csr)`` takes any object with
    ``n``, ``row_ptr``, ``col`` and ``val`` (None for an unweighted graph)."""

    def __init__(self, handle: int):
        self.handle = handle
        self.info = mcmf_graph_info(handle)

    @classmethod
    def from_csr(cls, csr, flags: int = MCMF_SYMMETRIC, device: bool = True):
        row_ptr = np.ascontiguousarray(csr.row_ptr, dtype=np.int64)
        col = np.ascontiguousarray(csr.col, dtype=np.int32)
        val = None if csr.val is None else np.ascontiguousarray(csr.val, dtype=np.float64)
        if device:
            import torch
            row_ptr = torch.from_numpy(row_ptr).cuda()
            col = torch.from_numpy(col).cuda()
            val = None if val is None else torch.from_numpy(val).cuda()
            torch.cuda.synchronize()
        return cls(mcmf_graph_create(csr.n, row_ptr, col, val, flags))

    def close(self):
        if self.handle:
            mcmf_graph_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
