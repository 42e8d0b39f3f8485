"""Autotuner cache: tuning results of mcmf_tune kept in a JSON file, keyed by
a fingerprint of the graph and the request shape, and reapplied with
mcmf_graph_set_tuning.  The measurement itself is native (mcmf_tune)."""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

from . import mcmf as M


def fingerprint(csr, n_walks: int, K: int) -> str:
    """Hash of the CSR arrays (row_ptr, col, values) and the request shape."""
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(csr.row_ptr, dtype=np.int64).tobytes())
    h.update(np.ascontiguousarray(csr.col, dtype=np.int32).tobytes())
    if getattr(csr, "val", None) is not None:
        h.update(np.ascontiguousarray(csr.val, dtype=np.float64).tobytes())
    h.update(f"N={int(n_walks)},K={int(K)}".encode())
    return h.hexdigest()[:32]


def _load(path: str) -> dict:
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def autotune(graph, csr, fn: M.mcmf_fn, n_walks: int, K: int, cache_path: str) -> dict:
    """Applies the cached tuning of (graph, N, K) or measures it with
    mcmf_tune and stores it.  Returns the tuning as a dict (with "cached")."""
    key = fingerprint(csr, n_walks, K)
    cache = _load(cache_path)
    if key in cache:
        d = cache[key]
        t = M.mcmf_graph_get_tuning(graph.handle)  # keeps the graph's other settings
        t.hub_count = 0
        for name in ("action_sampler", "action_stream", "diag_sampler", "diag_stream",
                     "walk_threads", "gather_item", "hub_min_degree"):
            if name in d:
                setattr(t, name, int(d[name]))
        M.mcmf_graph_set_tuning(graph.handle, t)
        return dict(d, cached=True)
    t = M.mcmf_tune(graph.handle, fn, n_walks, K)
    d = t.as_dict()
    cache[key] = d
    os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
    tmp = cache_path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    os.replace(tmp, cache_path)
    return dict(d, cached=False)
