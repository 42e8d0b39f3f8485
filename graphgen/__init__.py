"""Seeded synthetic graph and vector generators.

This module only builds inputs: CSR adjacency matrices of undirected graphs
and right-hand-side vectors.  It holds none of the Monte Carlo estimator's
arithmetic, so both the GPU library and the CPU oracle can be fed from it.

Every generator returns a :class:`CSR` with ``row_ptr`` int64[n+1], ``col``
int32[nnz] (sorted within each row) and ``val`` either ``None`` (all stored
entries equal 1, the unweighted graphs the paper studies, Section 2.1) or a
float64[nnz] array.

The graph families follow their textbook definitions:

* Erdos-Renyi G(n, p) and G(n, M);
* R-MAT (Chakrabarti, Zhan, Faloutsos 2004): recursive quadrant choice with
  probabilities (a, b, c, d), then a random vertex relabelling; the
  Kronecker graphs of the paper's Table 1 are R-MAT graphs of this kind;
* Barabasi-Albert preferential attachment (see :mod:`graphgen.ba`);
* Watts-Strogatz ring lattice with random rewiring (the paper's
  ``smallworld`` family, Section 4);
* 2D grids and tori, complete graphs K_n, complete bipartite graphs K_{p,q},
  stars, paths, cycles, circulant (d-regular) graphs and hypercubes.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass
from typing import Optional

import numpy as np

__all__ = [
    "CSR", "from_edges", "erdos_renyi_dense", "erdos_renyi_gnm", "rmat",
    "grid2d", "torus2d", "complete", "complete_bipartite", "star", "path",
    "cycle", "circulant", "hypercube", "watts_strogatz", "with_random_weights",
    "lambda_max", "ones", "uniform_vector", "random_rows", "barabasi_albert", "rmat_native",
]


@dataclass
class CSR:
    n: int
    row_ptr: np.ndarray  # int64[n+1]
    col: np.ndarray      # int32[nnz]
    val: Optional[np.ndarray] = None  # float64[nnz] or None (implicit ones)
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def deg(self) -> np.ndarray:
        return np.diff(self.row_ptr)

    @property
    def d_max(self) -> int:
        return int(self.deg.max()) if self.n else 0

    def values(self) -> np.ndarray:
        """Stored values as float64 (ones when the graph is unweighted)."""
        if self.val is None:
            return np.ones(self.nnz, dtype=np.float64)
        return self.val

    def sha256(self) -> str:
        h = hashlib.sha256()
        h.update(np.int64(self.n).tobytes())
        h.update(np.ascontiguousarray(self.row_ptr, dtype=np.int64).tobytes())
        h.update(np.ascontiguousarray(self.col, dtype=np.int32).tobytes())
        if self.val is not None:
            h.update(np.ascontiguousarray(self.val, dtype=np.float64).tobytes())
        return h.hexdigest()

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.values(), self.col, self.row_ptr), shape=(self.n, self.n))

    def dense(self) -> np.ndarray:
        a = np.zeros((self.n, self.n), dtype=np.float64)
        rows = np.repeat(np.arange(self.n), self.deg)
        a[rows, self.col] = self.values()
        return a


def from_edges(n: int, src, dst, name: str = "", symmetric: bool = True,
               keep_loops: bool = False) -> CSR:
    """CSR of the graph on ``n`` nodes with the given edges.

    With ``symmetric`` each edge is stored in both directions.  Duplicates
    are removed and, unless ``keep_loops``, so are self-loops (the paper's
    clean-up of its Kronecker graphs, Section 4).  Isolated nodes are kept.
    """
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    if not keep_loops:
        m = src != dst
        src, dst = src[m], dst[m]
    if symmetric:
        src, dst = np.concatenate([src, dst]), np.concatenate([dst, src])
    key = np.unique(src * n + dst)
    rows = key // n
    col = (key % n).astype(np.int32)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=row_ptr[1:])
    return CSR(n, row_ptr, col, None, name)


def erdos_renyi_dense(n: int = 1000, p: float = 0.01, seed: int = 0) -> CSR:
    """G(n, p) drawn from one uniform n x n matrix: edge i<j iff U[i,j] < p."""
    rng = np.random.default_rng(seed)
    u = rng.random((n, n))
    iu, ju = np.nonzero(np.triu(u < p, k=1))
    return from_edges(n, iu, ju, name=f"er-{n}-p{p}-s{seed}")


def erdos_renyi_gnm(n: int, m: int, seed: int = 0) -> CSR:
    """G(n, M): M distinct undirected edges drawn uniformly (rejection of
    loops and repeats, topped up until M distinct pairs exist)."""
    rng = np.random.default_rng(seed)
    have = np.empty(0, dtype=np.int64)
    while have.size < m:
        need = int((m - have.size) * 1.1) + 16
        a = rng.integers(0, n, need, dtype=np.int64)
        b = rng.integers(0, n, need, dtype=np.int64)
        keep = a != b
        lo, hi = np.minimum(a[keep], b[keep]), np.maximum(a[keep], b[keep])
        have = np.unique(np.concatenate([have, lo * n + hi]))
    have = have[rng.permutation(have.size)[:m]]
    return from_edges(n, have // n, have % n, name=f"gnm-{n}-{m}-s{seed}")


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19,
         c: float = 0.19, seed: int = 0, permute: bool = True) -> CSR:
    """R-MAT graph with 2^scale nodes and edge_factor * 2^scale edge draws.

    Each draw descends ``scale`` levels; at each level it picks quadrant
    (0,0), (0,1), (1,0), (1,1) with probabilities a, b, c, d = 1-a-b-c.
    Vertices are then relabelled by a seeded random permutation.  The result
    is symmetrised, deduplicated and loop-free; isolated vertices are kept so
    that n = 2^scale.
    """
    n = 1 << scale
    m = edge_factor * n
    rng = np.random.default_rng(seed)
    src = np.zeros(m, dtype=np.int64)
    dst = np.zeros(m, dtype=np.int64)
    ab, abc = a + b, a + b + c
    for level in range(scale):
        r = rng.random(m)
        sbit = r >= ab
        dbit = ((r >= a) & (r < ab)) | (r >= abc)
        src |= sbit.astype(np.int64) << level
        dst |= dbit.astype(np.int64) << level
        del r, sbit, dbit
    if permute:
        perm = rng.permutation(n)
        src = perm[src]
        dst = perm[dst]
    return from_edges(n, src, dst, name=f"rmat-{scale}-ef{edge_factor}-s{seed}")


def grid2d(rows: int, cols: int) -> CSR:
    """5-point grid graph (4-neighbour, no wrap-around)."""
    idx = np.arange(rows * cols, dtype=np.int64).reshape(rows, cols)
    src = np.concatenate([idx[:, :-1].ravel(), idx[:-1, :].ravel()])
    dst = np.concatenate([idx[:, 1:].ravel(), idx[1:, :].ravel()])
    return from_edges(rows * cols, src, dst, name=f"grid-{rows}x{cols}")


def torus2d(rows: int, cols: int) -> CSR:
    """2D torus: every node has exactly 4 neighbours (rows, cols >= 3)."""
    idx = np.arange(rows * cols, dtype=np.int64).reshape(rows, cols)
    src = np.concatenate([idx.ravel(), idx.ravel()])
    dst = np.concatenate([np.roll(idx, -1, axis=1).ravel(), np.roll(idx, -1, axis=0).ravel()])
    return from_edges(rows * cols, src, dst, name=f"torus-{rows}x{cols}")


def complete(n: int) -> CSR:
    i, j = np.triu_indices(n, k=1)
    return from_edges(n, i, j, name=f"K{n}")


def complete_bipartite(p: int, q: int) -> CSR:
    """K_{p,q}: nodes 0..p-1 on one side, p..p+q-1 on the other."""
    i = np.repeat(np.arange(p), q)
    j = p + np.tile(np.arange(q), p)
    return from_edges(p + q, i, j, name=f"K{p},{q}")


def star(leaves: int) -> CSR:
    """Star K_{1,leaves}; node 0 is the hub."""
    return complete_bipartite(1, leaves)


def path(n: int) -> CSR:
    i = np.arange(n - 1)
    return from_edges(n, i, i + 1, name=f"P{n}")


def cycle(n: int) -> CSR:
    i = np.arange(n)
    return from_edges(n, i, (i + 1) % n, name=f"C{n}")


def circulant(n: int, half_degree: int) -> CSR:
    """Node i is joined to i+-1, ..., i+-half_degree (mod n): 2*half_degree-regular."""
    i = np.repeat(np.arange(n), half_degree)
    off = np.tile(np.arange(1, half_degree + 1), n)
    return from_edges(n, i, (i + off) % n, name=f"circ-{n}-{half_degree}")


def hypercube(dim: int) -> CSR:
    """dim-dimensional hypercube: dim-regular and bipartite."""
    n = 1 << dim
    i = np.repeat(np.arange(n), dim)
    bit = np.tile(np.arange(dim), n)
    return from_edges(n, i, i ^ (1 << bit), name=f"Q{dim}")


def watts_strogatz(n: int, k: int = 10, beta: float = 0.1, seed: int = 0) -> CSR:
    """Ring lattice where each node is joined to its k nearest neighbours
    (k/2 on each side); each lattice edge (i, i+o) is rewired with
    probability beta to (i, w), w uniform among nodes that create neither a
    loop nor a repeated edge."""
    rng = np.random.default_rng(seed)
    half = k // 2
    adj = [set() for _ in range(n)]
    edges = []
    for o in range(1, half + 1):
        for i in range(n):
            j = (i + o) % n
            adj[i].add(j)
            adj[j].add(i)
            edges.append((i, j))
    for idx, (i, j) in enumerate(edges):
        if rng.random() < beta:
            if len(adj[i]) >= n - 1:
                continue
            while True:
                w = int(rng.integers(0, n))
                if w != i and w not in adj[i]:
                    break
            adj[i].discard(j)
            adj[j].discard(i)
            adj[i].add(w)
            adj[w].add(i)
            edges[idx] = (i, w)
    e = np.array(edges, dtype=np.int64)
    return from_edges(n, e[:, 0], e[:, 1], name=f"ws-{n}-{k}-{beta}-s{seed}")


def with_random_weights(g: CSR, seed: int = 0, low: float = 0.1, high: float = 2.0,
                        negative_fraction: float = 0.0) -> CSR:
    """Symmetric random weights on the same pattern: the weight of an
    undirected edge is drawn once and stored in both directions."""
    rng = np.random.default_rng(seed)
    rows = np.repeat(np.arange(g.n, dtype=np.int64), g.deg)
    lo = np.minimum(rows, g.col)
    hi = np.maximum(rows, g.col)
    key = lo * g.n + hi
    uniq, inv = np.unique(key, return_inverse=True)
    w = rng.uniform(low, high, uniq.size)
    if negative_fraction > 0:
        w = np.where(rng.random(uniq.size) < negative_fraction, -w, w)
    return CSR(g.n, g.row_ptr, g.col, w[inv].astype(np.float64), g.name + "-w")


def lambda_max(g: CSR, iters: int = 50) -> float:
    """Largest eigenvalue estimate by power iteration from 1/sqrt(n) * 1:
    x <- A x / ||A x|| for ``iters - 1`` steps, then lambda = ||A x||_2."""
    a = g.to_scipy()
    x = np.full(g.n, 1.0 / np.sqrt(g.n))
    for _ in range(iters - 1):
        y = a @ x
        x = y / np.linalg.norm(y)
    return float(np.linalg.norm(a @ x))


def ones(n: int) -> np.ndarray:
    return np.ones(n, dtype=np.float64)


def uniform_vector(n: int, seed: int = 0) -> np.ndarray:
    return np.random.default_rng(seed).random(n)


def random_rows(n: int, count: int, seed: int = 0, replace: bool = False) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.choice(n, size=count, replace=replace).astype(np.int32)


def rmat_native(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19,
                c: float = 0.19, seed: int = 0, permute: bool = True) -> CSR:
    """R-MAT by the multithreaded C generator (see :mod:`graphgen.rmatgen`)."""
    from .rmatgen import rmat_native as _rmat_native
    return _rmat_native(scale, edge_factor, a, b, c, seed, permute)


def barabasi_albert(n: int, m: int = 8, seed: int = 0) -> CSR:
    from .ba import barabasi_albert as _ba
    return _ba(n, m, seed)
