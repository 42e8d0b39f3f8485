"""Directed graphs through MCMF_DIGRAPH: the library stores
B = [[0, A], [A^T, 0]] (Section 4, Eq. digraph_sym) and every estimate on it
matches the oracle run on B assembled independently with scipy (walk paths
bit-exact, estimates within 1e-10)."""
import numpy as np
import pytest
import scipy.sparse as sp

import graphgen as G
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from _gpu import assert_close, default_sampler, gpu_action, gpu_diag, oracle_fn  # noqa: E402
from paper_2308_01037_amd import mcmf as M  # noqa: E402


def directed(n, m, seed, weighted=False):
    rng = np.random.default_rng(seed)
    src = rng.integers(0, n, m)
    dst = rng.integers(0, n, m)
    keep = src != dst
    a = sp.coo_matrix((np.ones(keep.sum()), (src[keep], dst[keep])), shape=(n, n)).tocsr()
    a.sum_duplicates()
    a.sort_indices()
    if weighted:
        a.data = rng.uniform(-1.0, 2.0, a.nnz)
    return a


def as_csr(a, name):
    val = None if np.all(a.data == 1.0) else a.data.astype(np.float64)
    return G.CSR(a.shape[0], a.indptr.astype(np.int64), a.indices.astype(np.int32), val, name)


@pytest.mark.parametrize("weighted", [False, True])
@pytest.mark.parametrize("device_input", [False, True])
def test_digraph_symmetrised_matches_oracle(weighted, device_input):
    a = directed(700, 5000, seed=3 + weighted, weighted=weighted)
    b = sp.bmat([[None, a], [a.T, None]]).tocsr()
    b.sort_indices()
    bcsr = as_csr(b, "B")
    acsr = as_csr(a, "A")
    g = M.Graph.from_csr(acsr, flags=M.MCMF_DIGRAPH, device=device_input)
    try:
        assert g.info["n"] == 2 * a.shape[0] and g.info["nnz"] == 2 * a.nnz
        scale = 1.0 / max(1.0, float(abs(b).sum(axis=1).max()))
        for fn in ("exp", "resolvent"):
            o = oracle.diag(bcsr, oracle_fn(fn), N=64, K=12, scale=scale, seed=4, want_digest=True,
                            sampler=default_sampler(bcsr))
            r = gpu_diag(g, fn, 64, 12, scale, seed=4, want_digest=True)
            assert np.array_equal(r["digest"], o["digest"])
            assert_close(r["d"], o["d"], 1e-10, atol=1e-13 * np.max(np.abs(o["d"])))
            v = np.random.default_rng(5).random(b.shape[0])
            o = oracle.action(bcsr, oracle_fn(fn), v, N=64, K=12, scale=scale, seed=4, want_digest=True,
                              sampler=default_sampler(bcsr))
            r = gpu_action(g, fn, v, 64, 12, scale, seed=4, want_digest=True)
            assert np.array_equal(r["digest"], o["digest"])
            assert_close(r["y"], o["y"], 1e-10, atol=1e-13 * np.max(np.abs(o["y"])))
    finally:
        g.close()
