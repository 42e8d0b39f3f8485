"""Hub rows of the diagonal gather on the GPU.

For a start row k next to one of the graph's hub rows h, <Q_k, C_h> of Eq.
rand_funm_formula_diag is summed from a per-node mask of adjacent hubs
instead of by probing Q_k with every entry of row h.  Both ways sum the same
terms: the walks (path digests, step counts) are bit-identical, the
estimates agree within 1e-10 relative, and both match the oracle.
"""
import numpy as np
import pytest

import graphgen as G
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from _gpu import assert_close, gpu_diag, graph, oracle_fn  # noqa: E402
from _reqs import Req, run_batch  # noqa: E402
from paper_2308_01037_amd import mcmf as M  # noqa: E402

OFF = 2**31 - 1  # no hub reaches this degree: the hub pass is off


def hubs(g, min_degree):
    t = M.mcmf_graph_get_tuning(g.handle)
    t.hub_min_degree = min_degree
    t.hub_count = 0
    M.mcmf_graph_set_tuning(g.handle, t)
    return M.mcmf_graph_get_tuning(g.handle).hub_count


def both(g, *args, **kw):
    hubs(g, 1)
    on = gpu_diag(g, *args, want_digest=True, stats=True, **kw)
    hubs(g, OFF)
    off = gpu_diag(g, *args, want_digest=True, stats=True, **kw)
    return on, off


def check_same(on, off):
    assert np.array_equal(on["digest"], off["digest"])
    assert on["stats"]["walk_steps"] == off["stats"]["walk_steps"]
    assert_close(on["d"], off["d"], 1e-10, what="hub pass vs probes")


@pytest.mark.parametrize("rows", [None, "subset"])
@pytest.mark.parametrize("fn", ["exp", "resolvent"])
def test_hub_pass_matches_probes_and_oracle(rows, fn):
    csr = G.rmat(11, seed=4)
    K, N, s = 12, 40, 0.9 / csr.d_max
    sel = None if rows is None else G.random_rows(csr.n, 300, seed=2)
    # Requested hubs and unrequested ones: the first rows by degree.
    if sel is not None:
        top = np.argsort(-np.diff(csr.row_ptr), kind="stable")[:32]
        sel = np.concatenate([sel, top[::3]]).astype(np.int32)
    with graph(csr) as g:
        assert hubs(g, 1) == 32
        on, off = both(g, fn, N, K, s, seed=5, rows=sel)
        check_same(on, off)
        # The hub pass replaces probes: fewer 4-byte reads in all.
        assert on["stats"]["gather_probes"] < off["stats"]["gather_probes"]
        o = oracle.diag(csr, oracle_fn(fn), N=N, K=K, scale=s, seed=5, rows=sel, want_digest=True)
        assert np.array_equal(on["digest"], o["digest"])
        assert_close(on["d"], o["d"], 1e-10, what="hub pass vs oracle")


def test_automatic_threshold_and_more_than_four_hubs_per_row():
    # A dense core: many rows are adjacent to most of the 32 hubs, so a walk
    # adds each visit into several hub sums.
    csr = G.rmat(11, edge_factor=64, seed=3)
    K, N, s = 10, 64, 0.5 / csr.d_max
    with graph(csr) as g:
        hubs(g, 0)
        auto = gpu_diag(g, "exp", N, K, s, seed=1, want_digest=True, stats=True)
        on, off = both(g, "exp", N, K, s, seed=1)
        check_same(on, off)
        check_same(auto, off)


def test_hub_pass_with_several_walk_passes():
    # n above the LDS table and N (K-1) visits beyond it: the walks of a row
    # are taken in passes, each with its own hub sums.
    csr = G.rmat(14, seed=7)
    rows = G.random_rows(csr.n, 40, seed=3)
    with graph(csr) as g:
        on, off = both(g, "exp", 600, 30, 0.5 / csr.d_max, seed=2, rows=rows)
        check_same(on, off)


@pytest.mark.parametrize("N", [16, 48, 160])
def test_fp32_weights_and_batch_use_the_hub_pass(N):
    # Batched walk tasks: N >= 128 one start row per task, 32 <= N < 128
    # several rows each with its own hub sums, N < 32 no hub sums at all.
    csr = G.rmat(12, seed=9)
    K, s = 14, 0.8 / csr.d_max
    top = np.argsort(-np.diff(csr.row_ptr), kind="stable")[:32]
    sel = np.concatenate([G.random_rows(csr.n, 200, seed=4), top[::2]]).astype(np.int32)
    with graph(csr) as g:
        def reqs():
            return [Req(g, csr, M.MCMF_REQ_DIAG, "exp", s, N, K, seed=6),
                    Req(g, csr, M.MCMF_REQ_DIAG, "exp", s, N, K, seed=6,
                        precision=M.MCMF_PRECISION_FP32_WEIGHTS),
                    Req(g, csr, M.MCMF_REQ_DIAG, "resolvent", s, N, K, seed=7, request=2, rows=sel)]
        hubs(g, OFF)
        want = [q.single() for q in reqs()]
        hubs(g, 1)
        got, _ = run_batch(reqs())
        for r, w in zip(got, want):
            assert np.array_equal(r["digest"], w["digest"])
            assert r["steps"] == w["steps"]
            assert_close(r["x"], w["x"], 1e-10)


def test_graphs_without_hubs():
    # Weighted graphs and graphs whose rows are not strictly increasing keep
    # no hub rows; neither does a graph created without MCMF_SYMMETRIC.
    base = G.rmat(9, seed=1)
    with graph(G.with_random_weights(base, seed=2)) as g:
        assert hubs(g, 1) == 0
    with graph(base, flags=0) as g:
        assert hubs(g, 1) == 0
    rp = base.row_ptr.astype(np.int64)
    col = base.col.astype(np.int32).copy()
    i = int(np.argmax(np.diff(rp)))
    col[rp[i]:rp[i + 1]] = col[rp[i]:rp[i + 1]][::-1]
    h = M.mcmf_graph_create(base.n, rp, col, None, M.MCMF_SYMMETRIC)
    try:
        t = M.mcmf_graph_get_tuning(h)
        assert t.hub_count == 0
    finally:
        M.mcmf_graph_destroy(h)


def test_hub_threshold_argument_error():
    with graph(G.path(4)) as g:
        t = M.mcmf_tuning()
        t.hub_min_degree = -1
        with pytest.raises(M.MCMFError) as e:
            M.mcmf_graph_set_tuning(g.handle, t)
        assert e.value.status == M.MCMF_E_ARG


def test_hub_pass_closed_form_complete_bipartite():
    # K_{p,q}: the diagonal is the closed form on every walk, so the hub sums
    # (all 5 rows of the small side are hubs, plus 27 rows of the other side)
    # must give it to rounding.
    p, q, K, s = 5, 300, 10, 0.9 / 300
    csr = G.complete_bipartite(p, q)
    c = oracle.coeffs(oracle.FN_EXP, K)

    def closed(own, other):
        return c[0] + sum(c[2 * m] * s ** (2 * m) * own * (own * other) ** (m - 1)
                          for m in range(1, K // 2 + 1))
    want = np.array([closed(q, p)] * p + [closed(p, q)] * q)
    with graph(csr) as g:
        assert hubs(g, 1) == 32
        on, off = both(g, "exp", 16, K, s, seed=3)
        check_same(on, off)
        assert on["stats"]["gather_probes"] < off["stats"]["gather_probes"]
    assert_close(on["d"], want, 1e-12, what="K_pq closed form with hub sums")


def test_hub_rows_with_self_loops_and_digraph():
    # Self-loops on hub rows (a hub adjacent to itself) and the symmetrised
    # digraph B = [[0, A], [A^T, 0]], whose hubs are rows of both halves.
    rng = np.random.default_rng(8)
    n = 600
    src = np.concatenate([rng.integers(0, n, 6000), np.zeros(300, np.int64), np.arange(0, 40)])
    dst = np.concatenate([rng.integers(0, n, 6000), rng.integers(0, n, 300), np.arange(0, 40)])
    csr = G.from_edges(n, src, dst, keep_loops=True)
    with graph(csr) as g:
        assert hubs(g, 1) == 32
        on, off = both(g, "resolvent", 24, 9, 0.5 / csr.d_max, seed=4)
        check_same(on, off)
        o = oracle.diag(csr, oracle_fn("resolvent"), N=24, K=9, scale=0.5 / csr.d_max, seed=4)
        assert_close(on["d"], o["d"], 1e-10, what="loops vs oracle")
    dg = G.from_edges(n, src, dst, symmetric=False)
    h = M.mcmf_graph_create(dg.n, dg.row_ptr.astype(np.int64), dg.col.astype(np.int32), None,
                            M.MCMF_DIGRAPH)
    g = M.Graph(h)
    try:
        assert hubs(g, 1) == 32
        on, off = both(g, "exp", 20, 8, 0.5 / g.info["d_max"], seed=6)
        check_same(on, off)
    finally:
        g.close()
