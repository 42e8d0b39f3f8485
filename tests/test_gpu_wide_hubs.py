"""Wide hubs of the diagonal walk on the GPU.

A graph with more than 32 candidate hub rows keeps its (up to 1024) rows of
largest degree as wide hubs, with a 128-byte mask per node of the wide hubs
adjacent to it; with MCMF_SAMPLER_WIDE the walk of start row k sums
<Q_k, C_h> of Eq. rand_funm_formula_diag for every requested wide hub h next
to k while it records the visits; the gather then probes Q_k with the other
neighbours only.  Both ways sum the same terms:
walks (path digests, step counts) are bit-identical to the EDGE and ROW
walks, the estimates agree within 1e-10 relative, and both match the oracle
(and closed forms where the graph has one).
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
from paper_2308_01037_amd import mcmf as M  # noqa: E402

OFF = 2**31 - 1  # no hub reaches this degree: hub sums off


def setup(g, sampler, min_degree=1):
    t = M.mcmf_graph_get_tuning(g.handle)
    t.diag_sampler, t.hub_min_degree, t.hub_count = sampler, min_degree, 0
    M.mcmf_graph_set_tuning(g.handle, t)


def run3(g, *args, **kw):
    """WIDE with every wide hub active, EDGE with the 32 narrow hubs, and
    EDGE without hub sums, on the same walks."""
    out = {}
    for name, sampler, deg in (("wide", M.MCMF_SAMPLER_WIDE, 1), ("narrow", M.MCMF_SAMPLER_EDGE, 1),
                               ("off", M.MCMF_SAMPLER_EDGE, OFF)):
        setup(g, sampler, deg)
        out[name] = gpu_diag(g, *args, want_digest=True, stats=True, **kw)
    return out


def check_same(r):
    for other in ("narrow", "off"):
        assert np.array_equal(r["wide"]["digest"], r[other]["digest"])
        assert r["wide"]["stats"]["walk_steps"] == r[other]["stats"]["walk_steps"]
        assert_close(r["wide"]["d"], r[other]["d"], 1e-10, what=f"wide vs {other}")


def top_rows(csr, m):
    deg = np.diff(csr.row_ptr)
    return np.lexsort((np.arange(csr.n), -deg))[:m]


@pytest.mark.parametrize("rows", [None, "subset"])
@pytest.mark.parametrize("fn", ["exp", "resolvent"])
def test_wide_hubs_match_narrow_probes_and_oracle(rows, fn):
    csr = G.rmat(12, seed=4)
    K, N, s = 12, 40, 0.9 / csr.d_max
    sel = None
    if rows is not None:
        # Random rows plus every 7th wide hub: requested wide hubs, narrow
        # hubs among them, and unrequested ones.
        sel = np.concatenate([G.random_rows(csr.n, 300, seed=2), top_rows(csr, 1024)[::7]])
        sel = np.unique(sel).astype(np.int32)
    with graph(csr) as g:
        t = M.mcmf_graph_get_tuning(g.handle)
        assert (t.hub_count, t.wide_hub_count) == (32, 1024)
        r = run3(g, fn, N, K, s, seed=5, rows=sel)
        check_same(r)
        # The wide sums replace probes: fewer than with 32 hubs, fewer than none.
        probes = [r[k]["stats"]["gather_probes"] for k in ("wide", "narrow", "off")]
        assert probes[0] < probes[1] < probes[2]
        o = oracle.diag(csr, oracle_fn(fn), N=N, K=K, scale=s, seed=5, rows=sel, want_digest=True)
        assert np.array_equal(r["wide"]["digest"], o["digest"])
        assert_close(r["wide"]["d"], o["d"], 1e-10, what="wide vs oracle")


@pytest.mark.parametrize("min_degree", [0, 60, 200])
def test_threshold_picks_a_prefix_of_wide_hubs(min_degree):
    # hub_min_degree (0: automatic, N (K-1) / 4) leaves the wide hubs below
    # it to the gather; every threshold gives the same estimate.
    csr = G.rmat(12, edge_factor=24, seed=8)
    K, N, s = 10, 48, 0.6 / csr.d_max
    deg = np.sort(np.diff(csr.row_ptr))[::-1]
    with graph(csr) as g:
        setup(g, M.MCMF_SAMPLER_EDGE, OFF)
        off = gpu_diag(g, "exp", N, K, s, seed=2, want_digest=True, stats=True)
        setup(g, M.MCMF_SAMPLER_WIDE, min_degree)
        r = gpu_diag(g, "exp", N, K, s, seed=2, want_digest=True, stats=True)
    thr = N * (K - 1) // 4 if min_degree == 0 else min_degree
    assert 0 < np.count_nonzero(deg[:1024] >= thr) < 1024  # a real prefix
    assert np.array_equal(r["digest"], off["digest"])
    assert r["stats"]["gather_probes"] < off["stats"]["gather_probes"]
    assert_close(r["d"], off["d"], 1e-10, what=f"threshold {min_degree}")


def test_wide_hubs_with_fp32_weights_cutoff_and_passes():
    # FP32 walk weights and a weight cutoff (walks end early), and N (K-1)
    # beyond one LDS table so the gather takes each row in passes.
    csr = G.rmat(14, seed=7)
    rows = np.concatenate([G.random_rows(csr.n, 40, seed=3), top_rows(csr, 1024)[::50]]).astype(np.int32)
    s = 0.5 / csr.d_max
    with graph(csr) as g:
        for N, K, kw in ((48, 14, {"cutoff": 1e-3}), (600, 30, {})):
            r = run3(g, "exp", N, K, s, seed=2, rows=rows, **kw)
            check_same(r)
        stream = torch.cuda.current_stream().cuda_stream
        res = {}
        for name, sampler in (("wide", M.MCMF_SAMPLER_WIDE), ("edge", M.MCMF_SAMPLER_EDGE)):
            setup(g, sampler, 1 if sampler == M.MCMF_SAMPLER_WIDE else OFF)
            out = torch.empty(csr.n, dtype=torch.float64, device="cuda")
            M.mcmf_diag(g.handle, M.make_fn(M.MCMF_FN_EXP, s), None, 0, 64, 16,
                        M.make_opts(seed=3, precision=M.MCMF_PRECISION_FP32_WEIGHTS, stream=stream), out)
            torch.cuda.synchronize()
            res[name] = out.cpu().numpy()
        # The same FP32 visit weights, summed in FP64 in another order.
        assert_close(res["wide"], res["edge"], 1e-10, what="FP32 weights")


def test_wide_hubs_with_norm_allocation():
    # Walks allocated by column norm (a different walk count per start row).
    csr = G.rmat(12, seed=11)
    s = 0.7 / csr.d_max
    with graph(csr) as g:
        res = {}
        for name, sampler, deg in (("wide", M.MCMF_SAMPLER_WIDE, 1), ("off", M.MCMF_SAMPLER_EDGE, OFF)):
            setup(g, sampler, deg)
            dig = torch.zeros(csr.n, dtype=torch.int64, device="cuda")
            out = torch.empty(csr.n, dtype=torch.float64, device="cuda")
            M.mcmf_diag(g.handle, M.make_fn(M.MCMF_FN_RESOLVENT, s), None, 0, 64 * csr.n, 12,
                        M.make_opts(seed=4, allocation=M.MCMF_ALLOC_NORM_MIN1, path_digest=dig,
                                    stream=torch.cuda.current_stream().cuda_stream), out)
            torch.cuda.synchronize()
            res[name] = (out.cpu().numpy(), dig.cpu().numpy())
        assert np.array_equal(res["wide"][1], res["off"][1])
        assert_close(res["wide"][0], res["off"][0], 1e-10, what="norm allocation")


def test_wide_hub_closed_form_complete_bipartite():
    # K_{p,q} with p + q < 1024: every row is a wide hub, so every neighbour
    # of every start row is summed by the walk and the gather probes nothing.
    p, q, K, s = 5, 300, 10, 0.9 / 300
    csr = G.complete_bipartite(p, q)
    c = oracle.coeffs(oracle.FN_EXP, K)

    def closed(own, other):
        return c[0] + sum(c[2 * m] * s ** (2 * m) * own * (own * other) ** (m - 1)
                          for m in range(1, K // 2 + 1))
    want = np.array([closed(q, p)] * p + [closed(p, q)] * q)
    with graph(csr) as g:
        r = run3(g, "exp", 16, K, s, seed=3)
        check_same(r)
        assert r["wide"]["stats"]["gather_probes"] == 0
    assert_close(r["wide"]["d"], want, 1e-12, what="K_pq closed form with wide hubs")


def test_wide_hubs_with_self_loops():
    # Self-loops on hub rows (a hub adjacent to itself).
    rng = np.random.default_rng(8)
    n = 2000
    src = np.concatenate([rng.integers(0, n, 16000), np.zeros(300, np.int64), np.arange(0, 60)])
    dst = np.concatenate([rng.integers(0, n, 16000), rng.integers(0, n, 300), np.arange(0, 60)])
    csr = G.from_edges(n, src, dst, keep_loops=True)
    with graph(csr) as g:
        r = run3(g, "resolvent", 24, 9, 0.5 / csr.d_max, seed=4)
        check_same(r)
        o = oracle.diag(csr, oracle_fn("resolvent"), N=24, K=9, scale=0.5 / csr.d_max, seed=4)
        assert_close(r["wide"]["d"], o["d"], 1e-10, what="loops vs oracle")


def test_graphs_without_wide_hubs_reject_the_layout():
    # At most 32 rows with entries, weighted graphs, and graphs created
    # without MCMF_SYMMETRIC keep no wide hubs.
    base = G.rmat(9, seed=1)
    for csr, flags in ((G.path(20), M.MCMF_SYMMETRIC), (G.with_random_weights(base, seed=2), M.MCMF_SYMMETRIC),
                       (base, 0)):
        with graph(csr, flags=flags) as g:
            assert M.mcmf_graph_get_tuning(g.handle).diag_sampler != M.MCMF_SAMPLER_WIDE
            assert M.mcmf_graph_get_tuning(g.handle).wide_hub_count == 0
            t = M.mcmf_graph_get_tuning(g.handle)
            t.diag_sampler, t.hub_count = M.MCMF_SAMPLER_WIDE, 0
            with pytest.raises(M.MCMFError) as e:
                M.mcmf_graph_set_tuning(g.handle, t)
            assert e.value.status == M.MCMF_E_ARG
    with graph(base) as g:  # has them: accepted
        setup(g, M.MCMF_SAMPLER_WIDE)
        assert M.mcmf_graph_get_tuning(g.handle).diag_sampler == M.MCMF_SAMPLER_WIDE
        t = M.mcmf_graph_get_tuning(g.handle)
        t.action_sampler, t.hub_count = M.MCMF_SAMPLER_WIDE, 0  # the diagonal's only
        with pytest.raises(M.MCMFError):
            M.mcmf_graph_set_tuning(g.handle, t)


@pytest.mark.parametrize("K", [2, 3])
def test_wide_hubs_with_the_shortest_walks(K):
    # K = 2 records only step 0 (the start row itself: every hub next to k
    # gets the row's whole sum); K = 3 adds one transition.
    csr = G.rmat(11, seed=13)
    s = 0.7 / csr.d_max
    sel = np.concatenate([G.random_rows(csr.n, 100, seed=5), top_rows(csr, 1024)[::9]]).astype(np.int32)
    with graph(csr) as g:
        for rows in (None, sel):
            r = run3(g, "exp", 64, K, s, seed=7, rows=rows)
            check_same(r)
            o = oracle.diag(csr, oracle_fn("exp"), N=64, K=K, scale=s, seed=7, rows=rows, want_digest=True)
            assert np.array_equal(r["wide"]["digest"], o["digest"])
            assert_close(r["wide"]["d"], o["d"], 1e-10, what=f"K={K}")


def test_batched_requests_use_wide_hub_sums():
    # Batched diagonal requests with N >= 128 (one start row per task) on a
    # graph whose layout is WIDE take the wide hub sums too; requests with
    # fewer walks keep the 32 hubs.  Each equals its single call (which walks
    # with the wide sums) and the oracle; the wide sums leave fewer probes.
    from _reqs import Req, run_batch
    csr = G.rmat(12, seed=17)
    s = 0.8 / csr.d_max
    sel = np.concatenate([G.random_rows(csr.n, 200, seed=6), top_rows(csr, 1024)[::5]]).astype(np.int32)

    def reqs(g):
        return [Req(g, csr, M.MCMF_REQ_DIAG, "exp", s, 160, 10, seed=1),
                Req(g, csr, M.MCMF_REQ_DIAG, "resolvent", s, 128, 12, seed=2, request=1, rows=sel),
                Req(g, csr, M.MCMF_REQ_DIAG, "exp", s, 48, 9, seed=3, request=2, rows=sel),
                Req(g, csr, M.MCMF_REQ_DIAG, "exp", s, 256, 8, seed=4, request=3,
                    precision=M.MCMF_PRECISION_FP32_WEIGHTS, cutoff=1e-4),
                Req(g, csr, M.MCMF_REQ_ACTION, "exp", s, 64, 10, seed=5, request=4)]
    with graph(csr) as g:
        setup(g, M.MCMF_SAMPLER_WIDE, 1)
        rs = reqs(g)
        want = [q.single() for q in rs]
        eager, st_wide = run_batch(rs)
        captured, _ = run_batch(rs, use_graph=True)
        setup(g, M.MCMF_SAMPLER_EDGE, 1)
        narrow, st_narrow = run_batch(reqs(g))
    for got in (eager, captured, narrow):
        for r, w in zip(got, want):
            assert np.array_equal(r["digest"], w["digest"])
            assert r["steps"] == w["steps"]
            assert_close(r["x"], w["x"], 1e-10)
    assert st_wide["gather_probes"] < st_narrow["gather_probes"]
    o = oracle.diag(csr, oracle_fn("resolvent"), N=128, K=12, scale=s, seed=2, request=1, rows=sel,
                    want_digest=True)
    assert np.array_equal(eager[1]["digest"], o["digest"])
    assert_close(eager[1]["x"], o["d"], 1e-10, what="batched wide diag vs oracle")


def _auto_takes_wide(csr, N, K):
    # The AUTO rule: the squared degrees of the active wide hubs beyond the
    # first 32 (degree >= N (K-1) / 4), over the recorded states, at least 4.
    deg = np.sort(np.diff(csr.row_ptr))[::-1][:1024].astype(float)
    thr = max(1, N * (K - 1) // 4)
    act = int(np.count_nonzero(deg >= thr))
    saved = float((deg[min(act, 32):act] ** 2).sum())
    states = np.count_nonzero(np.diff(csr.row_ptr)) * N * (K - 1)
    return saved >= 4 * states


@pytest.mark.parametrize("N,K", [(16, 10), (2048, 40)])
def test_auto_layout_chooses_per_call(N, K):
    # MCMF_SAMPLER_AUTO walks with the wide hub sums exactly when they save at
    # least 4 probed entries per recorded state; the probe count tells which
    # kernel ran, the estimate is the same either way.
    csr = G.rmat(14, seed=21)
    s = 0.5 / csr.d_max
    rows = G.random_rows(csr.n, 64, seed=2)
    with graph(csr) as g:
        setup(g, M.MCMF_SAMPLER_AUTO, 0)
        auto = gpu_diag(g, "exp", N, K, s, seed=3, rows=rows, want_digest=True, stats=True)
        setup(g, M.MCMF_SAMPLER_WIDE, 0)
        wide = gpu_diag(g, "exp", N, K, s, seed=3, rows=rows, want_digest=True, stats=True)
        setup(g, M.MCMF_SAMPLER_EDGE, 0)
        edge = gpu_diag(g, "exp", N, K, s, seed=3, rows=rows, want_digest=True, stats=True)
    takes = _auto_takes_wide(csr, N, K)
    assert takes == (N == 16)  # the two cases fall on either side of the rule
    want = wide if takes else edge
    assert auto["stats"]["gather_probes"] == want["stats"]["gather_probes"]
    if takes:
        assert wide["stats"]["gather_probes"] < edge["stats"]["gather_probes"]
    assert np.array_equal(auto["digest"], edge["digest"])
    assert_close(auto["d"], edge["d"], 1e-10, what=f"AUTO N={N} K={K}")
