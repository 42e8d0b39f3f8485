"""The alias sampler for weighted rows on the GPU.

MCMF_SAMPLER_ALIAS makes a weighted walk step read one 16-byte record of
Walker's alias tables (built on the device by Vose's construction) instead
of searching the running sums of |a|.  The oracle's alias mode builds the
same tables from the same definition, so the library's walks must match it
path for path (digests, step counts) with estimates within 1e-10 relative:
diagonal and action, row subsets, signed weights, rows of zeros, a weight
cutoff, walk allocation by column norm, FP32 weights within the stated
bound, and batched requests equal to single calls.
"""
import numpy as np
import pytest

import graphgen as G
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from _gpu import assert_close, gpu_action, gpu_diag, graph, oracle_fn  # noqa: E402
from _reqs import Req, run_batch  # noqa: E402
from paper_2308_01037_amd import mcmf as M  # noqa: E402


def use(g, action=M.MCMF_SAMPLER_ALIAS, diag=M.MCMF_SAMPLER_ALIAS):
    t = M.mcmf_graph_get_tuning(g.handle)
    t.action_sampler, t.diag_sampler, t.hub_count = action, diag, 0
    M.mcmf_graph_set_tuning(g.handle, t)


def weighted(scale=11, seed=2, negative_fraction=0.3):
    return G.with_random_weights(G.rmat(scale, seed=seed), seed=seed + 1,
                                 negative_fraction=negative_fraction)


def row_abs_max(csr):
    return float(np.max(np.add.reduceat(np.abs(csr.val), csr.row_ptr[:-1][csr.deg > 0])))


@pytest.mark.parametrize("fn", ["exp", "resolvent"])
@pytest.mark.parametrize("rows", [None, "subset"])
def test_alias_walks_match_the_oracle(fn, rows):
    csr = weighted()
    s = 0.6 / row_abs_max(csr)
    K, N = 12, 40
    sel = None if rows is None else G.random_rows(csr.n, 300, seed=4)
    v = G.uniform_vector(csr.n, seed=5)
    with graph(csr) as g:
        use(g)
        d = gpu_diag(g, fn, N, K, s, seed=3, rows=sel, want_digest=True, stats=True)
        a = gpu_action(g, fn, v, N, K, s, seed=3, want_digest=True, stats=True)
        use(g, M.MCMF_SAMPLER_EDGE, M.MCMF_SAMPLER_EDGE)
        d_cdf = gpu_diag(g, fn, N, K, s, seed=3, rows=sel, want_digest=True)
    od = oracle.diag(csr, oracle_fn(fn), N=N, K=K, scale=s, seed=3, rows=sel, want_digest=True,
                     sampler="alias")
    oa = oracle.action(csr, oracle_fn(fn), v, N=N, K=K, scale=s, seed=3, want_digest=True,
                       sampler="alias")
    assert np.array_equal(d["digest"], od["digest"])
    assert d["stats"]["walk_steps"] == od["steps"]
    assert_close(d["d"], od["d"], 1e-10, what="alias diag")
    assert np.array_equal(a["digest"], oa["digest"])
    assert a["stats"]["walk_steps"] == oa["steps"]
    assert_close(a["y"], oa["y"], 1e-10, what="alias action")
    # The running sums walk other paths (same law).
    assert not np.array_equal(d["digest"], d_cdf["digest"])


def test_alias_with_zero_rows_cutoff_and_norm_allocation():
    # A non-symmetric weighted graph with exact zeros, a row of zeros only
    # and rows of one entry; a weight cutoff; walks allocated by column norm.
    rng = np.random.default_rng(9)
    n = 500
    src = np.concatenate([rng.integers(0, n, 4000), np.full(5, 7)])
    dst = np.concatenate([rng.integers(0, n, 4000), np.arange(20, 25)])
    base = G.from_edges(n, src, dst, symmetric=False)
    val = rng.uniform(-1.5, 2.0, base.nnz)
    val[rng.random(base.nnz) < 0.1] = 0.0
    val[base.row_ptr[7]:base.row_ptr[8]] = 0.0
    csr = G.CSR(base.n, base.row_ptr, base.col, val, "zeros")
    s = 0.5 / row_abs_max(csr)
    v = G.uniform_vector(n, seed=1)
    with graph(csr, flags=0) as g:
        use(g)
        a = gpu_action(g, "exp", v, 30, 10, s, seed=6, cutoff=1e-3, want_digest=True, stats=True)
        oa = oracle.action(csr, oracle_fn("exp"), v, N=30, K=10, scale=s, seed=6, cutoff=1e-3,
                           want_digest=True, sampler="alias")
        assert np.array_equal(a["digest"], oa["digest"])
        assert a["stats"]["walk_steps"] == oa["steps"]
        assert_close(a["y"], oa["y"], 1e-10, what="alias action, zeros and cutoff")
    # Walks allocated by column norm (symmetric weighted graphs only).
    sym = weighted(10, seed=12)
    s = 0.5 / row_abs_max(sym)
    n = sym.n
    v = G.uniform_vector(n, seed=2)
    with graph(sym) as g:
        use(g)
        walks = torch.zeros(n, dtype=torch.int32, device="cuda")
        dig = torch.zeros(n, dtype=torch.int64, device="cuda")
        out = torch.empty(n, dtype=torch.float64, device="cuda")
        M.mcmf_action(g.handle, M.make_fn(M.MCMF_FN_RESOLVENT, s), torch.as_tensor(v, device="cuda"), 40 * n, 9,
                      M.make_opts(seed=2, allocation=M.MCMF_ALLOC_NORM, walks_out=walks, path_digest=dig,
                                  stream=torch.cuda.current_stream().cuda_stream), out)
        torch.cuda.synchronize()
    wk = walks.cpu().numpy().astype(np.int64)
    oa = oracle.action(sym, oracle_fn("resolvent"), v, N=1, K=9, scale=s, seed=2, want_digest=True,
                       walks=wk, sampler="alias")
    assert np.array_equal(dig.cpu().numpy().view(np.uint64), oa["digest"])
    assert_close(out.cpu().numpy(), oa["y"], 1e-10, what="alias action, norm allocation")


def test_alias_fp32_weights_within_bound():
    csr = weighted(12, seed=5, negative_fraction=0.0)
    s = 0.7 / row_abs_max(csr)
    K, N = 16, 64
    with graph(csr) as g:
        use(g)
        stream = torch.cuda.current_stream().cuda_stream
        res = {}
        for prec in (M.MCMF_PRECISION_FP64, M.MCMF_PRECISION_FP32_WEIGHTS):
            out = torch.empty(csr.n, dtype=torch.float64, device="cuda")
            M.mcmf_diag(g.handle, M.make_fn(M.MCMF_FN_EXP, s), None, 0, N, K,
                        M.make_opts(seed=8, precision=prec, stream=stream), out)
            torch.cuda.synchronize()
            res[prec] = out.cpu().numpy()
    c = oracle.coeffs(oracle.FN_EXP, K)
    mc = np.abs(res[M.MCMF_PRECISION_FP64] - c[0])  # non-negative terms: sum|terms| = MC part
    bound = 2 * K * 2.0 ** -24 * mc + 4 * np.finfo(np.float64).eps * np.abs(res[M.MCMF_PRECISION_FP64])
    assert np.all(np.abs(res[M.MCMF_PRECISION_FP32_WEIGHTS] - res[M.MCMF_PRECISION_FP64]) <= bound + 1e-300)
    assert not np.array_equal(res[M.MCMF_PRECISION_FP32_WEIGHTS], res[M.MCMF_PRECISION_FP64])


def test_batched_alias_requests_equal_single_calls():
    csr = weighted(11, seed=7)
    s = 0.6 / row_abs_max(csr)
    with graph(csr) as g:
        use(g)
        sel = G.random_rows(csr.n, 100, seed=3)
        reqs = [Req(g, csr, M.MCMF_REQ_DIAG, "exp", s, 48, 10, seed=1),
                Req(g, csr, M.MCMF_REQ_DIAG, "resolvent", s, 16, 12, seed=2, request=1, rows=sel),
                Req(g, csr, M.MCMF_REQ_ACTION, "exp", s, 200, 9, seed=3, request=2,
                    v=G.uniform_vector(csr.n, seed=4))]
        want = [q.single() for q in reqs]
        got, _ = run_batch(reqs)
    for r, w in zip(got, want):
        assert np.array_equal(r["digest"], w["digest"])
        assert r["steps"] == w["steps"]
        assert_close(r["x"], w["x"], 1e-10)
    od = oracle.diag(csr, oracle_fn("exp"), N=48, K=10, scale=s, seed=1, want_digest=True, sampler="alias")
    assert np.array_equal(got[0]["digest"], od["digest"])
    assert_close(got[0]["x"], od["d"], 1e-10, what="batched alias diag vs oracle")


def test_alias_layout_argument_errors():
    with graph(G.rmat(8, seed=1)) as g:  # unweighted: no alias records
        for field in ("action_sampler", "diag_sampler"):
            t = M.mcmf_graph_get_tuning(g.handle)
            setattr(t, field, M.MCMF_SAMPLER_ALIAS)
            t.hub_count = 0
            with pytest.raises(M.MCMFError) as e:
                M.mcmf_graph_set_tuning(g.handle, t)
            assert e.value.status == M.MCMF_E_ARG
    with graph(weighted(8)) as g:
        use(g, M.MCMF_SAMPLER_ALIAS, M.MCMF_SAMPLER_EDGE)
        t = M.mcmf_graph_get_tuning(g.handle)
        assert (t.action_sampler, t.diag_sampler) == (M.MCMF_SAMPLER_ALIAS, M.MCMF_SAMPLER_EDGE)


def test_tuner_times_the_alias_layout():
    csr = weighted(12, seed=3)
    s = 0.6 / row_abs_max(csr)
    with graph(csr) as g:
        a = M.mcmf_tune(g.handle, M.make_fn(M.MCMF_FN_EXP, s), 64, 12).as_dict()
        assert all(ms > 0 for ms in a["alias_ms"])
        if a["action_sampler"] == M.MCMF_SAMPLER_ALIAS:
            assert a["alias_ms"][0] < min(a["action_ms"])
        else:
            assert a["alias_ms"][0] >= min(a["action_ms"])
        if a["diag_sampler"] == M.MCMF_SAMPLER_ALIAS:
            assert a["alias_ms"][1] < min(a["diag_ms"])
        else:
            assert a["alias_ms"][1] >= min(a["diag_ms"])
        # Whatever it picked, the walks match the oracle in that layout.
        r = gpu_diag(g, "exp", 32, 10, s, seed=4, want_digest=True)
    mode = "alias" if a["diag_sampler"] == M.MCMF_SAMPLER_ALIAS else "cdf"
    o = oracle.diag(csr, oracle_fn("exp"), N=32, K=10, scale=s, seed=4, want_digest=True, sampler=mode)
    assert np.array_equal(r["digest"], o["digest"])
    assert_close(r["d"], o["d"], 1e-10)


def test_graph_keeps_running_sums_when_alias_records_do_not_fit(monkeypatch):
    # Creating a weighted graph never fails for want of room for its alias
    # records: it keeps the running sums (EDGE), whose walks are the oracle's
    # default mode; asking for ALIAS then reports MCMF_E_NOMEM.
    csr = weighted(9, seed=4)
    s = 0.5 / row_abs_max(csr)
    monkeypatch.setenv("MCMF_TEST_FAIL_ALIAS", "1")
    with graph(csr) as g:
        t = M.mcmf_graph_get_tuning(g.handle)
        assert (t.action_sampler, t.diag_sampler) != (M.MCMF_SAMPLER_ALIAS, M.MCMF_SAMPLER_ALIAS)
        assert t.diag_sampler != M.MCMF_SAMPLER_ALIAS
        r = gpu_diag(g, "exp", 24, 8, s, seed=2, want_digest=True)
        o = oracle.diag(csr, oracle_fn("exp"), N=24, K=8, scale=s, seed=2, want_digest=True)
        assert np.array_equal(r["digest"], o["digest"])
        assert_close(r["d"], o["d"], 1e-10)
        with pytest.raises(M.MCMFError) as e:
            use(g)
        assert e.value.status == M.MCMF_E_NOMEM
        monkeypatch.delenv("MCMF_TEST_FAIL_ALIAS")
        use(g)  # room again: built on demand
        r = gpu_diag(g, "exp", 24, 8, s, seed=2, want_digest=True)
    o = oracle.diag(csr, oracle_fn("exp"), N=24, K=8, scale=s, seed=2, want_digest=True, sampler="alias")
    assert np.array_equal(r["digest"], o["digest"])
    assert_close(r["d"], o["d"], 1e-10)
