"""GPU parity: the HIP library (through its C ABI) against the CPU oracle on
the same seeded inputs.

Bar: walk paths bit-exact (per-start-row path digests equal), estimates
within 1e-10 relative in FP64, element by element, both for the full value
and for its Monte Carlo part (q for the action, x - h for the diagonal).
"""
import numpy as np
import pytest

import graphgen as G
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from _gpu import (assert_close, assert_mc_part_close, default_sampler, gpu_action, gpu_diag, graph,  # noqa: E402
                  oracle_fn)
from paper_2308_01037_amd import mcmf as M  # noqa: E402

RTOL = 1e-10


def _h_action(g, fn, K, scale, v):
    c = oracle.coeffs(oracle_fn(fn), K) if isinstance(fn, str) else np.asarray(fn, float)
    h = c[0] * v
    if K >= 1:
        h = h + c[1] * scale * (g.to_scipy() @ v)
    return h


def _h_diag(g, fn, K, scale, rows=None):
    c = oracle.coeffs(oracle_fn(fn), K) if isinstance(fn, str) else np.asarray(fn, float)
    aii = g.to_scipy().diagonal()
    h = c[0] + (c[1] * scale * aii if K >= 1 else 0.0)
    h = np.broadcast_to(h, (g.n,)).copy()
    return h if rows is None else h[np.asarray(rows)]


def check_action(csr, fn, N, K, scale, seed=1, request=0, cutoff=0.0, v=None, flags=M.MCMF_SYMMETRIC,
                 host=False):
    v = np.ones(csr.n) if v is None else v
    o = oracle.action(csr, oracle_fn(fn), v, N=N, K=K, scale=scale, seed=seed, request=request,
                      cutoff=cutoff, want_q=True, want_digest=True, sampler=default_sampler(csr))
    with graph(csr, flags) as g:
        r = gpu_action(g, fn, v, N, K, scale, seed, request, cutoff, want_q=True, want_digest=True,
                       stats=True, host=host)
    assert np.array_equal(r["digest"], o["digest"]), "walk paths differ"
    assert_close(r["q"], o["q"], RTOL, what="q")
    assert_close(r["y"], o["y"], RTOL, what="y")
    assert_mc_part_close(r["y"], o["y"], _h_action(csr, fn, K, scale, v), RTOL, what="y")
    assert r["stats"]["walk_steps"] == o["steps"]
    return r, o


def check_diag(csr, fn, N, K, scale, seed=1, request=0, cutoff=0.0, rows=None, host=False):
    o = oracle.diag(csr, oracle_fn(fn), N=N, K=K, scale=scale, seed=seed, request=request,
                    cutoff=cutoff, rows=rows, want_digest=True, sampler=default_sampler(csr))
    with graph(csr) as g:
        r = gpu_diag(g, fn, N, K, scale, seed, request, cutoff, rows=rows, want_digest=True,
                     stats=True, host=host)
    assert np.array_equal(r["digest"], o["digest"]), "walk paths differ"
    assert_close(r["d"], o["d"], RTOL, what="d")
    assert_mc_part_close(r["d"], o["d"], _h_diag(csr, fn, K, scale, rows), RTOL, what="d")
    assert r["stats"]["walk_steps"] == o["steps"]
    return r, o


# ------------------------------------------------------------------ config 1


def test_er1000_exp_action_and_diag():
    # Erdos-Renyi G(1000, 0.01), exp(A), K = 30, N = 1000 walks per row.
    g = G.erdos_renyi_dense(1000, 0.01, seed=0)
    check_action(g, "exp", N=1000, K=30, scale=1.0)
    check_diag(g, "exp", N=1000, K=30, scale=1.0)


# ------------------------------------------------------------------ shapes and edges


GRAPHS = {
    "rmat10": lambda: G.rmat(10, seed=3),
    "star": lambda: G.star(3000),
    "kpq": lambda: G.complete_bipartite(5, 700),
    "isolated": lambda: G.from_edges(300, np.arange(0, 100), np.arange(100, 200)),
    "weighted": lambda: G.with_random_weights(G.rmat(9, seed=5), seed=6, negative_fraction=0.3),
    "grid": lambda: G.grid2d(30, 41),
}


@pytest.mark.parametrize("name", sorted(GRAPHS))
@pytest.mark.parametrize("fn", ["exp", "resolvent"])
def test_graph_families(name, fn):
    csr = GRAPHS[name]()
    scale = (0.5 if fn == "exp" else 0.85) / max(csr.d_max, 1)
    check_action(csr, fn, N=96, K=12, scale=scale, v=G.uniform_vector(csr.n, seed=4))
    check_diag(csr, fn, N=96, K=12, scale=scale)


@pytest.mark.parametrize("K", [0, 1, 2, 3, 30, 40])
def test_K_values(K):
    csr = G.rmat(9, seed=11)
    scale = 1.0 / csr.d_max
    check_action(csr, "exp", N=64, K=K, scale=scale)
    check_diag(csr, "exp", N=64, K=K, scale=scale)


@pytest.mark.parametrize("N", [1, 7, 64, 256, 1000])
def test_walk_counts(N):
    csr = G.rmat(8, seed=12)
    check_action(csr, "exp", N=N, K=10, scale=0.02)
    check_diag(csr, "exp", N=N, K=10, scale=0.02)


def test_custom_coefficients_and_seeds():
    csr = G.erdos_renyi_dense(400, 0.02, seed=9)
    c = np.random.default_rng(3).random(16)
    check_action(csr, c, N=50, K=15, scale=0.05, seed=2**40 + 17, request=77)
    check_diag(csr, c, N=50, K=15, scale=0.05, seed=2**40 + 17, request=77)


@pytest.mark.parametrize("rows", [[], [5], [17, 3, 17, 250, 0, 3], list(range(511, -1, -7))])
def test_row_subsets(rows):
    csr = G.rmat(9, seed=21)
    check_diag(csr, "exp", N=80, K=14, scale=0.01, rows=np.array(rows, dtype=np.int32))


def test_weight_cutoff():
    csr = G.rmat(9, seed=4)
    check_action(csr, "exp", N=50, K=30, scale=0.5 / csr.d_max, cutoff=1e-6)
    check_diag(csr, "exp", N=50, K=30, scale=0.5 / csr.d_max, cutoff=1e-6)


def test_nonsymmetric_action():
    rng = np.random.default_rng(8)
    csr = G.from_edges(500, rng.integers(0, 450, 3000), rng.integers(0, 500, 3000), symmetric=False)
    assert np.any(csr.deg == 0)
    check_action(csr, "exp", N=40, K=9, scale=0.1, v=G.uniform_vector(500, 1), flags=0)
    with graph(csr, 0) as g:
        with pytest.raises(M.MCMFError) as e:
            gpu_diag(g, "exp", 4, 5)
        assert e.value.status == M.MCMF_E_NOT_SYMMETRIC


def test_host_buffers():
    csr = G.rmat(8, seed=2)
    check_action(csr, "resolvent", N=33, K=8, scale=0.3 / csr.d_max, host=True)
    check_diag(csr, "resolvent", N=33, K=8, scale=0.3 / csr.d_max, rows=np.array([4, 9, 4]), host=True)


def test_multi_pass_gather_and_chunks(monkeypatch):
    # n above the LDS table size and N (K-1) visits beyond it: walks are
    # taken in several passes; a tiny chunk budget forces many chunks.
    csr = G.rmat(14, seed=7)
    rows = G.random_rows(csr.n, 12, seed=1)
    check_diag(csr, "exp", N=600, K=30, scale=0.5 / csr.d_max, rows=rows)
    monkeypatch.setenv("MCMF_DIAG_CHUNK_BYTES", str(3 * 600 * 29 * 12))
    check_diag(csr, "exp", N=600, K=30, scale=0.5 / csr.d_max, rows=rows)


def test_visit_buffer_halved_when_memory_refuses(monkeypatch):
    # A full diagonal whose visit records (about 1.2 GB) fit the default
    # buffer in one chunk.  With every allocation above 300 MiB refused, the
    # call halves its buffer until it fits (256 MiB: several chunks) and gives
    # the same walks and estimates; with the buffer size fixed by
    # MCMF_DIAG_CHUNK_BYTES it reports MCMF_E_NOMEM instead.
    csr = G.rmat(14, seed=3)
    N, K, s = 256, 40, 1.0 / csr.d_max
    with graph(csr) as g:
        whole = gpu_diag(g, "exp", N, K, s, want_digest=True, stats=True)
        assert whole["stats"]["walk_steps"] * 12 > 600 << 20
        monkeypatch.setenv("MCMF_TEST_FAIL_ALLOC_ABOVE", str(300 << 20))
        halved = gpu_diag(g, "exp", N, K, s, want_digest=True, stats=True)
        assert np.array_equal(whole["digest"], halved["digest"])
        assert whole["stats"]["walk_steps"] == halved["stats"]["walk_steps"]
        assert_close(halved["d"], whole["d"], RTOL, what="halved visit buffer")
        monkeypatch.setenv("MCMF_DIAG_CHUNK_BYTES", str(1 << 30))
        with pytest.raises(M.MCMFError) as e:
            gpu_diag(g, "exp", N, K, s)
        assert e.value.status == M.MCMF_E_NOMEM


@pytest.mark.parametrize("cap", [0, 7])
def test_item_map_fallback(monkeypatch, cap):
    # Gather items beyond the launch's item map find their start row by binary
    # search over the item offsets.  With the map capped at 0 or 7 entries the
    # full diagonal and a row subset (rows of several items each included)
    # take the same walks and give the uncapped estimates.
    csr = G.rmat(12, seed=5)
    rows = np.concatenate([np.argsort(csr.deg)[-3:], G.random_rows(csr.n, 40, seed=2)]).astype(np.int32)
    with graph(csr) as g:
        for r in (None, rows):
            want = gpu_diag(g, "exp", 64, 12, 1.0 / csr.d_max, rows=r, want_digest=True)
            monkeypatch.setenv("MCMF_TEST_ITEM_MAP_CAP", str(cap))
            got = gpu_diag(g, "exp", 64, 12, 1.0 / csr.d_max, rows=r, want_digest=True)
            monkeypatch.delenv("MCMF_TEST_ITEM_MAP_CAP")
            assert np.array_equal(got["digest"], want["digest"])
            assert_close(got["d"], want["d"], RTOL, what=f"item map capped at {cap}")


def test_validation_errors():
    csr = G.path(6)
    bad = G.CSR(6, csr.row_ptr.copy(), csr.col.copy())
    bad.col[2] = 99
    with pytest.raises(M.MCMFError) as e:
        graph(bad, M.MCMF_SYMMETRIC | M.MCMF_VALIDATE)
    assert e.value.status == M.MCMF_E_CSR
    rp = csr.row_ptr.copy()
    rp[3], rp[4] = rp[4], rp[3]
    with pytest.raises(M.MCMFError) as e:
        graph(G.CSR(6, rp, csr.col.copy()))
    assert e.value.status == M.MCMF_E_CSR
    asym = G.from_edges(5, [0, 1], [1, 2], symmetric=False)
    with pytest.raises(M.MCMFError) as e:
        graph(asym, M.MCMF_SYMMETRIC | M.MCMF_VALIDATE)
    assert e.value.status == M.MCMF_E_NOT_SYMMETRIC
    with graph(csr) as g:
        out = torch.full((2,), 7.0, dtype=torch.float64, device="cuda")
        with pytest.raises(M.MCMFError) as e:
            M.mcmf_diag(g.handle, M.make_fn(), torch.tensor([1, 6], dtype=torch.int32, device="cuda"),
                        2, 10, 5, None, out)
        assert e.value.status == M.MCMF_E_ARG
        assert torch.all(out == 7.0)
        with pytest.raises(M.MCMFError) as e:
            M.mcmf_action(g.handle, M.make_fn(), torch.ones(6, dtype=torch.float64, device="cuda"),
                          0, 5, None, torch.empty(6, dtype=torch.float64, device="cuda"))
        assert e.value.status == M.MCMF_E_ARG


def test_byte_budget(monkeypatch):
    monkeypatch.setenv("MCMF_TEST_FAIL_ALLOC", "1")
    with pytest.raises(M.MCMFError) as e:
        graph(G.path(10))
    assert e.value.status == M.MCMF_E_NOMEM


def test_repeat_is_deterministic():
    csr = G.rmat(10, seed=1)
    with graph(csr) as g:
        a = gpu_diag(g, "exp", 64, 20, 0.5 / csr.d_max, want_digest=True)
        b = gpu_diag(g, "exp", 64, 20, 0.5 / csr.d_max, want_digest=True)
        assert np.array_equal(a["digest"], b["digest"])
        assert_close(a["d"], b["d"], 1e-13)
        x = gpu_action(g, "exp", np.ones(csr.n), 64, 20, 0.5 / csr.d_max)
        y = gpu_action(g, "exp", np.ones(csr.n), 64, 20, 0.5 / csr.d_max)
        assert np.array_equal(x["y"], y["y"])
