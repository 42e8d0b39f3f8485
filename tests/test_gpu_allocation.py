"""Walk allocation p ~ ||C_i||_2 (Eq. initial_prob, N_i = N_s P(l0 = i)):
the library's walks per start row equal the oracle's allocation exactly, and
with those counts its estimates match the oracle (paths bit-exact, 1e-10),
for the full diagonal, row subsets (several visit-record chunks), the action
on symmetric and on directed graphs, and FP32 weights.  MCMF_ALLOC_NORM is
the paper's rounding, under which a start row may get no walk;
MCMF_ALLOC_NORM_MIN1 gives every start row one at least.  Rows whose whole
neighbourhood got no walk return exactly the H part (Section 4.1)."""
import numpy as np
import pytest
import scipy.sparse as sp

import graphgen as G
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from _gpu import assert_close, default_sampler, fn_struct, graph, oracle_fn  # noqa: E402
from paper_2308_01037_amd import mcmf as M  # noqa: E402


def run(g, kind, fn, scale, Ns, K, v=None, rows=None, seed=2, precision=M.MCMF_PRECISION_FP64,
        alloc=M.MCMF_ALLOC_NORM):
    n = g.info["n"]
    walks = torch.zeros(n, dtype=torch.int32, device="cuda")
    dig = torch.zeros(n, dtype=torch.int64, device="cuda")
    st = M.mcmf_stats()
    opts = M.make_opts(seed=seed, stream=torch.cuda.current_stream().cuda_stream, path_digest=dig,
                       allocation=alloc, walks_out=walks, precision=precision)
    f = fn_struct(fn, scale)
    if kind == "action":
        out = torch.empty(n, dtype=torch.float64, device="cuda")
        M.mcmf_action(g.handle, f, torch.as_tensor(v, device="cuda"), Ns, K, opts, out, st)
    else:
        rt = None if rows is None else torch.as_tensor(np.asarray(rows, np.int32), device="cuda")
        out = torch.empty(n if rows is None else len(rows), dtype=torch.float64, device="cuda")
        M.mcmf_diag(g.handle, f, rt, 0 if rows is None else len(rows), Ns, K, opts, out, st)
    torch.cuda.synchronize()
    return (out.cpu().numpy(), walks.cpu().numpy().astype(np.int64), dig.cpu().numpy().view(np.uint64),
            st.as_dict())


def starts_of(csr, rows):
    if rows is None:
        return np.nonzero(csr.deg > 0)[0].astype(np.int32)
    flags = np.zeros(csr.n, bool)
    for r in rows:
        flags[csr.col[csr.row_ptr[r]:csr.row_ptr[r + 1]]] = True
    flags &= csr.deg > 0
    return np.nonzero(flags)[0].astype(np.int32)


ALLOCS = [(M.MCMF_ALLOC_NORM, False), (M.MCMF_ALLOC_NORM_MIN1, True)]


@pytest.mark.parametrize("maker", [lambda: G.rmat(11, seed=4),
                                   lambda: G.with_random_weights(G.rmat(10, seed=5), seed=6,
                                                                 negative_fraction=0.3)])
@pytest.mark.parametrize("subset", [False, True])
@pytest.mark.parametrize("per_row", [40, 0.5])
@pytest.mark.parametrize("alloc,min_one", ALLOCS)
def test_diag_with_norm_allocation(maker, subset, per_row, alloc, min_one, monkeypatch):
    csr = maker()
    rows = np.arange(3, csr.n, 11) if subset else None
    if subset:
        monkeypatch.setenv("MCMF_DIAG_CHUNK_BYTES", str(400_000))  # many chunks of unequal rows
    K, Ns = 12, int(per_row * csr.n)
    scale = 1.0 / float(np.max(abs(csr.to_scipy()).sum(axis=1)))
    with graph(csr) as g:
        d, walks, dig, st = run(g, "diag", "exp", scale, Ns, K, rows=rows, alloc=alloc)
    want_walks = oracle.allocation(csr, Ns, starts_of(csr, rows), min_one=min_one)
    assert np.array_equal(walks, want_walks)
    if per_row < 1 and not min_one:
        assert np.any(want_walks[starts_of(csr, rows)] == 0)
    assert st["walks"] == int(want_walks.sum())
    assert st["start_rows"] == int(np.count_nonzero(want_walks))
    o = oracle.diag(csr, oracle_fn("exp"), N=1, K=K, scale=scale, seed=2, rows=rows, want_digest=True,
                    walks=want_walks, sampler=default_sampler(csr))
    assert np.array_equal(dig, o["digest"])
    assert st["walk_steps"] == o["steps"]
    assert_close(d, o["d"], 1e-10, atol=1e-13 * np.max(np.abs(o["d"])))


@pytest.mark.parametrize("directed", [False, True])
@pytest.mark.parametrize("per_row", [20, 0.5])
@pytest.mark.parametrize("alloc,min_one", ALLOCS)
def test_action_with_norm_allocation(directed, per_row, alloc, min_one):
    if directed:
        rng = np.random.default_rng(8)
        src, dst = rng.integers(0, 900, 6000), rng.integers(0, 900, 6000)
        keep = src != dst
        csr = G.from_edges(900, src[keep], dst[keep], symmetric=False)
        flags = 0
    else:
        csr = G.barabasi_albert(3000, 4, seed=3)
        flags = M.MCMF_SYMMETRIC
    K, Ns = 14, int(per_row * csr.n)
    v = np.random.default_rng(1).random(csr.n)
    scale = 0.5 / max(1, csr.d_max)
    with graph(csr, flags=flags) as g:
        y, walks, dig, st = run(g, "action", "resolvent", scale, Ns, K, v=v, alloc=alloc)
        y32, walks32, dig32, _ = run(g, "action", "resolvent", scale, Ns, K, v=v,
                                     precision=M.MCMF_PRECISION_FP32_WEIGHTS, alloc=alloc)
    want_walks = oracle.allocation(csr, Ns, starts_of(csr, None), symmetric=not directed,
                                   min_one=min_one)
    assert np.array_equal(walks, want_walks) and np.array_equal(walks32, want_walks)
    o = oracle.action(csr, oracle_fn("resolvent"), v, N=1, K=K, scale=scale, seed=2, want_digest=True,
                      walks=want_walks, sampler=default_sampler(csr))
    assert np.array_equal(dig, o["digest"]) and np.array_equal(dig32, o["digest"])
    assert st["walk_steps"] == o["steps"]
    assert_close(y, o["y"], 1e-10, atol=1e-13 * np.max(np.abs(o["y"])))
    assert np.max(np.abs(y32 - y)) <= 2 * K * 2.0 ** -24 * np.max(np.abs(y)) * 4


def test_rows_without_walks_keep_only_H():
    # K_50 next to the pair 50-51 (node 50 with a self-loop): with N_s = 100
    # the pair gets no walk, so its outputs are exactly the H terms, while the
    # K_50 rows match the oracle.
    src, dst = np.triu_indices(50, k=1)
    csr = G.from_edges(52, np.concatenate([src, [50, 50]]), np.concatenate([dst, [51, 50]]),
                       keep_loops=True)
    K, s = 8, 0.05
    c = oracle.coeffs(oracle.FN_EXP, K)
    v = np.linspace(0.5, 1.5, csr.n)
    with graph(csr) as g:
        d, walks, dig, st = run(g, "diag", "exp", s, 100, K)
        y, walks_a, _, _ = run(g, "action", "exp", s, 100, K, v=v)
    assert walks[50] == 0 and walks[51] == 0 and np.all(walks[:50] == 2)
    assert np.array_equal(walks, walks_a)
    # Exact up to the rounding of c0 + c1 x itself (the device may fuse it).
    h = np.array([c[0] + c[1] * (s * 1.0), c[0]])
    assert np.all(np.abs(d[50:] - h) <= 2 * np.finfo(float).eps * h)
    h = np.array([c[0] * v[50] + c[1] * (s * (v[50] + v[51])), c[0] * v[51] + c[1] * (s * v[50])])
    assert np.all(np.abs(y[50:] - h) <= 2 * np.finfo(float).eps * h)
    assert dig[50] == 0 and dig[51] == 0 and st["start_rows"] == 50
    o = oracle.diag(csr, oracle_fn("exp"), N=1, K=K, scale=s, seed=2, walks=walks, want_digest=True,
                    sampler=default_sampler(csr))
    assert np.array_equal(dig, o["digest"])
    assert_close(d, o["d"], 1e-10)
    o = oracle.action(csr, oracle_fn("exp"), v, N=1, K=K, scale=s, seed=2, walks=walks,
                      sampler=default_sampler(csr))
    assert_close(y, o["y"], 1e-10)


def test_weighted_directed_is_refused():
    a = sp.random(50, 50, density=0.1, random_state=3, format="csr")
    a.setdiag(0)
    a.eliminate_zeros()
    csr = G.CSR(50, a.indptr.astype(np.int64), a.indices.astype(np.int32), a.data.astype(np.float64))
    with graph(csr, flags=0) as g:
        out = torch.empty(50, dtype=torch.float64, device="cuda")
        opts = M.make_opts(allocation=M.MCMF_ALLOC_NORM)
        with pytest.raises(M.MCMFError) as e:
            M.mcmf_action(g.handle, fn_struct("exp", 0.1), torch.ones(50, dtype=torch.float64, device="cuda"),
                          100, 5, opts, out)
        assert e.value.status == M.MCMF_E_UNSUPPORTED
