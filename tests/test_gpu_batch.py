"""Batched execution (mcmf_batch) on the GPU.

A request run inside a batch draws the walks its own single call draws (same
keyed Philox counters), so per request: path digests and walk-step counts
equal the single call's exactly, and estimates agree within 1e-10 relative
(only the order of FP64 additions differs).  A few requests are also checked
against the oracle directly, and a batch recorded into a hipGraph must give
the eager batch's results on every launch.
"""
import os

import numpy as np
import pytest

import graphgen as G
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from _gpu import assert_close, assert_mc_part_close, fn_struct, graph, oracle_fn  # noqa: E402
from paper_2308_01037_amd import mcmf as M  # noqa: E402

RTOL = 1e-10


class Req:
    """One request: its arguments, its single-call result and its batch slot."""

    def __init__(self, g, csr, kind, fn, scale, N, K, seed=0, request=0, rows=None,
                 precision=M.MCMF_PRECISION_FP64, cutoff=0.0, v=None):
        self.g, self.csr, self.kind, self.fn, self.scale = g, csr, kind, fn, scale
        self.N, self.K, self.seed, self.request, self.rows = N, K, seed, request, rows
        self.precision, self.cutoff = precision, cutoff
        n = csr.n
        if kind == M.MCMF_REQ_ACTION:
            self.v = np.ones(n) if v is None else np.asarray(v, dtype=np.float64)
            self.count = n
        else:
            self.v = None
            self.count = n if rows is None else len(rows)

    def _dev(self):
        vt = None if self.v is None else torch.as_tensor(self.v, device="cuda")
        rt = None if self.rows is None else torch.as_tensor(np.asarray(self.rows, np.int32),
                                                            device="cuda")
        return vt, rt

    def single(self):
        n = self.csr.n
        vt, rt = self._dev()
        out = torch.empty(max(self.count, 1), dtype=torch.float64, device="cuda")
        dig = torch.zeros(n, dtype=torch.int64, device="cuda")
        st = M.mcmf_stats()
        opts = M.make_opts(seed=self.seed, request_id=self.request, precision=self.precision,
                           weight_cutoff=self.cutoff,
                           stream=torch.cuda.current_stream().cuda_stream, path_digest=dig)
        f = fn_struct(self.fn, self.scale)
        if self.kind == M.MCMF_REQ_ACTION:
            M.mcmf_action(self.g.handle, f, vt, self.N, self.K, opts, out, st)
        else:
            M.mcmf_diag(self.g.handle, f, rt, 0 if self.rows is None else len(self.rows), self.N,
                        self.K, opts, out, st)
        torch.cuda.synchronize()
        return {"x": out.cpu().numpy()[:self.count], "digest": dig.cpu().numpy().view(np.uint64),
                "steps": st.walk_steps}

    def make(self, host=False):
        """The mcmf_request plus the buffers it writes."""
        n = self.csr.n
        if host:
            vt = None if self.v is None else self.v.copy()
            rt = None if self.rows is None else np.asarray(self.rows, np.int32)
            out = np.full(max(self.count, 1), np.nan)
            dig = np.zeros(n, dtype=np.uint64)
        else:
            vt, rt = self._dev()
            out = torch.full((max(self.count, 1),), float("nan"), dtype=torch.float64, device="cuda")
            dig = torch.zeros(n, dtype=torch.int64, device="cuda")
        r = M.make_request(self.kind, self.g.handle, fn_struct(self.fn, self.scale), self.K, self.N,
                           out, rows=rt, v=vt, seed=self.seed, request_id=self.request,
                           precision=self.precision, weight_cutoff=self.cutoff, path_digest=dig)
        return r, out, dig

    @staticmethod
    def fetch(out, dig, count):
        if isinstance(out, np.ndarray):
            return {"x": out[:count].copy(), "digest": dig.copy()}
        return {"x": out.cpu().numpy()[:count], "digest": dig.cpu().numpy().view(np.uint64)}

    def h(self):
        """The deterministic part c0 + c1 s a_ii (diag) or c0 v + c1 s A v (action)."""
        c = (oracle.coeffs(oracle_fn(self.fn), self.K) if isinstance(self.fn, str)
             else np.asarray(self.fn, float))
        A = self.csr.to_scipy()
        if self.kind == M.MCMF_REQ_ACTION:
            h = c[0] * self.v
            return h + (c[1] * self.scale * (A @ self.v) if self.K >= 1 else 0.0)
        h = c[0] + (c[1] * self.scale * A.diagonal() if self.K >= 1 else 0.0)
        h = np.broadcast_to(h, (self.csr.n,)).copy()
        return h if self.rows is None else h[np.asarray(self.rows)]


def run_batch(reqs, host=False, use_graph=False, stream=True):
    made = [q.make(host) for q in reqs]
    o = M.mcmf_batch_opts()
    o.use_graph = 1 if use_graph else 0
    o.stream = torch.cuda.current_stream().cuda_stream if stream else None
    st = M.mcmf_stats()
    M.mcmf_batch([m[0] for m in made], o, st)
    torch.cuda.synchronize()
    res = []
    for q, (r, out, dig) in zip(reqs, made):
        assert r.status == M.MCMF_OK
        d = Req.fetch(out, dig, q.count)
        d["steps"] = r.walk_steps
        res.append(d)
    return res, st.as_dict()


def check_same(q, got, want, what):
    # Paths and step counts exact; estimates to 1e-10 relative, full value and
    # Monte Carlo part.
    assert np.array_equal(got["digest"], want["digest"]), f"{what}: walk paths differ"
    assert got["steps"] == want["steps"], what
    h = q.h()
    assert_close(got["x"], want["x"], RTOL, atol=1e-13 * np.max(np.abs(want["x"]), initial=0.0),
                 what=what)
    assert_mc_part_close(got["x"], want["x"], h, RTOL, what=what)


@pytest.fixture(scope="module")
def graphs():
    csrs = {
        "rmat11": G.rmat(11, seed=7),
        "er": G.erdos_renyi_dense(700, 0.02, seed=8),
        "torus": G.torus2d(40, 40),
        "weighted": G.with_random_weights(G.rmat(10, seed=9), seed=10, negative_fraction=0.3),
        "ba": G.barabasi_albert(3000, 5, seed=11),
    }
    gs = {k: graph(v) for k, v in csrs.items()}
    yield {k: (gs[k], csrs[k]) for k in csrs}
    for g in gs.values():
        g.close()


def _mixed(graphs):
    A, D = M.MCMF_REQ_ACTION, M.MCMF_REQ_DIAG
    g1, c1 = graphs["rmat11"]
    g2, c2 = graphs["er"]
    g3, c3 = graphs["torus"]
    g4, c4 = graphs["weighted"]
    g5, c5 = graphs["ba"]
    s4 = 1.0 / float(np.max(abs(c4.to_scipy()).sum(axis=1)))
    rng = np.random.default_rng(3)
    return [
        Req(g1, c1, A, "exp", 1.0 / c1.d_max, 96, 20, seed=1, request=0),
        Req(g1, c1, D, "exp", 1.0 / c1.d_max, 96, 20, seed=1, request=1),
        Req(g2, c2, D, "resolvent", 0.05, 200, 15, seed=2, rows=rng.choice(c2.n, 50, replace=False)),
        Req(g3, c3, A, "resolvent", 0.2, 33, 25, seed=3, v=rng.standard_normal(c3.n)),
        Req(g4, c4, D, "exp", s4, 64, 12, seed=4, precision=M.MCMF_PRECISION_FP32_WEIGHTS),
        Req(g4, c4, A, "exp", s4, 130, 12, seed=4, cutoff=1e-3),
        Req(g5, c5, D, "exp", 1.0 / c5.d_max, 17, 30, seed=5, cutoff=1e-6,
            rows=np.arange(0, c5.n, 7)),
        Req(g5, c5, A, [1.0, 0.5, 0.25, 0.125, 0.0625], 0.1, 257, 4, seed=6,
            precision=M.MCMF_PRECISION_FP32_WEIGHTS),
        Req(g2, c2, D, "exp", 0.1, 10, 1),   # K = 1: no walks
        Req(g2, c2, A, "exp", 0.1, 10, 0),   # K = 0: c0 v
        Req(g3, c3, D, "exp", 0.25, 5, 2, rows=np.array([], np.int32)),  # empty row list
    ]


def test_mixed_batch_equals_single_calls(graphs):
    reqs = _mixed(graphs)
    want = [q.single() for q in reqs]
    got, st = run_batch(reqs)
    for i, (q, g, w) in enumerate(zip(reqs, got, want)):
        check_same(q, g, w, f"request {i}")
    assert st["walk_steps"] == sum(w["steps"] for w in want)


def test_mixed_batch_host_buffers_and_library_stream(graphs):
    reqs = _mixed(graphs)[:6]
    want = [q.single() for q in reqs]
    got, _ = run_batch(reqs, host=True, stream=False)
    for i, (q, g, w) in enumerate(zip(reqs, got, want)):
        check_same(q, g, w, f"request {i}")


def test_batch_against_oracle(graphs):
    g1, c1 = graphs["rmat11"]
    g4, c4 = graphs["weighted"]
    A, D = M.MCMF_REQ_ACTION, M.MCMF_REQ_DIAG
    reqs = [Req(g1, c1, D, "exp", 1.0 / c1.d_max, 40, 10, seed=9, request=2),
            Req(g4, c4, A, "resolvent", 0.1, 50, 9, seed=9, request=3),
            Req(g1, c1, A, "exp", 1.0 / c1.d_max, 40, 10, seed=9, request=4, cutoff=1e-4)]
    got, _ = run_batch(reqs)
    for q, r in zip(reqs, got):
        if q.kind == A:
            o = oracle.action(q.csr, oracle_fn(q.fn), q.v, N=q.N, K=q.K, scale=q.scale, seed=q.seed,
                              request=q.request, cutoff=q.cutoff, want_digest=True)
            x = o["y"]
        else:
            o = oracle.diag(q.csr, oracle_fn(q.fn), N=q.N, K=q.K, scale=q.scale, seed=q.seed,
                            request=q.request, cutoff=q.cutoff, rows=q.rows, want_digest=True)
            x = o["d"]
        assert np.array_equal(r["digest"], o["digest"])
        assert r["steps"] == o["steps"]
        assert_close(r["x"], x, RTOL, atol=1e-13 * np.max(np.abs(x)))
        assert_mc_part_close(r["x"], x, q.h(), RTOL)


def test_small_visit_chunks(graphs, monkeypatch):
    # A visit budget of about three start rows splits the diag requests over
    # many walk/gather launches, across request boundaries.
    reqs = _mixed(graphs)[:7]
    want = [q.single() for q in reqs]
    monkeypatch.setenv("MCMF_DIAG_CHUNK_BYTES", str(3 * 200 * 14 * 12))
    got, _ = run_batch(reqs)
    for i, (q, g, w) in enumerate(zip(reqs, got, want)):
        check_same(q, g, w, f"request {i}")


def test_graph_launch_matches_eager(graphs):
    # The batch recorded into a hipGraph and launched, three times, with eager
    # batches and synchronisations in between: every launch equals eager.
    reqs = _mixed(graphs)[:8]
    eager, _ = run_batch(reqs)
    for rep in range(3):
        got, _ = run_batch(reqs, use_graph=True)
        for i, (q, g, w) in enumerate(zip(reqs, got, eager)):
            check_same(q, g, w, f"graph launch {rep}, request {i}")
        again, _ = run_batch(reqs)
        for i, (q, g, w) in enumerate(zip(reqs, again, eager)):
            check_same(q, g, w, f"eager after launch {rep}, request {i}")


def test_many_small_requests(graphs):
    # 64 requests on one graph with distinct request ids: one batch equals 64
    # single calls.
    g1, c1 = graphs["rmat11"]
    kinds = [M.MCMF_REQ_DIAG, M.MCMF_REQ_ACTION]
    rng = np.random.default_rng(12)
    reqs = [Req(g1, c1, kinds[i % 2], "exp", 1.0 / c1.d_max, 8 + (i % 5) * 16, 6 + i % 7,
                seed=21, request=100 + i,
                rows=(rng.choice(c1.n, 20, replace=False) if i % 4 == 0 else None))
            for i in range(64)]
    want = [q.single() for q in reqs]
    got, _ = run_batch(reqs)
    for i, (q, g, w) in enumerate(zip(reqs, got, want)):
        check_same(q, g, w, f"request {i}")


def test_batch_rejects_before_any_output():
    # A diag request on a graph not created as symmetric fails the batch with
    # that request's status; the valid request before it writes nothing.
    csr = G.rmat(8, seed=1)
    with graph(csr) as gs, graph(csr, flags=0) as gn:
        ok = Req(gs, csr, M.MCMF_REQ_ACTION, "exp", 0.1, 8, 5)
        bad = Req(gn, csr, M.MCMF_REQ_DIAG, "exp", 0.1, 8, 5)
        r0, out0, _ = ok.make()
        r1, out1, _ = bad.make()
        with pytest.raises(M.MCMFError) as e:
            M.mcmf_batch([r0, r1])
        assert e.value.status == M.MCMF_E_NOT_SYMMETRIC
        assert r1.status == M.MCMF_E_NOT_SYMMETRIC and r0.status == M.MCMF_OK
        torch.cuda.synchronize()
        assert torch.isnan(out0).all() and torch.isnan(out1).all()
        rows = torch.tensor([0, csr.n], dtype=torch.int32, device="cuda")
        out2 = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
        r2 = M.make_request(M.MCMF_REQ_DIAG, gs.handle, fn_struct("exp", 0.1), 5, 8, out2, rows=rows)
        r0, out0, _ = ok.make()
        with pytest.raises(M.MCMFError) as e:
            M.mcmf_batch([r0, r2])
        assert e.value.status == M.MCMF_E_ARG and r2.status == M.MCMF_E_ARG
        torch.cuda.synchronize()
        assert torch.isnan(out0).all() and torch.isnan(out2).all()
