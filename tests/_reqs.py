"""Shared helpers of the batched and served GPU tests: one request's
arguments, its single-call result, its mcmf_request form, and a mixed set of
requests over several graphs."""
import numpy as np
import torch

import graphgen as G
import oracle
from _gpu import assert_close, assert_mc_part_close, default_sampler, fn_struct, graph, oracle_fn
from paper_2308_01037_amd import mcmf as M

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

    def make(self, host=False, digest=True):
        """The mcmf_request plus the buffers it writes.  Without a path digest
        an action on an unweighted graph walks over value records."""
        n = self.csr.n
        if host:
            vt = None if self.v is None else self.v.copy()
            rt = None if self.rows is None else np.asarray(self.rows, np.int32)
            out = np.full(max(self.count, 1), np.nan)
            dig = np.zeros(n, dtype=np.uint64) if digest else None
        else:
            vt, rt = self._dev()
            out = torch.full((max(self.count, 1),), float("nan"), dtype=torch.float64, device="cuda")
            dig = torch.zeros(n, dtype=torch.int64, device="cuda") if digest else None
        r = M.make_request(self.kind, self.g.handle, fn_struct(self.fn, self.scale), self.K, self.N,
                           out, rows=rt, v=vt, seed=self.seed, request_id=self.request,
                           precision=self.precision, weight_cutoff=self.cutoff, path_digest=dig)
        return r, out, dig

    @staticmethod
    def fetch(out, dig, count):
        if isinstance(out, np.ndarray):
            return {"x": out[:count].copy(), "digest": None if dig is None else dig.copy()}
        return {"x": out.cpu().numpy()[:count],
                "digest": None if dig is None else dig.cpu().numpy().view(np.uint64)}

    def oracle(self):
        """The oracle's result for this request (FP64, with path digests)."""
        if self.kind == M.MCMF_REQ_ACTION:
            o = oracle.action(self.csr, oracle_fn(self.fn), self.v, N=self.N, K=self.K, scale=self.scale,
                              seed=self.seed, request=self.request, cutoff=self.cutoff, want_digest=True,
                              sampler=default_sampler(self.csr))
            return {"x": o["y"], "digest": o["digest"], "steps": o["steps"]}
        o = oracle.diag(self.csr, oracle_fn(self.fn), N=self.N, K=self.K, scale=self.scale, seed=self.seed,
                        request=self.request, cutoff=self.cutoff, rows=self.rows, want_digest=True,
                        sampler=default_sampler(self.csr))
        return {"x": o["d"], "digest": o["digest"], "steps": o["steps"]}

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


def run_batch(reqs, host=False, use_graph=False, stream=True, digest=True):
    made = [q.make(host, digest) for q in reqs]
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


def check_oracle(q, got, what=""):
    """A request's result against the oracle: paths (when a digest was taken)
    and step counts exact, FP64 estimates within 1e-10 relative (full value
    and Monte Carlo part), FP32-weight estimates within the stated bound
    2 K 2^-24 sum|terms| (sum|terms| is the Monte Carlo part on the
    non-negative inputs these requests use)."""
    o = q.oracle()
    if got.get("digest") is not None:
        assert np.array_equal(got["digest"], o["digest"]), f"{what}: walk paths differ"
    if "steps" in got:
        assert got["steps"] == o["steps"], what
    h = q.h()
    if q.precision == M.MCMF_PRECISION_FP32_WEIGHTS:
        mc = np.abs(o["x"] - h)
        bound = 2 * q.K * 2.0 ** -24 * mc + 4 * np.finfo(np.float64).eps * np.abs(o["x"]) + 1e-30
        assert np.all(np.abs(got["x"] - o["x"]) <= bound), what
        return
    assert_close(got["x"], o["x"], RTOL, atol=1e-13 * np.max(np.abs(o["x"]), initial=0.0), what=what)
    assert_mc_part_close(got["x"], o["x"], h, RTOL, what=what)


def make_graphs():
    csrs = {
        "rmat11": G.rmat(11, seed=7),
        "er": G.erdos_renyi_dense(700, 0.02, seed=8),
        "torus": G.torus2d(40, 40),
        "weighted": G.with_random_weights(G.rmat(10, seed=9), seed=10, negative_fraction=0.3),
        "ba": G.barabasi_albert(3000, 5, seed=11),
    }
    return {k: (graph(v), v) for k, v in csrs.items()}


def close_graphs(gs):
    for g, _ in gs.values():
        g.close()


def mixed_requests(graphs):
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
