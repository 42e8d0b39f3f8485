"""The request server (mcmf_server_*) on the GPU: continuous batching over
several streams with admission by a device-memory budget.

Every request's result in the mix equals its own single call's (path digests
and step counts exact, estimates within 1e-10 relative), whatever batch it
lands in; the admission estimate in flight never exceeds the budget unless a
request runs alone; destroying the server runs what is still queued.
"""
import threading

import numpy as np
import pytest

import graphgen as G

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from _gpu import fn_struct, graph  # noqa: E402
from _reqs import Req, check_oracle, check_same, close_graphs, make_graphs, mixed_requests  # noqa: E402
from paper_2308_01037_amd import mcmf as M  # noqa: E402


@pytest.fixture(scope="module")
def graphs():
    gs = make_graphs()
    yield gs
    close_graphs(gs)


def server(**kw):
    o = M.mcmf_server_opts()
    for k, v in kw.items():
        setattr(o, k, v)
    return M.mcmf_server_create(o)


def serve(srv, reqs, threads=1, host=False, digest=True):
    """Submits reqs (from `threads` host threads), waits for all; returns the
    results in request order and the ticket infos."""
    made = [q.make(host, digest) for q in reqs]
    tickets = [None] * len(reqs)

    def submit(idx):
        for i in idx:
            tickets[i] = M.mcmf_server_submit(srv, made[i][0])

    parts = [list(range(t, len(reqs), threads)) for t in range(threads)]
    ths = [threading.Thread(target=submit, args=(p,)) for p in parts]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    infos = [M.mcmf_server_wait(srv, t) for t in tickets]
    torch.cuda.synchronize()
    res = []
    for q, (r, out, dig) in zip(reqs, made):
        assert r.status == M.MCMF_OK
        d = Req.fetch(out, dig, q.count)
        d["steps"] = r.walk_steps
        res.append(d)
    return res, infos


def test_served_mix_equals_single_calls(graphs):
    reqs = mixed_requests(graphs) * 3
    want = [q.single() for q in reqs]
    srv = server(n_streams=3, max_batch=5)
    try:
        got, infos = serve(srv, reqs, threads=4)
        st = M.mcmf_server_query(srv)
    finally:
        M.mcmf_server_destroy(srv)
    for i, (q, g, w) in enumerate(zip(reqs, got, want)):
        check_same(q, g, w, f"request {i}")
    assert st["submitted"] == st["completed"] == len(reqs)
    assert st["largest_batch"] <= 5
    assert all(1 <= inf.batch_size <= 5 and inf.queue_ms >= 0 and inf.run_ms > 0 for inf in infos)


@pytest.mark.parametrize("digest", [True, False])
def test_served_requests_against_oracle(graphs, digest):
    # Served diagonal (full and row subset) and action requests, in batches
    # of up to three over two streams, against the oracle directly.  Without
    # digests the actions walk over value records.
    g1, c1 = graphs["rmat11"]
    g2, c2 = graphs["er"]
    A, D = M.MCMF_REQ_ACTION, M.MCMF_REQ_DIAG
    rng = np.random.default_rng(8)
    reqs = [Req(g1, c1, D, "exp", 1.0 / c1.d_max, 64, 20, seed=11, request=1),
            Req(g1, c1, A, "exp", 1.0 / c1.d_max, 256, 40, seed=11, request=2),
            Req(g2, c2, D, "resolvent", 0.05, 100, 15, seed=11, request=3,
                rows=rng.choice(c2.n, 60, replace=False)),
            Req(g2, c2, A, "resolvent", 0.05, 193, 15, seed=11, request=4, v=rng.random(c2.n)),
            Req(g1, c1, D, "resolvent", 0.5 / c1.d_max, 32, 12, seed=11, request=5,
                rows=np.arange(0, c1.n, 5), precision=M.MCMF_PRECISION_FP32_WEIGHTS)]
    srv = server(n_streams=2, max_batch=3)
    try:
        got, infos = serve(srv, reqs, threads=2, digest=digest)
    finally:
        M.mcmf_server_destroy(srv)
    for i, (q, r) in enumerate(zip(reqs, got)):
        check_oracle(q, r, f"served request {i}")


def test_host_buffers_and_hipgraph_batches(graphs):
    reqs = mixed_requests(graphs)[:8]
    want = [q.single() for q in reqs]
    srv = server(n_streams=2, max_batch=3, use_graph=1)
    try:
        got, _ = serve(srv, reqs, threads=2, host=True)
    finally:
        M.mcmf_server_destroy(srv)
    for i, (q, g, w) in enumerate(zip(reqs, got, want)):
        check_same(q, g, w, f"request {i}")


def test_budget_admission(graphs):
    # A budget that holds about two of these requests: the estimate in flight
    # stays within it, and every request still completes.
    g1, c1 = graphs["rmat11"]
    reqs = [Req(g1, c1, M.MCMF_REQ_DIAG, "exp", 1.0 / c1.d_max, 32, 10, seed=3, request=i,
                rows=np.arange(i, c1.n, 17)) for i in range(12)]
    want = [q.single() for q in reqs]
    probe = reqs[0].make()[0]
    srv0 = server(n_streams=1)
    try:
        t = M.mcmf_server_submit(srv0, probe)
        one = M.mcmf_server_wait(srv0, t).est_bytes
    finally:
        M.mcmf_server_destroy(srv0)
    budget = int(2.5 * one)
    srv = server(n_streams=4, max_batch=8, hbm_budget_bytes=budget, visit_chunk_bytes=1 << 20)
    try:
        got, infos = serve(srv, reqs, threads=3)
        st = M.mcmf_server_query(srv)
    finally:
        M.mcmf_server_destroy(srv)
    for i, (q, g, w) in enumerate(zip(reqs, got, want)):
        check_same(q, g, w, f"request {i}")
    assert st["peak_bytes_in_flight"] <= budget
    assert st["completed"] == len(reqs)


def test_request_larger_than_budget_runs_alone(graphs):
    g1, c1 = graphs["rmat11"]
    reqs = [Req(g1, c1, M.MCMF_REQ_ACTION, "exp", 1.0 / c1.d_max, 16, 8, seed=4, request=i)
            for i in range(4)]
    want = [q.single() for q in reqs]
    srv = server(n_streams=3, hbm_budget_bytes=1024)
    try:
        got, infos = serve(srv, reqs, threads=2)
        st = M.mcmf_server_query(srv)
    finally:
        M.mcmf_server_destroy(srv)
    for i, (q, g, w) in enumerate(zip(reqs, got, want)):
        check_same(q, g, w, f"request {i}")
    assert st["peak_batches_in_flight"] == 1
    assert all(inf.batch_size == 1 for inf in infos)


def test_invalid_request_is_refused_and_destroy_drains(graphs):
    g1, c1 = graphs["rmat11"]
    csr = G.rmat(8, seed=1)
    with graph(csr, flags=0) as gn:
        bad = Req(gn, csr, M.MCMF_REQ_DIAG, "exp", 0.1, 8, 5).make()[0]
        srv = server(n_streams=2)
        try:
            with pytest.raises(M.MCMFError) as e:
                M.mcmf_server_submit(srv, bad)
            assert e.value.status == M.MCMF_E_NOT_SYMMETRIC
            with pytest.raises(M.MCMFError):
                M.mcmf_server_wait(srv, 12345)
            ok = Req(g1, c1, M.MCMF_REQ_ACTION, "resolvent", 0.05, 16, 6, seed=5)
            made = [ok.make() for _ in range(6)]
            for r, _, _ in made:
                M.mcmf_server_submit(srv, r)
        finally:
            M.mcmf_server_destroy(srv)  # runs the queued requests first
        torch.cuda.synchronize()
        want = ok.single()
        for r, out, dig in made:
            assert r.status == M.MCMF_OK
            got = Req.fetch(out, dig, ok.count)
            got["steps"] = r.walk_steps
            check_same(ok, got, want, "drained request")


def test_batches_stay_small_and_step_bounds_hold(graphs):
    # With a walk-step limit of one step per batch every request runs alone;
    # for actions and full diagonals the step estimate is an upper bound of
    # the steps actually recorded.
    reqs = mixed_requests(graphs)[:7]
    want = [q.single() for q in reqs]
    srv = server(n_streams=2, max_batch=8, max_batch_steps=1)
    try:
        made = [q.make() for q in reqs]
        tickets = [M.mcmf_server_submit(srv, m[0]) for m in made]
        infos = [M.mcmf_server_wait(srv, t) for t in tickets]
    finally:
        M.mcmf_server_destroy(srv)
    torch.cuda.synchronize()
    for i, (q, (r, out, dig), inf, w) in enumerate(zip(reqs, made, infos, want)):
        got = Req.fetch(out, dig, q.count)
        got["steps"] = r.walk_steps
        check_same(q, got, w, f"request {i}")
        if q.kind == M.MCMF_REQ_ACTION or q.rows is None:
            assert inf.est_steps >= r.walk_steps, (i, inf.est_steps, r.walk_steps)
        if inf.est_steps > 1:
            assert inf.batch_size == 1


@pytest.mark.parametrize("limit", [1, 2])
def test_large_requests_in_flight_are_limited(graphs, limit):
    # With a one-step batch limit every request that walks is large and runs
    # alone; at most `limit` of them run at once on the three streams, the
    # small ones (K <= 1: no walk steps) pass the waiting large ones, and
    # every result equals its single call.
    reqs = mixed_requests(graphs)
    want = [q.single() for q in reqs]
    srv = server(n_streams=3, max_batch=4, max_batch_steps=1, max_large_in_flight=limit)
    try:
        got, infos = serve(srv, reqs * 2, threads=3)
        st = M.mcmf_server_query(srv)
    finally:
        M.mcmf_server_destroy(srv)
    for i, (q, g, w) in enumerate(zip(reqs * 2, got, want * 2)):
        check_same(q, g, w, f"request {i}")
    assert 1 <= st["peak_large_in_flight"] <= limit
    assert st["completed"] == 2 * len(reqs)
