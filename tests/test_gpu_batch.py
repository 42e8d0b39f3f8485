"""Batched execution (mcmf_batch) on the GPU.

A request run inside a batch draws the walks its own single call draws (same
keyed Philox counters), so per request: path digests and walk-step counts
equal the single call's exactly, and estimates agree within 1e-10 relative
(only the order of FP64 additions differs).  A few requests are also checked
against the oracle directly, and a batch recorded into a hipGraph must give
the eager batch's results on every launch.
"""
import numpy as np
import pytest

import graphgen as G

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from _gpu import fn_struct, graph  # noqa: E402
from _reqs import Req, check_oracle, check_same, close_graphs, make_graphs, run_batch  # noqa: E402
from _reqs import mixed_requests as _mixed  # noqa: E402
from paper_2308_01037_amd import mcmf as M  # noqa: E402


@pytest.fixture(scope="module")
def graphs():
    gs = make_graphs()
    yield gs
    close_graphs(gs)


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


@pytest.mark.parametrize("digest", [True, False])
def test_batch_against_oracle(graphs, digest):
    # With digests the batched walks read edge records; without, the action
    # requests on unweighted graphs walk over value records.
    g1, c1 = graphs["rmat11"]
    g4, c4 = graphs["weighted"]
    A, D = M.MCMF_REQ_ACTION, M.MCMF_REQ_DIAG
    reqs = [Req(g1, c1, D, "exp", 1.0 / c1.d_max, 40, 10, seed=9, request=2),
            Req(g4, c4, A, "resolvent", 0.1, 50, 9, seed=9, request=3),
            Req(g1, c1, A, "exp", 1.0 / c1.d_max, 40, 10, seed=9, request=4, cutoff=1e-4),
            Req(g1, c1, A, "exp", 1.0 / c1.d_max, 256, 40, seed=9, request=5),
            Req(g1, c1, A, "resolvent", 0.5 / c1.d_max, 193, 30, seed=9, request=6,
                v=np.random.default_rng(4).random(c1.n)),
            Req(g1, c1, A, "exp", 1.0 / c1.d_max, 256, 40, seed=9, request=7,
                precision=M.MCMF_PRECISION_FP32_WEIGHTS)]
    got, _ = run_batch(reqs, digest=digest)
    for i, (q, r) in enumerate(zip(reqs, got)):
        check_oracle(q, r, f"request {i}")


def test_small_visit_chunks(graphs, monkeypatch):
    # A visit budget of about three start rows splits the diag requests over
    # many walk/gather launches, across request boundaries.
    reqs = _mixed(graphs)[:7]
    want = [q.single() for q in reqs]
    monkeypatch.setenv("MCMF_DIAG_CHUNK_BYTES", str(3 * 200 * 14 * 12))
    got, _ = run_batch(reqs)
    for i, (q, g, w) in enumerate(zip(reqs, got, want)):
        check_same(q, g, w, f"request {i}")


@pytest.mark.parametrize("cap", [0, 5])
def test_item_map_fallback(graphs, monkeypatch, cap):
    # Gather items beyond the launch's item map find their run and start row
    # by binary search: with the map capped at 0 or 5 entries nearly every
    # item does, and every request still equals its single call.
    reqs = _mixed(graphs)[:8]
    want = [q.single() for q in reqs]
    monkeypatch.setenv("MCMF_TEST_ITEM_MAP_CAP", str(cap))
    got, _ = run_batch(reqs)
    for i, (q, g, w) in enumerate(zip(reqs, got, want)):
        check_same(q, g, w, f"item map capped at {cap}, request {i}")


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


def test_failed_capture_runs_the_launches_directly(graphs, monkeypatch):
    # A capture that fails (as when another host thread invalidates it) falls
    # back to launching the batch directly: same results as eager.
    reqs = _mixed(graphs)[:6]
    eager, _ = run_batch(reqs)
    monkeypatch.setenv("MCMF_TEST_FAIL_CAPTURE", "1")
    got, _ = run_batch(reqs, use_graph=True)
    monkeypatch.delenv("MCMF_TEST_FAIL_CAPTURE")
    for i, (q, g, w) in enumerate(zip(reqs, got, eager)):
        check_same(q, g, w, f"after a failed capture, request {i}")
    got, _ = run_batch(reqs, use_graph=True)  # and the next capture works
    for i, (q, g, w) in enumerate(zip(reqs, got, eager)):
        check_same(q, g, w, f"capture after the failed one, request {i}")


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
