"""Walk-kernel tuning: every sampler layout and load policy gives the same
walks (paths bit-exact against the oracle, estimates within 1e-10), and the
autotuner (mcmf_tune) with its JSON cache picks and reapplies a choice."""
import numpy as np
import pytest

import graphgen as G
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from _gpu import assert_close, gpu_action, gpu_diag, graph, oracle_fn  # noqa: E402
from paper_2308_01037_amd import mcmf as M  # noqa: E402
from paper_2308_01037_amd import tuning  # noqa: E402


def set_tuning(g, sampler, stream):
    t = M.mcmf_tuning()
    t.action_sampler = t.diag_sampler = sampler
    t.action_stream = t.diag_stream = stream
    M.mcmf_graph_set_tuning(g.handle, t)


@pytest.mark.parametrize("maker", [lambda: G.rmat(11, seed=2), lambda: G.grid2d(30, 30)])
@pytest.mark.parametrize("sampler", [M.MCMF_SAMPLER_EDGE, M.MCMF_SAMPLER_ROW])
@pytest.mark.parametrize("stream", [0, 1])
def test_every_variant_matches_oracle(maker, sampler, stream):
    csr = maker()
    K, N, s = 15, 48, 1.0 / csr.d_max
    with graph(csr) as g:
        set_tuning(g, sampler, stream)
        t = M.mcmf_graph_get_tuning(g.handle)
        assert (t.action_sampler, t.action_stream) == (sampler, stream)
        o = oracle.diag(csr, oracle_fn("exp"), N=N, K=K, scale=s, seed=3, want_digest=True)
        r = gpu_diag(g, "exp", N, K, s, seed=3, want_digest=True)
        assert np.array_equal(r["digest"], o["digest"])
        assert_close(r["d"], o["d"], 1e-10)
        v = np.random.default_rng(1).random(csr.n)
        o = oracle.action(csr, oracle_fn("resolvent"), v, N=N, K=K, scale=s, seed=3, want_digest=True)
        r = gpu_action(g, "resolvent", v, N, K, s, seed=3, want_digest=True)
        assert np.array_equal(r["digest"], o["digest"])
        assert_close(r["y"], o["y"], 1e-10)


def test_tuning_argument_errors():
    with graph(G.path(5)) as g:
        t = M.mcmf_tuning()
        t.action_sampler = 2
        with pytest.raises(M.MCMFError):
            M.mcmf_graph_set_tuning(g.handle, t)
        t = M.mcmf_tuning()
        t.diag_stream = 3
        with pytest.raises(M.MCMFError):
            M.mcmf_graph_set_tuning(g.handle, t)
        t = M.mcmf_tuning()
        t.reserved[1] = 1
        with pytest.raises(M.MCMFError):
            M.mcmf_graph_set_tuning(g.handle, t)
        with pytest.raises(M.MCMFError):
            M.mcmf_tune(g.handle, M.make_fn(M.MCMF_FN_EXP, 0.5), 16, 1)


def test_autotune_measures_then_caches(tmp_path):
    csr = G.rmat(13, seed=5)
    path = str(tmp_path / "tune.json")
    f = M.make_fn(M.MCMF_FN_EXP, 1.0 / csr.d_max)
    with graph(csr) as g:
        a = tuning.autotune(g, csr, f, 64, 20, path)
        assert not a["cached"] and a["sample_rows"] > 0
        assert all(ms > 0 for ms in a["action_ms"]) and all(ms > 0 for ms in a["diag_ms"])
        best_a = int(np.argmin(a["action_ms"]))
        assert (a["action_sampler"], a["action_stream"]) == (best_a >> 1, best_a & 1)
        t = M.mcmf_graph_get_tuning(g.handle)
        assert (t.diag_sampler, t.diag_stream) == (a["diag_sampler"], a["diag_stream"])
    with graph(csr) as g2:
        b = tuning.autotune(g2, csr, f, 64, 20, path)
        assert b["cached"]
        t = M.mcmf_graph_get_tuning(g2.handle)
        assert (t.action_sampler, t.action_stream, t.diag_sampler, t.diag_stream) == \
            (a["action_sampler"], a["action_stream"], a["diag_sampler"], a["diag_stream"])
        # Tuned and default walks agree exactly.
        x = gpu_diag(g2, "exp", 32, 12, 1.0 / csr.d_max, seed=9, want_digest=True)
        set_tuning(g2, M.MCMF_SAMPLER_EDGE, 0)
        y = gpu_diag(g2, "exp", 32, 12, 1.0 / csr.d_max, seed=9, want_digest=True)
        assert np.array_equal(x["digest"], y["digest"])
        assert_close(x["d"], y["d"], 1e-12)
