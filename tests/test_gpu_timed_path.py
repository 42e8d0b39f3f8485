"""The kernels the benchmark times, against the oracle.

A path digest needs the row index of every visited state, so a call that
asks for one runs the edge-record walk kernels.  The benchmark asks for none:
its action walks over per-call value records and its diagonal walk is the
digest-free instantiation.  These tests run exactly those kernels (no digest)
and compare every output with the oracle:

* action, value records, N in {193, 256, 1000} (partial last wavefront, one
  full 256-lane workgroup, several walks per lane), FP64 within 1e-10 on the
  full value, on q and on the Monte Carlo part, FP32 walk weights within the
  stated bound 2 K 2^-24 sum|terms|;
* diagonal, digest-free walk in the EDGE, ROW and WIDE layouts (WIDE, with
  its hub sums, is what large graphs default to), the same N (N = 1000 also
  takes the gather through several table passes);
* the first draw of walk 0 from row 0 with seed 0 and request 0 is the
  published Philox4x32-10 known answer for counter 0 and key 0, read back
  through the walk it picks on a star (independent of the oracle).
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

from _gpu import assert_close, assert_mc_part_close, gpu_action, gpu_diag, graph  # noqa: E402
from paper_2308_01037_amd import mcmf as M  # noqa: E402

RTOL = 1e-10


@pytest.fixture(scope="module")
def rmat10():
    return G.rmat(10, seed=31)


def _bound_ok(x32, x64, h, K):
    mc = np.abs(x64 - h)
    bound = 2 * K * 2.0 ** -24 * mc + 4 * np.finfo(np.float64).eps * np.abs(x64) + 1e-30
    return np.all(np.abs(x32 - x64) <= bound)


@pytest.mark.parametrize("N", [193, 256, 1000])
def test_value_record_action_matches_oracle(rmat10, N):
    csr = rmat10
    K, s = 30, 1.0 / csr.d_max
    v = G.uniform_vector(csr.n, seed=2)
    o = oracle.action(csr, oracle.FN_EXP, v, N=N, K=K, scale=s, seed=7, request=3, want_q=True)
    with graph(csr) as g:
        t = M.mcmf_graph_get_tuning(g.handle)
        assert t.action_sampler == M.MCMF_SAMPLER_VALUE  # the default, as benchmarked
        r = gpu_action(g, "exp", v, N, K, s, seed=7, request=3, want_q=True, stats=True)
        vt = torch.as_tensor(v, device="cuda")
        y32 = torch.empty(csr.n, dtype=torch.float64, device="cuda")
        M.mcmf_action(g.handle, M.make_fn(M.MCMF_FN_EXP, s), vt, N, K,
                      M.make_opts(seed=7, request_id=3, precision=M.MCMF_PRECISION_FP32_WEIGHTS,
                                  stream=torch.cuda.current_stream().cuda_stream), y32)
        torch.cuda.synchronize()
        y32 = y32.cpu().numpy()
    assert r["stats"]["walk_steps"] == o["steps"]
    assert_close(r["q"], o["q"], RTOL, what="q")
    assert_close(r["y"], o["y"], RTOL, what="y")
    c = oracle.coeffs(oracle.FN_EXP, K)
    h = c[0] * v + c[1] * s * (csr.to_scipy() @ v)
    assert_mc_part_close(r["y"], o["y"], h, RTOL, what="y")
    assert _bound_ok(y32, o["y"], h, K), "FP32 weights outside the stated bound"
    assert not np.array_equal(y32, r["y"])  # the FP32 path really ran


@pytest.mark.parametrize("sampler", [M.MCMF_SAMPLER_EDGE, M.MCMF_SAMPLER_ROW, M.MCMF_SAMPLER_WIDE])
@pytest.mark.parametrize("N", [193, 256, 1000])
def test_digest_free_diag_matches_oracle(rmat10, N, sampler):
    csr = rmat10
    K, s = 30, 0.8 / csr.d_max
    o = oracle.diag(csr, oracle.FN_RESOLVENT, N=N, K=K, scale=s, seed=8)
    with graph(csr) as g:
        t = M.mcmf_graph_get_tuning(g.handle)
        t.diag_sampler, t.hub_count = sampler, 0
        M.mcmf_graph_set_tuning(g.handle, t)
        r = gpu_diag(g, "resolvent", N, K, s, seed=8, stats=True)
    assert r["stats"]["walk_steps"] == o["steps"]
    assert_close(r["d"], o["d"], RTOL, what="d")
    assert_mc_part_close(r["d"], o["d"], np.ones(csr.n), RTOL, what="d")


def test_first_draw_is_the_philox_known_answer():
    # Philox4x32-10 at counter (0, 0, 0, 0), key (0, 0) gives X0 = 0x6627e8d5,
    # X1 = 0xe169c58d (published known-answer vector).  Walk 0 from the hub of
    # a star with 2^20 leaves (seed 0, request 0) picks entry
    # floor(u 2^20 / 2^64) = u >> 44 of u = X1 2^32 + X0, i.e. leaf j + 1.
    kat = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "philox4x32_10_kat.txt")
    first = [line.split() for line in open(kat) if line.strip() and not line.startswith("#")][0]
    assert [int(x, 16) for x in first[:6]] == [0] * 6
    x0, x1 = int(first[6], 16), int(first[7], 16)
    u = (x1 << 32) | x0
    leaves = 1 << 20
    j = u >> 44
    csr = G.star(leaves)
    h = 0xCBF29CE484222325
    for state in (0, j + 1):
        h = ((h ^ state) * 0x100000001B3) % 2**64
    with graph(csr) as g:
        r = gpu_action(g, "exp", np.ones(csr.n), 1, 3, 1e-6, seed=0, request=0, want_digest=True)
    assert int(r["digest"][0]) == h
