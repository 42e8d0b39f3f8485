"""FP32 walk weights with FP64 accumulation: the paths are the FP64 paths
(bit-identical digests) and every output stays within the stated rounding
bound |x32 - x64| <= 2 K 2^-24 sum|terms| of the FP64 result (step t's
weight carries at most 2t roundings, a term at most four more).  On the
non-negative graphs used here every term is non-negative, so sum|terms| is
the Monte Carlo part x64 - h itself."""
import numpy as np
import pytest

import graphgen as G
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from _gpu import graph  # noqa: E402
from paper_2308_01037_amd import mcmf as M  # noqa: E402


def run(g, what, precision, n, N, K, scale, rows=None, seed=5):
    dig = torch.zeros(n, dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    opts = M.make_opts(seed=seed, precision=precision, stream=stream, path_digest=dig)
    f = M.make_fn(M.MCMF_FN_EXP, scale)
    if what == "action":
        out = torch.empty(n, dtype=torch.float64, device="cuda")
        M.mcmf_action(g.handle, f, torch.ones(n, dtype=torch.float64, device="cuda"), N, K, opts, out)
    else:
        count = n if rows is None else len(rows)
        out = torch.empty(count, dtype=torch.float64, device="cuda")
        rt = None if rows is None else torch.as_tensor(rows, dtype=torch.int32, device="cuda")
        M.mcmf_diag(g.handle, f, rt, 0 if rows is None else len(rows), N, K, opts, out)
    torch.cuda.synchronize()
    return out.cpu().numpy(), dig.cpu().numpy()


def check_bound(x32, x64, h, K, what):
    mc = x64 - h
    assert np.all(mc >= -1e-15 * np.abs(x64)), what
    bound = 2 * K * 2.0 ** -24 * np.abs(mc) + 4 * np.finfo(np.float64).eps * np.abs(x64) + 1e-30
    err = np.abs(x32 - x64)
    assert np.all(err <= bound), (what, float(np.max(err / np.maximum(bound, 1e-300))))
    return float(np.max(err[mc > 0] / mc[mc > 0])) if np.any(mc > 0) else 0.0


@pytest.mark.parametrize("maker", [lambda: G.erdos_renyi_dense(600, 0.02, seed=3),
                                   lambda: G.rmat(12, seed=4),
                                   lambda: G.barabasi_albert(5000, 8, seed=2)])
def test_fp32_weights_within_bound(maker):
    csr = maker()
    K, N = 40, 64
    s = 1.0 / csr.d_max
    c = oracle.coeffs(oracle.FN_EXP, K)
    with graph(csr) as g:
        ya, da = run(g, "action", M.MCMF_PRECISION_FP64, csr.n, N, K, s)
        yb, db = run(g, "action", M.MCMF_PRECISION_FP32_WEIGHTS, csr.n, N, K, s)
        xa, ea = run(g, "diag", M.MCMF_PRECISION_FP64, csr.n, N, K, s)
        xb, eb = run(g, "diag", M.MCMF_PRECISION_FP32_WEIGHTS, csr.n, N, K, s)
    assert np.array_equal(da, db) and np.array_equal(ea, eb), "FP32 mode changed the walks"
    rel_a = check_bound(yb, ya, c[0] + c[1] * s * csr.deg, K, "action")
    rel_d = check_bound(xb, xa, np.full(csr.n, c[0]), K, "diag")
    # The FP32 path is really taken: results differ from FP64 by rounding.
    assert not np.array_equal(ya, yb) and not np.array_equal(xa, xb)
    assert rel_a < 2 * K * 2.0 ** -24 and rel_d < 2 * K * 2.0 ** -24


def test_fp32_against_oracle_on_sampled_rows():
    # Barabasi-Albert graph, exp(A/d_max), full action and the diagonal on 1% of
    # the rows; the FP64 oracle recomputes 200 sampled outputs of each.
    csr = G.barabasi_albert(200_000, 8, seed=0)
    K, N = 40, 256
    s = 1.0 / csr.d_max
    rows = G.random_rows(csr.n, csr.n // 100, seed=0)
    with graph(csr) as g:
        y32, _ = run(g, "action", M.MCMF_PRECISION_FP32_WEIGHTS, csr.n, N, K, s, seed=1)
        d32, _ = run(g, "diag", M.MCMF_PRECISION_FP32_WEIGHTS, csr.n, N, K, s, rows=rows, seed=1)
    pick = np.random.default_rng(3).choice(len(rows), 200, replace=False)
    sample = np.sort(rows[pick]).astype(np.int32)
    oa = oracle.action(csr, oracle.FN_EXP, np.ones(csr.n), N=N, K=K, scale=s, seed=1, rows=sample)
    od = oracle.diag(csr, oracle.FN_EXP, N=N, K=K, scale=s, seed=1, rows=sample, assume_symmetric=True)
    c = oracle.coeffs(oracle.FN_EXP, K)
    check_bound(y32[sample], oa["y"], c[0] + c[1] * s * csr.deg[sample], K, "action vs oracle")
    pos = {int(r): i for i, r in enumerate(rows)}
    d_s = np.array([d32[pos[int(r)]] for r in sample])
    check_bound(d_s, od["d"], np.full(sample.size, c[0]), K, "diag vs oracle")


@pytest.mark.timeout(900)
def test_ba_four_million_full_size():
    # The Barabasi-Albert configuration at full size: n = 4,000,000, m = 8
    # (64M stored entries), exp(A/d_max), K = 40, N = 256; the full action and
    # the diagonal on 1% of the rows, FP32 walk weights against FP64.  The
    # FP32 paths equal the FP64 paths, every FP32 output is within the stated
    # bound of its FP64 output, and the FP64 oracle recomputes 1,000 sampled
    # rows of each (FP64 within 1e-10, FP32 within the bound).
    csr = G.barabasi_albert(4_000_000, 8, seed=0)
    K, N = 40, 256
    s = 1.0 / csr.d_max
    rows = G.random_rows(csr.n, csr.n // 100, seed=0)
    with graph(csr) as g:
        y64, da = run(g, "action", M.MCMF_PRECISION_FP64, csr.n, N, K, s, seed=1)
        y32, db = run(g, "action", M.MCMF_PRECISION_FP32_WEIGHTS, csr.n, N, K, s, seed=1)
        assert np.array_equal(da, db)
        d64, ea = run(g, "diag", M.MCMF_PRECISION_FP64, csr.n, N, K, s, rows=rows, seed=1)
        d32, eb = run(g, "diag", M.MCMF_PRECISION_FP32_WEIGHTS, csr.n, N, K, s, rows=rows, seed=1)
        assert np.array_equal(ea, eb)
    c = oracle.coeffs(oracle.FN_EXP, K)
    check_bound(y32, y64, c[0] + c[1] * s * csr.deg, K, "action FP32 vs FP64")
    check_bound(d32, d64, np.full(len(rows), c[0]), K, "diag FP32 vs FP64")
    pick = np.random.default_rng(3).choice(len(rows), 1000, replace=False)
    sample = np.sort(rows[pick]).astype(np.int32)
    oa = oracle.action(csr, oracle.FN_EXP, np.ones(csr.n), N=N, K=K, scale=s, seed=1, rows=sample,
                       want_digest=True)
    started = oa["digest"] != 0
    assert np.array_equal(da[started].view(np.uint64), oa["digest"][started])
    h = c[0] + c[1] * s * csr.deg[sample]
    mc = oa["y"] - h
    assert np.all(np.abs(y64[sample] - oa["y"]) <= 1e-10 * np.abs(mc) + 8 * np.finfo(float).eps * oa["y"])
    check_bound(y32[sample], oa["y"], h, K, "action FP32 vs oracle")
    od = oracle.diag(csr, oracle.FN_EXP, N=N, K=K, scale=s, seed=1, rows=sample, assume_symmetric=True)
    pos = {int(r): i for i, r in enumerate(rows)}
    at = np.array([pos[int(r)] for r in sample])
    mcd = od["d"] - c[0]
    assert np.all(np.abs(d64[at] - od["d"]) <= 1e-10 * np.abs(mcd) + 8 * np.finfo(float).eps * od["d"])
    check_bound(d32[at], od["d"], np.full(sample.size, c[0]), K, "diag FP32 vs oracle")
