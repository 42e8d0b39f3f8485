"""Pins for the oracle's estimators against what mathematics fixes.

None of these compares the oracle with itself.  They use:

* zero-variance cases, where every walk gives the exact truncated series:
  K <= 2 on any graph; the diagonal on complete bipartite graphs; the action
  on 1 for regular graphs; the odd-power terms on triangle-free graphs;
* the exact-expectation mode (distribution propagation) against the dense
  truncated series sum_k c_k (sA)^k evaluated by Horner's rule;
* closed forms of the full functions (K_n, regular graphs, paths, cycles);
* statistics: unbiasedness z-tests, the N^-1/2 error rate (Section 4.1);
* structural identities: linearity in v, subset consistency, the weight
  cutoff on regular graphs.
"""
import math

import numpy as np
import pytest

import graphgen as G


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


def _graphs_small():
    return [
        G.erdos_renyi_dense(40, 0.15, seed=1),
        G.rmat(6, seed=2),
        G.with_random_weights(G.erdos_renyi_dense(30, 0.2, seed=3), seed=4, negative_fraction=0.3),
        G.path(9),
        G.star(7),
    ]


# ------------------------------------------------------------ dense checker


def test_dense_series_matches_expm_and_inverse(orc):
    from scipy.linalg import expm
    g = G.erdos_renyi_dense(50, 0.1, seed=7)
    a = g.dense()
    s = 0.3
    K = 40
    f = orc.dense_series(a, orc.coeffs(orc.FN_EXP, K), s)
    norm = np.linalg.norm(s * a, 2)
    tail = sum(norm ** k / math.factorial(k) for k in range(K + 1, K + 60))
    assert np.max(np.abs(f - expm(s * a))) <= tail + 1e-12 * np.max(np.abs(f))
    lam = np.max(np.abs(np.linalg.eigvalsh(a)))
    gamma = 0.5 / lam
    fr = orc.dense_series(a, orc.coeffs(orc.FN_RESOLVENT, 200), gamma)
    inv = np.linalg.inv(np.eye(g.n) - gamma * a)
    assert np.max(np.abs(fr - inv)) <= 2 * 0.5 ** 201 / 0.5 + 1e-12


def test_coefficients(orc):
    c = orc.coeffs(orc.FN_EXP, 20)
    assert np.allclose(c, [1 / math.factorial(k) for k in range(21)], rtol=1e-15, atol=0)
    assert np.all(orc.coeffs(orc.FN_RESOLVENT, 7) == 1.0)


# ------------------------------------------------------------ exact cases


@pytest.mark.parametrize("K", [0, 1, 2])
def test_K_at_most_two_is_exact(orc, K):
    # Only H = c0 I + c1 B and the first walk state (W_0 = 1 at the start row) enter.
    for g in _graphs_small():
        c = orc.coeffs(orc.FN_EXP, K)
        s = 0.37
        dense = orc.dense_series(g.dense(), c, s)
        v = G.uniform_vector(g.n, seed=1)
        for N, seed in ((1, 0), (7, 99)):
            y = orc.action(g, c, v, N=N, K=K, scale=s, seed=seed)["y"]
            assert _rel(y, dense @ v) < 1e-13
            d = orc.diag(g, c, N=N, K=K, scale=s, seed=seed)["d"]
            assert _rel(d, np.diag(dense)) < 1e-13
            rows = np.array([g.n - 1, 0, 2, 2], dtype=np.int32)
            d = orc.diag(g, c, N=N, K=K, scale=s, seed=seed, rows=rows)["d"]
            assert _rel(d, np.diag(dense)[rows]) < 1e-13
            y = orc.action(g, c, v, N=N, K=K, scale=s, seed=seed, rows=rows)["y"]
            assert _rel(y, (dense @ v)[rows]) < 1e-13


@pytest.mark.parametrize("p,q", [(1, 9), (3, 5), (4, 4), (2, 40)])
def test_complete_bipartite_diag_closed_form(orc, p, q):
    # Closed walks of length 2m from a node of degree q in K_{p,q}: q (pq)^(m-1).
    g = G.complete_bipartite(p, q)
    K = 9
    s = 0.21
    for fn in (orc.FN_EXP, orc.FN_RESOLVENT):
        c = orc.coeffs(fn, K)

        def closed(own_deg, other_deg):
            return c[0] + sum(c[2 * m] * s ** (2 * m) * own_deg * (own_deg * other_deg) ** (m - 1)
                              for m in range(1, K // 2 + 1))
        want = np.array([closed(q, p)] * p + [closed(p, q)] * q)
        d = orc.diag(g, c, N=3, K=K, scale=s, seed=5, request=2)["d"]
        assert _rel(d, want) < 1e-13


@pytest.mark.parametrize("maker", [lambda: G.cycle(11), lambda: G.circulant(30, 3),
                                   lambda: G.torus2d(6, 7), lambda: G.hypercube(5),
                                   lambda: G.complete(9)])
def test_regular_graph_action_on_ones(orc, maker):
    # d-regular: A 1 = d 1, so f(sA) 1 = sum_k c_k (s d)^k 1 on every walk.
    g = maker()
    d = int(g.deg[0])
    assert np.all(g.deg == d)
    K = 25
    s = 0.4 / d
    for fn in (orc.FN_EXP, orc.FN_RESOLVENT):
        c = orc.coeffs(fn, K)
        want = sum(c[k] * (s * d) ** k for k in range(K + 1))
        y = orc.action(g, c, np.ones(g.n), N=2, K=K, scale=s, seed=3)["y"]
        assert _rel(y, np.full(g.n, want)) < 1e-13


@pytest.mark.parametrize("maker", [lambda: G.hypercube(4), lambda: G.grid2d(4, 5),
                                   lambda: G.cycle(10),
                                   lambda: G.from_edges(24, np.random.default_rng(1).integers(0, 12, 40),
                                                        np.random.default_rng(2).integers(12, 24, 40))])
def test_triangle_free_third_power_vanishes(orc, maker):
    # With K = 3 the estimate is c0 + c2 s^2 deg(i) + c3 s^3 (A^3)_ii and
    # (A^3)_ii counts triangles: zero on triangle-free graphs, on every walk.
    g = maker()
    a = g.dense()
    tri = np.diag(a @ a @ a)
    if np.any(tri):
        pytest.skip("graph has triangles")
    c = orc.coeffs(orc.FN_EXP, 3)
    s = 0.5
    d = orc.diag(g, c, N=5, K=3, scale=s, seed=8)["d"]
    assert _rel(d, c[0] + c[2] * s * s * g.deg) < 1e-14


# ------------------------------------------------------------ expectation mode


@pytest.mark.parametrize("K", [3, 6, 12])
def test_expectation_mode_equals_dense_series(orc, K):
    rng = np.random.default_rng(K)
    for g in _graphs_small():
        s = 0.8 / max(g.d_max, 1)
        for fn in (orc.FN_EXP, orc.FN_RESOLVENT, rng.random(K + 1)):
            c = orc.coeffs(fn, K) if isinstance(fn, int) else fn
            dense = orc.dense_series(g.dense(), c, s)
            v = rng.random(g.n) - 0.3
            y = orc.action(g, c, v, N=1, K=K, scale=s, expect=True)["y"]
            assert _rel(y, dense @ v) < 1e-12
            d = orc.diag(g, c, N=1, K=K, scale=s, expect=True)["d"]
            assert _rel(d, np.diag(dense)) < 1e-12


def test_expectation_mode_nonsymmetric_action(orc):
    # The action needs no symmetry; rows without entries end the walk.
    rng = np.random.default_rng(4)
    src = rng.integers(0, 20, 60)  # rows 20..24 have no entries
    dst = rng.integers(0, 25, 60)
    g = G.from_edges(25, src, dst, symmetric=False)
    assert np.any(g.deg == 0)
    c = orc.coeffs(orc.FN_EXP, 8)
    v = rng.random(25)
    y = orc.action(g, c, v, N=1, K=8, scale=0.7, expect=True)["y"]
    assert _rel(y, orc.dense_series(g.dense(), c, 0.7) @ v) < 1e-12
    with pytest.raises(orc.OracleError):
        orc.diag(g, c, N=4, K=8, scale=0.7)


# ------------------------------------------------------------ full-function closed forms


def test_complete_graph_exp_diag_closed_form(orc):
    # exp(A)_ii on K_n = (e^(n-1) + (n-1) e^(-1)) / n.
    for n in (4, 7):
        g = G.complete(n)
        d = orc.diag(g, orc.FN_EXP, N=1, K=60, expect=True)["d"]
        want = (math.exp(n - 1) + (n - 1) * math.exp(-1)) / n
        assert _rel(d, np.full(n, want)) < 1e-13


def test_regular_graph_exp_action_closed_form(orc):
    # exp(A) 1 = e^d 1 for a d-regular graph (sampled walks, zero variance).
    g = G.torus2d(5, 6)
    y = orc.action(g, orc.FN_EXP, np.ones(g.n), N=3, K=50, seed=1)["y"]
    assert _rel(y, np.full(g.n, math.exp(4))) < 1e-13


@pytest.mark.parametrize("kind", ["path", "cycle"])
def test_path_and_cycle_spectral_closed_forms(orc, kind):
    # Path P_n: f_ii = 2/(n+1) sum_j sin^2(pi i j/(n+1)) f(2 cos(pi j/(n+1)))
    # Cycle C_n: f_ii = 1/n sum_j f(2 cos(2 pi j/n)); exp(A) and (I - gamma A)^-1.
    n = 8
    g = G.path(n) if kind == "path" else G.cycle(n)
    gamma = 0.3
    K = 120
    for fn, f in ((orc.FN_EXP, math.exp), (orc.FN_RESOLVENT, lambda x: 1.0 / (1.0 - gamma * x))):
        s = 1.0 if fn == orc.FN_EXP else gamma
        d = orc.diag(g, fn, N=1, K=K, scale=s, expect=True)["d"]
        if kind == "path":
            want = [2 / (n + 1) * sum(math.sin(math.pi * i * j / (n + 1)) ** 2 *
                                      f(2 * math.cos(math.pi * j / (n + 1))) for j in range(1, n + 1))
                    for i in range(1, n + 1)]
        else:
            want = [sum(f(2 * math.cos(2 * math.pi * j / n)) for j in range(n)) / n] * n
        assert _rel(d, want) < 1e-12


# ------------------------------------------------------------ statistics


def _z_test(estimates, exact, tol=5.0):
    est = np.asarray(estimates)
    mean = est.mean(axis=0)
    se = est.std(axis=0, ddof=1) / np.sqrt(est.shape[0])
    mask = se > 1e-14 * np.abs(exact).max()
    z = np.abs(mean - exact)[mask] / se[mask]
    assert np.all(np.abs(mean - exact)[~mask] < 1e-12 * np.abs(exact).max())
    return z.max() if z.size else 0.0


@pytest.mark.parametrize("which,sampler", [("er", "cdf"), ("rmat", "cdf"), ("weighted", "cdf"),
                                           ("weighted", "alias"), ("path", "cdf")])
def test_unbiased(orc, which, sampler):
    g = {"er": lambda: G.erdos_renyi_dense(30, 0.2, seed=11),
         "rmat": lambda: G.rmat(6, seed=3),
         "weighted": lambda: G.with_random_weights(G.erdos_renyi_dense(25, 0.25, seed=5), seed=6,
                                                   negative_fraction=0.3),
         "path": lambda: G.path(20)}[which]()
    K = 6
    s = 0.9 / max(g.d_max, 1)
    c = orc.coeffs(orc.FN_EXP, K)
    dense = orc.dense_series(g.dense(), c, s)
    v = G.uniform_vector(g.n, seed=2)
    R = 40
    ys = [orc.action(g, c, v, N=16, K=K, scale=s, seed=77, request=r, sampler=sampler)["y"] for r in range(R)]
    ds = [orc.diag(g, c, N=16, K=K, scale=s, seed=77, request=r, sampler=sampler)["d"] for r in range(R)]
    # 5 sigma over ~100 entries: a wrong term or sign fails by many sigma.
    assert _z_test(ys, dense @ v) < 5.0
    assert _z_test(ds, np.diag(dense)) < 5.0


@pytest.mark.slow
def test_error_decays_as_inverse_sqrt_N(orc):
    # Section 4.1: the error falls like N^-1/2 (fitted log-log slope about -0.5).
    g = G.erdos_renyi_dense(120, 0.06, seed=13)
    K = 8
    s = 0.5
    c = orc.coeffs(orc.FN_EXP, K)
    dense = orc.dense_series(g.dense(), c, s)
    exact_y = dense @ np.ones(g.n)
    exact_d = np.diag(dense)
    Ns = [16, 32, 64, 128, 256, 512, 1024, 2048]
    ey, ed = [], []
    for N in Ns:
        ey.append(np.mean([_rel(orc.action(g, c, np.ones(g.n), N=N, K=K, scale=s, seed=5,
                                           request=r)["y"], exact_y) for r in range(6)]))
        ed.append(np.mean([_rel(orc.diag(g, c, N=N, K=K, scale=s, seed=5, request=r)["d"],
                                exact_d) for r in range(6)]))
    for err in (ey, ed):
        slope = np.polyfit(np.log(Ns), np.log(err), 1)[0]
        assert -0.6 < slope < -0.4, slope


# ------------------------------------------------------------ identities


def test_action_is_linear_in_v(orc):
    g = G.rmat(7, seed=4)
    rng = np.random.default_rng(0)
    v1, v2 = rng.random(g.n), rng.random(g.n) - 0.5
    kw = dict(N=9, K=10, scale=0.05, seed=31, request=4)
    y1 = orc.action(g, orc.FN_EXP, v1, **kw)["y"]
    y2 = orc.action(g, orc.FN_EXP, v2, **kw)["y"]
    y12 = orc.action(g, orc.FN_EXP, 2.5 * v1 - 1.5 * v2, **kw)["y"]
    assert _rel(y12, 2.5 * y1 - 1.5 * y2) < 1e-13


def test_subsets_reproduce_the_full_run(orc):
    # Keyed walks: a row's estimate does not depend on which other rows are requested.
    g = G.rmat(7, seed=6)
    kw = dict(N=11, K=12, scale=0.03, seed=8, request=1)
    full = orc.diag(g, orc.FN_EXP, want_digest=True, **kw)
    rows = np.array([5, 17, 17, 3, 100, 64, 5], dtype=np.int32)
    sub = orc.diag(g, orc.FN_EXP, rows=rows, want_digest=True, **kw)
    assert np.array_equal(sub["d"], full["d"][rows])
    started = sub["digest"] != 0
    assert np.array_equal(sub["digest"][started], full["digest"][started])
    v = G.uniform_vector(g.n, seed=3)
    fa = orc.action(g, orc.FN_RESOLVENT, v, **kw)["y"]
    sa = orc.action(g, orc.FN_RESOLVENT, v, rows=rows, **kw)["y"]
    assert np.array_equal(sa, fa[rows])
    assert orc.diag(g, orc.FN_EXP, rows=np.zeros(0, np.int32), **kw)["d"].size == 0


def test_walk_count_and_digest_bookkeeping(orc):
    g = G.rmat(6, seed=1)
    active = int(np.count_nonzero(g.deg))
    r = orc.action(g, orc.FN_EXP, np.ones(g.n), N=7, K=9, scale=0.1, seed=2, want_digest=True,
                   want_q=True)
    assert r["steps"] == active * 7 * 8
    assert np.all((r["digest"] != 0) == (g.deg > 0))
    assert np.all(r["q"][g.deg == 0] == 0)
    r2 = orc.action(g, orc.FN_EXP, np.ones(g.n), N=7, K=9, scale=0.1, seed=2, request=1,
                    want_digest=True)
    assert np.count_nonzero(r2["digest"] == r["digest"]) == np.count_nonzero(g.deg == 0)


def test_isolated_rows(orc):
    g = G.from_edges(6, [0, 1], [1, 2])  # nodes 3, 4, 5 isolated
    c = orc.coeffs(orc.FN_EXP, 7)
    v = np.arange(6, dtype=float)
    y = orc.action(g, c, v, N=4, K=7, scale=0.5, seed=1)["y"]
    assert np.array_equal(y[3:], c[0] * v[3:])
    d = orc.diag(g, c, N=4, K=7, scale=0.5, seed=1)["d"]
    assert np.all(d[3:] == c[0])


def test_weight_cutoff_on_regular_graph(orc):
    # W_t = (s d)^t on a d-regular graph: with cutoff Wc the walk records the
    # steps with (s d)^t > Wc (Eq. weight_cutoff), so the action on 1 is the
    # series truncated there.
    g = G.circulant(20, 2)
    s = 0.1  # s d = 0.4
    K = 30
    c = orc.coeffs(orc.FN_EXP, K)
    for wc in (1e-3, 1e-6, 1e-300):
        last = max(t for t in range(K - 1) if 0.4 ** t > wc)
        want = c[0] + c[1] * 0.4 + sum(c[t + 2] * 0.4 ** (t + 2) for t in range(last + 1))
        y = orc.action(g, c, np.ones(g.n), N=3, K=K, scale=s, seed=4, cutoff=wc)["y"]
        assert _rel(y, np.full(g.n, want)) < 1e-14
    base = orc.action(g, c, np.ones(g.n), N=3, K=K, scale=s, seed=4)["y"]
    tiny = orc.action(g, c, np.ones(g.n), N=3, K=K, scale=s, seed=4, cutoff=1e-300)["y"]
    assert np.array_equal(base, tiny)


def test_argument_errors(orc):
    g = G.path(5)
    with pytest.raises(orc.OracleError):
        orc.action(g, orc.FN_EXP, np.ones(5), N=0, K=5)
    with pytest.raises(orc.OracleError):
        orc.diag(g, orc.FN_EXP, N=2, K=5, rows=np.array([7], np.int32))
    with pytest.raises(orc.OracleError):
        orc.action(g, [1.0, 1.0], np.ones(5), N=2, K=5)


# ------------------------------------------------------------------ walk allocation


def _allocation_by_formula(A, starts, Ns, min_one=False):
    """N_k = round-half-up(Ns ||C_k|| / sum over starts of ||C||), with column
    norms from the dense matrix (Eq. initial_prob; Algorithms 2-3 use
    N_i = N_s P(l0 = i), which may round to 0); max(1, .) with min_one."""
    import math
    norms = np.sqrt((np.asarray(A) ** 2).sum(axis=0))
    total = 0.0
    for k in starts:
        total += norms[k]
    out = np.zeros(A.shape[0], dtype=np.int64)
    for k in starts:
        w = int(math.floor(Ns * (norms[k] / total) + 0.5))
        out[k] = max(1, w) if min_one else w
    return out


@pytest.mark.parametrize("min_one", [False, True])
@pytest.mark.parametrize("which", ["weighted", "rmat", "directed"])
def test_allocation_follows_column_norms(orc, which, min_one):
    if which == "weighted":
        g = G.with_random_weights(G.erdos_renyi_dense(60, 0.1, seed=4), seed=5, negative_fraction=0.4)
        sym = True
    elif which == "rmat":
        g = G.rmat(8, seed=6)
        sym = True
    else:
        rng = np.random.default_rng(9)
        src, dst = rng.integers(0, 80, 400), rng.integers(0, 80, 400)
        keep = src != dst
        g = G.from_edges(80, src[keep], dst[keep], symmetric=False)
        sym = False
    starts = np.nonzero(g.deg > 0)[0].astype(np.int32)
    for Ns in (1, 50, 5000, 123457):
        got = orc.allocation(g, Ns, starts, symmetric=sym, min_one=min_one)
        want = _allocation_by_formula(g.dense(), starts, Ns, min_one)
        assert np.array_equal(got, want), (which, Ns)
    # Rows off the start list get none; the total is Ns up to one rounding
    # per start row (plus the forced walks with min_one).
    got = orc.allocation(g, 5000, starts, symmetric=sym, min_one=min_one)
    assert got.sum() - got[starts].sum() == 0
    assert abs(int(got.sum()) - 5000) <= starts.size
    small = orc.allocation(g, starts.size // 4, starts, symmetric=sym, min_one=min_one)
    if min_one:
        assert np.all(small[starts] >= 1)
    else:
        assert np.any(small[starts] == 0)  # N_s below the row count: some rows get none


def _two_components():
    """K_50 on nodes 0..49 next to the pair 50-51, node 50 with a self-loop."""
    src, dst = np.triu_indices(50, k=1)
    src = np.concatenate([src, [50, 50]])
    dst = np.concatenate([dst, [51, 50]])
    return G.from_edges(52, src, dst, keep_loops=True)


def test_rows_without_walks_keep_only_H(orc):
    # Section 4.1: with few walks a node whose neighbours started none keeps
    # only the exact terms, SC(i) = c0 + c1 s a_ii and TC(i) = c0 v_i + c1 (sAv)_i.
    # K_50 rows have norm 7, the pair's rows sqrt(2) and 1: with N_s = 100 the
    # pair is allocated round(0.40) = round(0.28) = 0 walks, each K_50 row 2.
    g = _two_components()
    K, s = 8, 0.05
    c = orc.coeffs(orc.FN_EXP, K)
    starts = np.nonzero(g.deg > 0)[0].astype(np.int32)
    walks = orc.allocation(g, 100, starts)
    assert walks[50] == 0 and walks[51] == 0 and np.all(walks[:50] == 2)
    d = orc.diag(g, c, N=1, K=K, scale=s, seed=2, walks=walks, want_digest=True)
    assert d["d"][50] == c[0] + c[1] * (s * 1.0)
    assert d["d"][51] == c[0]
    assert np.all(d["d"][:50] > c[0])  # the K_50 rows did get walks
    assert d["digest"][50] == 0 and d["digest"][51] == 0
    assert d["steps"] == 50 * 2 * (K - 1)
    v = np.linspace(0.5, 1.5, g.n)
    y = orc.action(g, c, v, N=1, K=K, scale=s, seed=2, walks=walks, want_q=True)
    for i, nb in ((50, v[50] + v[51]), (51, v[50])):
        assert y["y"][i] == c[0] * v[i] + c[1] * (s * nb)
    assert y["q"][50] == 0.0 and y["q"][51] == 0.0
    # With one walk at least (min_one) the pair's rows get Monte Carlo terms.
    w1 = orc.allocation(g, 100, starts, min_one=True)
    assert w1[50] == 1 and w1[51] == 1
    d1 = orc.diag(g, c, N=1, K=K, scale=s, seed=2, walks=w1)
    assert d1["d"][50] > c[0] + c[1] * s and d1["d"][51] > c[0]
    assert np.array_equal(d1["d"][:50], d["d"][:50])


def test_per_row_walk_counts(orc):
    g = G.erdos_renyi_dense(40, 0.15, seed=7)
    K, s = 6, 0.15
    c = orc.coeffs(orc.FN_EXP, K)
    # Equal per-row counts reproduce the uniform run exactly.
    same = np.where(g.deg > 0, 24, 0)
    a = orc.action(g, c, np.ones(g.n), N=24, K=K, scale=s, seed=3, want_digest=True)
    b = orc.action(g, c, np.ones(g.n), N=1, K=K, scale=s, seed=3, want_digest=True, walks=same)
    assert np.array_equal(a["y"], b["y"]) and np.array_equal(a["digest"], b["digest"])
    a = orc.diag(g, c, N=24, K=K, scale=s, seed=3, want_digest=True)
    b = orc.diag(g, c, N=1, K=K, scale=s, seed=3, want_digest=True, walks=same)
    assert np.array_equal(a["d"], b["d"]) and np.array_equal(a["digest"], b["digest"])
    # Unequal counts: still unbiased (each start row's average is), and the
    # step count is the sum over rows of walks * (K - 1) on a graph without
    # dead ends.
    starts = np.nonzero(g.deg > 0)[0].astype(np.int32)
    walks = orc.allocation(g, 40 * starts.size, starts)
    dense = orc.dense_series(g.dense(), c, s)
    ys = [orc.action(g, c, np.ones(g.n), N=1, K=K, scale=s, seed=11, request=r, walks=walks)["y"]
          for r in range(30)]
    ds = [orc.diag(g, c, N=1, K=K, scale=s, seed=11, request=r, walks=walks)["d"] for r in range(30)]
    assert _z_test(ys, dense @ np.ones(g.n)) < 5.0
    assert _z_test(ds, np.diag(dense)) < 5.0
    r = orc.action(g, c, np.ones(g.n), N=1, K=K, scale=s, seed=11, walks=walks)
    assert r["steps"] == int(walks.sum()) * (K - 1)
    with pytest.raises(orc.OracleError):
        bad = walks.copy()
        bad[starts[0]] = -1
        orc.action(g, c, np.ones(g.n), N=1, K=K, scale=s, walks=bad)
    # A row given no walk leaves q_k = 0 and starts nothing.
    none = walks.copy()
    none[starts[0]] = 0
    r0 = orc.action(g, c, np.ones(g.n), N=1, K=K, scale=s, seed=11, walks=none, want_q=True)
    assert r0["q"][starts[0]] == 0.0 and r0["steps"] == int(none.sum()) * (K - 1)
