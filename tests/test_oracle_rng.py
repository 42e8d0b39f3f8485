"""Pins for the oracle's random-number generator and transition sampler.

Philox (Salmon, Moraes, Dror, Shaw, SC'11) is written in the oracle from
its published round function.  Its structure (which words are multiplied,
the output permutation, the key schedule, the number of rounds) is pinned
by instantiating the same round function at W = 64 and comparing with
numpy's independent Philox4x64-10.  The Weyl key-schedule constants are
pinned by their definitions (fractional parts of the golden ratio and of
sqrt(3)).  The 32-bit instance used by the walks, its two round multipliers
included, is pinned by the published known-answer vectors of Philox4x32-10
(tests/golden/philox4x32_10_kat.txt), and checked for uniformity and
avalanche behaviour.
"""
import os
from decimal import Decimal, getcontext

import numpy as np
import pytest

import graphgen as G


def test_philox4x64_matches_numpy(orc):
    rng = np.random.default_rng(123)
    for _ in range(200):
        ctr = rng.integers(1, 2**63, 4, dtype=np.uint64)
        key = rng.integers(0, 2**63, 2, dtype=np.uint64)
        # numpy advances its 256-bit counter by one before each block.
        bg = np.random.Philox(counter=[int(ctr[0]) - 1, int(ctr[1]), int(ctr[2]), int(ctr[3])],
                              key=[int(key[0]), int(key[1])])
        assert np.array_equal(orc.philox4x64_10(ctr, key), bg.random_raw(4))


KAT_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "philox4x32_10_kat.txt")


def philox_kat_vectors():
    """(counter, key, expected output) triples of the known-answer file."""
    out = []
    for line in open(KAT_FILE):
        if line.strip() and not line.startswith("#"):
            w = [int(x, 16) for x in line.split()]
            out.append((w[0:4], w[4:6], w[6:10]))
    return out


def test_philox4x32_known_answers(orc):
    kats = philox_kat_vectors()
    assert len(kats) == 3
    for ctr, key, want in kats:
        got = [int(x) for x in orc.philox4x32_10(ctr, key)]
        assert got == want, (ctr, key, [hex(x) for x in got])


def _frac_bits(x: Decimal, bits: int) -> int:
    return int((x - int(x)) * (Decimal(2) ** bits))


def test_weyl_constants_are_their_definitions():
    # Key schedule increments: floor(2^W * (golden ratio - 1)) and
    # floor(2^W * (sqrt(3) - 1)), as given in the SC'11 paper.
    getcontext().prec = 60
    phi = (1 + Decimal(5).sqrt()) / 2
    s3 = Decimal(3).sqrt()
    assert _frac_bits(phi, 32) == 0x9E3779B9
    assert _frac_bits(s3, 32) == 0xBB67AE85
    assert _frac_bits(phi, 64) == 0x9E3779B97F4A7C15
    assert _frac_bits(s3, 64) == 0xBB67AE8584CAA73B
    src = open(__import__("oracle").__file__.replace("__init__.py", "mcmf_oracle.c")).read()
    for const in ("0x9E3779B9u", "0xBB67AE85u", "0x9E3779B97F4A7C15ull", "0xBB67AE8584CAA73Bull"):
        assert const in src


def test_philox4x32_uniform_and_avalanche(orc):
    # 4096 blocks of consecutive walk counters: byte histogram chi-square and
    # single-bit counter flips changing about half of the 128 output bits.
    outs = np.array([orc.philox4x32_10([k, w, 3, 0], [12345, 678]) for k in range(64)
                     for w in range(64)], dtype=np.uint32)
    bytes_ = outs.view(np.uint8).ravel()
    hist = np.bincount(bytes_, minlength=256)
    exp = bytes_.size / 256
    chi2 = ((hist - exp) ** 2 / exp).sum()
    assert chi2 < 350  # 255 d.o.f.: mean 255, sd ~22.6
    flips = []
    for b in range(32):
        a = orc.philox4x32_10([7, 9, 11, 13], [1, 2])
        c = orc.philox4x32_10([7 ^ (1 << b), 9, 11, 13], [1, 2])
        flips.append(sum(bin(int(x) ^ int(y)).count("1") for x, y in zip(a, c)))
    assert 56 < np.mean(flips) < 72
    assert len({tuple(o) for o in outs}) == len(outs)


def test_uniform_index_exact_boundaries(orc):
    # floor(u*deg/2^64): j is hit by exactly the u in [ceil(j 2^64/deg), ceil((j+1) 2^64/deg)).
    rng = np.random.default_rng(5)
    for deg in list(range(1, 40)) + [1000, 64701, 2**31 - 1]:
        for j in sorted(set(rng.integers(0, deg, 6).tolist() + [0, deg - 1])):
            lo = -((-j * 2**64) // deg)
            assert orc.uniform_index(lo, deg) == j
            if lo > 0:
                assert orc.uniform_index(lo - 1, deg) == j - 1
        assert orc.uniform_index(2**64 - 1, deg) == deg - 1


def test_uniform_index_histogram(orc):
    rng = np.random.default_rng(9)
    deg = 13
    us = rng.integers(0, 2**64, 20000, dtype=np.uint64, endpoint=False)
    js = np.array([orc.uniform_index(int(u), deg) for u in us])
    hist = np.bincount(js, minlength=deg)
    exp = us.size / deg
    assert ((hist - exp) ** 2 / exp).sum() < 40  # 12 d.o.f.


def test_weighted_sampler_frequencies(orc):
    # Definition 1 (ii): P(next = j) = |a_lj| / sum_k |a_lk|, signs ignored.
    g = G.with_random_weights(G.complete(6), seed=3, negative_fraction=0.4)
    row = 2
    lo, hi = g.row_ptr[row], g.row_ptr[row + 1]
    w = np.abs(g.val[lo:hi])
    rng = np.random.default_rng(11)
    us = rng.integers(0, 2**64, 20000, dtype=np.uint64, endpoint=False)
    js = np.array([orc.select_next(g, row, int(u)) for u in us])
    assert js.min() >= 0 and js.max() < hi - lo
    hist = np.bincount(js, minlength=hi - lo)
    exp = us.size * w / w.sum()
    assert ((hist - exp) ** 2 / exp).sum() < 25  # 4 d.o.f.
    # u = 0 picks the first entry; the largest u picks the last.
    assert orc.select_next(g, row, 0) == 0
    assert orc.select_next(g, row, 2**64 - 1) == hi - lo - 1


def test_unweighted_sampler_is_uniform_index(orc):
    g = G.star(9)
    rng = np.random.default_rng(2)
    for u in rng.integers(0, 2**64, 50, dtype=np.uint64, endpoint=False):
        assert orc.select_next(g, 0, int(u)) == orc.uniform_index(int(u), 9)
    assert orc.select_next(g, 0, 0) == 0
    assert orc.select_next(G.from_edges(3, [0], [1]), 2, 5) == -1  # no entries


def _alias_rows():
    """Weighted rows that stress the alias construction: random signed
    weights, exact zeros, all-equal weights, one dominant entry, rows of one
    entry, a row whose weights are all zero, and a long skewed row."""
    rng = np.random.default_rng(17)
    rows = [rng.uniform(0.1, 2.0, 7) * np.where(rng.random(7) < 0.4, -1, 1),
            np.array([0.5, 0.0, 1.5, 0.0, 2.0]),
            np.full(6, 0.75),
            np.array([1e-9, 1e-9, 5.0, 1e-9]),
            np.array([-3.0]),
            np.array([0.0, 0.0, 0.0]),
            rng.pareto(1.2, 300) + 1e-3]
    n = max(len(r) for r in rows)
    row_ptr = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int64)
    col = np.concatenate([np.arange(len(r)) for r in rows]).astype(np.int32)
    # Rows past the last listed one are empty; column indices stay below n.
    n = max(n, len(rows))
    row_ptr = np.concatenate([row_ptr, np.full(n - len(rows), row_ptr[-1])]).astype(np.int64)
    return G.CSR(n, row_ptr, col, np.concatenate(rows).astype(np.float64), "alias-rows"), rows


def test_alias_table_reproduces_row_distribution(orc):
    # Walker's alias method: entry j is drawn with probability
    # (prob_j + sum over i with alias_i = j of (1 - prob_i)) / d, which must be
    # |a_j| / sum |a| (Definition 1 (ii)); a row of zeros is drawn uniformly.
    g, rows = _alias_rows()
    prob, alias = orc.alias_table(g)
    for r, w in enumerate(rows):
        lo, d = int(g.row_ptr[r]), len(w)
        p, a = prob[lo:lo + d], alias[lo:lo + d]
        assert np.all((p >= 0) & (p <= 1)) and np.all((a >= 0) & (a < d))
        implied = p.copy()
        np.add.at(implied, a, 1.0 - p)
        implied /= d
        want = np.abs(w) / np.abs(w).sum() if np.abs(w).sum() > 0 else np.full(d, 1.0 / d)
        assert np.allclose(implied, want, rtol=1e-12, atol=1e-15), r
    # All-equal weights need no alias at all.
    lo = int(g.row_ptr[2])
    assert np.all(prob[lo:lo + 6] == 1.0) and np.all(alias[lo:lo + 6] == np.arange(6))


def test_alias_sampler_frequencies(orc):
    # Drawing through the tables with independent words (u, u2) gives the
    # row's distribution; u2 = 0 keeps the uniform pick whenever prob > 0.
    g = G.with_random_weights(G.complete(6), seed=3, negative_fraction=0.4)
    row = 2
    lo, hi = g.row_ptr[row], g.row_ptr[row + 1]
    w = np.abs(g.val[lo:hi])
    rng = np.random.default_rng(12)
    us = rng.integers(0, 2**64, (20000, 2), dtype=np.uint64, endpoint=False)
    js = np.array([orc.select_next(g, row, int(u), int(u2), sampler="alias") for u, u2 in us])
    assert js.min() >= 0 and js.max() < hi - lo
    hist = np.bincount(js, minlength=hi - lo)
    exp = us.shape[0] * w / w.sum()
    assert ((hist - exp) ** 2 / exp).sum() < 25  # 4 d.o.f.
    prob, alias = orc.alias_table(g)
    for u in rng.integers(0, 2**64, 50, dtype=np.uint64, endpoint=False):
        i = orc.uniform_index(int(u), hi - lo)
        assert orc.select_next(g, row, int(u), 0, sampler="alias") == (i if prob[lo + i] > 0 else alias[lo + i])
        want = i if prob[lo + i] == 1.0 else alias[lo + i]
        assert orc.select_next(g, row, int(u), 2**64 - 1, sampler="alias") == want
    # Unweighted rows ignore the mode.
    assert orc.select_next(G.star(9), 0, 2**63, 5, sampler="alias") == orc.uniform_index(2**63, 9)
