"""The pins must catch plausible mistakes in the oracle.

Each case below plants one mistake in a private copy of the oracle's C
source (a wrong coefficient index, a dropped scale or sign, a biased
sampler, a wrong scatter index, a broken Philox round ...), builds it into
a temporary library, and runs the pin tests against it.  At least one pin
must fail for every planted mistake.  Everything here runs on the CPU.
"""
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
import test_oracle_pins as P
import test_oracle_rng as R

SRC = os.path.join(os.path.dirname(oracle.__file__), "mcmf_oracle.c")

MUTATIONS = {
    "action coefficient index": ("c[t + 2] * wt[t] * r[st[t]]", "c[t + 1] * wt[t] * r[st[t]]"),
    "diag coefficient index": ("Q[st[t]] + c[t + 2] * wt[t]", "Q[st[t]] + c[t + 1] * wt[t]"),
    "H term uses v for r": ("yi = yi + c[1] * r[row];", "yi = yi + c[1] * v[row];"),
    "scale dropped from weight": ("W = W * (p->s * g->rowabs[l]);", "W = W * g->rowabs[l];"),
    "sign of negative entries dropped": ("        if (a < 0.0)\n            W = -W;\n        l = g->col[e];",
                                         "        l = g->col[e];"),
    "biased uniform index": ("(unsigned __int128)u * (uint64_t)deg;",
                             "(unsigned __int128)u * (uint64_t)(deg > 1 ? deg - 1 : deg);"),
    "biased weighted sampler": ("double target = u53 * g->rowabs[l];",
                                "double target = u53 * u53 * g->rowabs[l];"),
    "rowabs without absolute value": ("sum = sum + fabs(entry(g, e));", "sum = sum + entry(g, e);"),
    "scale dropped from diag gather": ("inner = s * inner;", "inner = inner;"),
    "wrong walk normalisation": ("q[k] = sum / (double)Nk;", "q[k] = sum / (double)(Nk + 1);"),
    "weight recorded after update": ("wt[cnt] = W;", "wt[cnt] = W * (p->s * g->rowabs[l]);"),
    "diag scattered to start row": ("dsum[ii] = dsum[ii] + (s * entry(&g, e)) * inner;",
                                    "dsum[k] = dsum[k] + (s * entry(&g, e)) * inner;"),
    "diag walks start at the requested rows": ("                    start[col[e]] = 1;\n\n    for (k = 0;",
                                               "                    start[i] = 1;\n\n    for (k = 0;"),
    "philox xor word swapped": ("y0 = (UINT)(p1 >> (BITS)) ^ x1 ^ k0;", "y0 = (UINT)(p1 >> (BITS)) ^ x3 ^ k0;"),
    "philox key schedule": ("k1 += (W1);", "k1 += (W0);"),
    "philox rounds": ("round < 10; ++round", "round < 9; ++round"),
    "walks of a row share one stream": ("ctr[1] = w;", "ctr[1] = 0;"),
    "action gather misses scale": ("        yi = yi + s * sum;", "        yi = yi + sum;"),
    "allocation by squared norms": ("norm[i] = sqrt(sq);", "norm[i] = sq;"),
    "allocation truncates": ("llround((double)Ns * (norm[k] / total))",
                             "(int64_t)((double)Ns * (norm[k] / total))"),
    "allocation floors at one walk": ("if (min_one && w < 1)", "if (w < 1)"),
    "philox multiplier of word 0": ("0xD2511F53u, 0xCD9E8D57u", "0xD2511F55u, 0xCD9E8D57u"),
    "philox multiplier of word 2": ("0xD2511F53u, 0xCD9E8D57u", "0xD2511F53u, 0xCD9E8D59u"),
    "philox multipliers swapped": ("0xD2511F53u, 0xCD9E8D57u", "0xCD9E8D57u, 0xD2511F53u"),
    "alias leftover mass": ("q[big] = (q[big] + q[s]) - 1.0;", "q[big] = q[big] - q[s];"),
    "alias scaled without the row length": ("q[j] = (fabs(entry(g, b + j)) * (double)d) / W;",
                                            "q[j] = fabs(entry(g, b + j)) / W;"),
    "alias keep and alias swapped": ("v53 < g->aprob[g->row_ptr[l] + i] ? i : g->alias[g->row_ptr[l] + i]",
                                     "v53 < g->aprob[g->row_ptr[l] + i] ? g->alias[g->row_ptr[l] + i] : i"),
    "alias second word is the first": ("select_next(g, l, u, ((uint64_t)x[3] << 32) | (uint64_t)x[2])",
                                       "select_next(g, l, u, u)"),
}

PINS = [
    lambda orc: R.test_philox4x32_known_answers(orc),
    lambda orc: R.test_philox4x64_matches_numpy(orc),
    lambda orc: R.test_weighted_sampler_frequencies(orc),
    lambda orc: R.test_uniform_index_histogram(orc),
    lambda orc: P.test_K_at_most_two_is_exact(orc, 2),
    lambda orc: P.test_complete_bipartite_diag_closed_form(orc, 3, 5),
    lambda orc: P.test_regular_graph_action_on_ones(orc, lambda: P.G.torus2d(6, 7)),
    lambda orc: P.test_expectation_mode_equals_dense_series(orc, 6),
    lambda orc: P.test_unbiased(orc, "weighted", "cdf"),
    lambda orc: R.test_alias_table_reproduces_row_distribution(orc),
    lambda orc: R.test_alias_sampler_frequencies(orc),
    lambda orc: P.test_unbiased(orc, "weighted", "alias"),
    lambda orc: P.test_unbiased(orc, "rmat", "cdf"),
    lambda orc: P.test_complete_graph_exp_diag_closed_form(orc),
    lambda orc: P.test_error_decays_as_inverse_sqrt_N(orc),
    lambda orc: P.test_allocation_follows_column_norms(orc, "weighted", False),
    lambda orc: P.test_rows_without_walks_keep_only_H(orc),
]


def _build(src_text: str, tmp: str) -> str:
    c = os.path.join(tmp, "m.c")
    so = os.path.join(tmp, "libm.so")
    with open(c, "w") as f:
        f.write(src_text)
    subprocess.check_call(["gcc", "-std=gnu99", "-O2", "-ffp-contract=off", "-shared", "-fPIC",
                           "-o", so, c, "-lm"])
    return so


def _first_failing_pin():
    for i, pin in enumerate(PINS):
        try:
            pin(oracle)
        except (AssertionError, oracle.OracleError):
            return i
    return None


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name):
    old, new = MUTATIONS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation anchor not found once: {name}"
    with tempfile.TemporaryDirectory() as tmp:
        so = _build(text.replace(old, new), tmp)
        prev = oracle._swap_library(so)
        try:
            caught = _first_failing_pin()
        finally:
            oracle._swap_library(None)
            oracle._lib = prev
    assert caught is not None, f"no pin caught: {name}"


def test_unmutated_copy_passes_every_pin():
    with tempfile.TemporaryDirectory() as tmp:
        so = _build(open(SRC).read(), tmp)
        prev = oracle._swap_library(so)
        try:
            assert _first_failing_pin() is None
        finally:
            oracle._swap_library(None)
            oracle._lib = prev


def test_path_digest_definition(orc):
    # On the single edge 0-1 every walk from 0 alternates 0, 1, 0, ...; the
    # digest is the sum over walks of FNV-1a over the 32-bit state words.
    g = P.G.path(2)
    K = 5
    h = 0xCBF29CE484222325
    for state in (0, 1, 0, 1):
        h = ((h ^ state) * 0x100000001B3) % 2**64
    r = orc.action(g, orc.FN_EXP, np.ones(2), N=3, K=K, want_digest=True)
    assert int(r["digest"][0]) == (3 * h) % 2**64
