"""The diagonal gather's table plan (csrc/plan.hpp), checked on the CPU over
a sweep of graph sizes, walk counts, series lengths and LDS budgets: every
pass must leave at least one empty slot (the probe sequences end at an empty
slot) and fit the budget, also for the restricted tables of small items,
whose keys are column entries rather than visited states."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2308_01037_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include "plan.hpp"
int main() {
    const long long ns[] = {1, 2, 7, 8, 9, 100, 1000, 12000, 1 << 20, 1LL << 30};
    const long long Ns[] = {1, 2, 3, 7, 8, 64, 100, 256, 1000, 4096, 65536, 1LL << 32};
    const int Ks[] = {2, 3, 4, 9, 10, 30, 40, 100, 1000, 4096};
    const size_t budgets[] = {16384, 32768, 65536, 100000, 150000, 155000};
    long long checked = 0;
    for (long long n : ns) for (long long N : Ns) for (int K : Ks) for (size_t b : budgets) {
        mcmf::GatherPlan p = mcmf::plan_gather(n, N, K, b, 8192, 8);
        const long long cap_max = ((long long)((b - 8192) / 12) / 8) * 8;
        const bool one_walk_fits = (long long)(K - 1) * 10 <= cap_max * 9 || n * 10 <= cap_max * 9;
        if (!p.ok) {
            if (one_walk_fits) { printf("FAIL plan refused n=%lld N=%lld K=%d b=%zu\n", n, N, K, b); return 1; }
            continue;
        }
        long long v = p.walks_per_pass * (long long)(K - 1);
        long long d = v < n ? v : n;
        // A restricted table (only when all N walks fit one pass) claims at
        // most visits * Den / Num column entries as keys, and at most n.
        if (p.walks_per_pass >= N) {
            long long keys = (N * (long long)(K - 1) * (long long)mcmf::kRestrictDen) /
                             (long long)mcmf::kRestrictNum;
            if (keys > n) keys = n;
            if (keys >= p.cap) { printf("FAIL restricted n=%lld N=%lld K=%d\n", n, N, K); return 1; }
        }
        if (p.cap % 8 || p.cap <= p.distinct_max || d != p.distinct_max || p.walks_per_pass < 1 ||
            p.walks_per_pass > N || p.lds_bytes > b) {
            printf("FAIL n=%lld N=%lld K=%d b=%zu cap=%lld wpp=%lld d=%lld lds=%zu\n", n, N, K, b,
                   (long long)p.cap, (long long)p.walks_per_pass, (long long)p.distinct_max, p.lds_bytes);
            return 1;
        }
        ++checked;
    }
    printf("ok %lld\n", checked);
    return 0;
}
"""


def test_plan_always_leaves_a_free_slot(tmp_path):
    src = tmp_path / "plan_check.cpp"
    src.write_text(DRIVER)
    exe = tmp_path / "plan_check"
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-I", CSRC, str(src), "-o", str(exe)])
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout
    assert out.stdout.startswith("ok")
