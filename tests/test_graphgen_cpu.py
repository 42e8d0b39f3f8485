"""The input generators on the CPU: the native R-MAT generator builds a
valid symmetric, loop-free, deduplicated CSR whatever the thread count, and
follows the same distribution as the numpy R-MAT definition."""
import os
import subprocess
import sys

import numpy as np

import graphgen as G

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _check_csr(g):
    assert g.row_ptr[0] == 0 and g.row_ptr[-1] == g.nnz == g.col.size
    assert np.all(np.diff(g.row_ptr) >= 0)
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    assert np.all((g.col >= 0) & (g.col < g.n))
    assert not np.any(rows == g.col), "self-loop"
    # Strictly increasing within each row: sorted and no duplicates.
    same_row = rows[1:] == rows[:-1]
    assert np.all(g.col[1:][same_row] > g.col[:-1][same_row])
    # Symmetric: the transposed entry set equals the entry set.
    fwd = rows.astype(np.int64) * g.n + g.col
    bwd = g.col.astype(np.int64) * g.n + rows
    assert np.array_equal(np.sort(fwd), np.sort(bwd))


def test_native_rmat_is_a_valid_symmetric_graph():
    g = G.rmat_native(12, seed=5)
    assert g.n == 4096
    _check_csr(g)


def test_native_rmat_does_not_depend_on_threads():
    code = ("import sys; sys.path.insert(0, %r); import graphgen as G; "
            "print(G.rmat_native(13, seed=9).sha256())" % ROOT)
    shas = set()
    for threads in ("1", "3"):
        env = dict(os.environ, OMP_NUM_THREADS=threads)
        shas.add(subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                                check=True).stdout.strip())
    assert len(shas) == 1
    assert G.rmat_native(13, seed=9).sha256() in shas
    assert G.rmat_native(13, seed=10).sha256() not in shas


def test_native_rmat_matches_the_numpy_distribution():
    a = G.rmat_native(16, seed=1)
    b = G.rmat(16, seed=1)
    # Different random streams, same construction: sizes agree to a few per cent.
    assert abs(a.nnz - b.nnz) / b.nnz < 0.01
    da, db = a.deg, b.deg
    assert abs((da == 0).mean() - (db == 0).mean()) < 0.01
    assert 0.8 < da.max() / db.max() < 1.25
    sa, sb = np.sort(da)[::-1][:100], np.sort(db)[::-1][:100]
    assert abs(sa.sum() - sb.sum()) / sb.sum() < 0.1
    # Quadrant probabilities all on (0,0): every edge draw is the loop (0,0).
    z = G.rmat_native(8, a=1.0, b=0.0, c=0.0, seed=3, permute=False)
    assert z.nnz == 0
