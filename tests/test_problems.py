"""The seeded input generators hold what their docstrings state (CPU only)."""

import numpy as np
import scipy.sparse as sp

from paper_1809_05805_amd import problems as P


def test_batch_generator_structure():
    bp = P.make_batch(nsys=20, seed=4, side_lo=5, side_hi=17)
    assert bp.nsys == 20 and bp.row_off[0] == 0
    assert np.array_equal(np.diff(bp.row_off), bp.sides.astype(np.int64) ** 2)
    assert bp.sides.min() >= 5 and bp.sides.max() <= 17
    assert np.all((bp.peclet >= 1.0) & (bp.peclet <= 100.0))
    assert np.all((bp.angle >= 0.0) & (bp.angle <= 2 * np.pi))
    A = sp.csr_matrix((bp.vals, bp.col_idx, bp.row_ptr), shape=(bp.n, bp.n))
    # block diagonal: every entry of system i's rows in system i's columns
    sysof = np.searchsorted(bp.row_off, np.arange(bp.n), side="right") - 1
    coo = A.tocoo()
    assert np.array_equal(sysof[coo.row], sysof[coo.col])
    assert np.allclose(A @ bp.x_true, bp.b, rtol=0, atol=1e-12 * np.abs(bp.b).max())
    for i in (0, 7, 19):
        s = bp.system(i)
        ref = P.convdiff(int(bp.sides[i]), 2, (np.cos(bp.angle[i]), np.sin(bp.angle[i])),
                         float(bp.peclet[i]))
        assert abs(s.scipy() - ref).max() == 0.0
        assert np.array_equal(s.b, bp.b[bp.row_off[i]: bp.row_off[i + 1]])


def test_batch_generator_seeded():
    a = P.make_batch(nsys=8, seed=1, side_lo=4, side_hi=9)
    b = P.make_batch(nsys=8, seed=1, side_lo=4, side_hi=9)
    c = P.make_batch(nsys=8, seed=2, side_lo=4, side_hi=9)
    assert np.array_equal(a.b, b.b) and np.array_equal(a.sides, b.sides)
    assert not np.array_equal(a.peclet, c.peclet)


def test_full_batch_shape():
    """The 512-system batch: sides 32..256 (n 1k to 65k per system)."""
    g = P.rng(5, 3, 0)
    sides = g.integers(32, 257, size=512)
    assert sides.min() >= 32 and sides.max() <= 256
    assert 10_000_000 < int((sides.astype(np.int64) ** 2).sum()) < 16_000_000
