"""Pins of the oracle's sampled form (``oracle.instance.LocalInstance``):
evaluated at every index of small instances it must give what the full
construction (``Instance``, itself pinned to the paper in
``test_oracle_pins.py``) gives: A's columns and rows (Algorithms MvPA /
MvPAt on sparse vectors, section 4), x*, g and sigma bit for bit, and b of
Procedure IGen (section 3.1) up to the order of the additions.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import instance as I

CASES = [
    (16, 8, 1e2, 2, 1.0, 7, 2),
    (8, 8, 10.0, 3, 0.5, 3, 2),        # square
    (6, 4, 3.0, 1, 1.0, 5, 2),         # smallest two-stage sides (cycles of 4 and 6)
    (4, 2, 3.0, 1, 1.0, 5, 1),         # smallest instance
    (1010, 502, 1e3, 7, 0.5, 17, 2),   # ragged
    (2048, 1024, 1e2, 10, 1.0, 1503035200, 1),
    (512, 256, 1e4, 0, 1.0, 9, 2),     # s = 0
]


@pytest.mark.parametrize("cfg", CASES)
def test_local_instance_equals_full_construction(cfg):
    m, n, kappa, s, tau, seed, r = cfg
    full = I.Instance(m, n, kappa, s, tau, seed, rounds=r)
    loc = I.LocalInstance(m, n, kappa, s, tau, seed, rounds=r)
    A = full.sparse_A()
    o, i, v = loc.columns(np.arange(n))
    B = sp.csc_matrix((v, (i, o)), shape=(m, n))
    assert abs(A - B).max() <= 4e-16 * max(1.0, abs(A).max())
    o, j, v = loc.rows(np.arange(m))
    C = sp.csr_matrix((v, (o, j)), shape=(m, n))
    assert abs(A - C).max() <= 4e-16 * max(1.0, abs(A).max())
    # the pattern too: every entry produced is one of A's
    Bc = B.tocoo()
    produced = {(a, b) for a, b, v in zip(Bc.row, Bc.col, Bc.data) if v != 0.0}
    assert produced <= set(zip(*A.nonzero()))
    assert np.array_equal(loc.sigma(np.arange(n)), full.sigma)
    assert np.array_equal(loc.xstar(np.arange(n)), full.xstar)
    assert np.array_equal(loc.subgradient(np.arange(n)), full.g)
    assert np.array_equal(loc.index(I.SIDE_N, np.arange(n)), full.perm_n)
    assert np.array_equal(loc.index(I.SIDE_M, np.arange(m)), full.perm_m)
    scale = max(1.0, np.abs(full.b).max())
    assert np.abs(loc.e(np.arange(m)) - full.e).max() <= 1e-13 * scale
    assert np.abs(loc.b(np.arange(m)) - full.b).max() <= 1e-13 * scale


def test_local_instance_sampled_subsets_agree_with_whole_evaluation():
    # evaluating a subset (in any order, with repeats) gives the same numbers
    # as evaluating everything: no hidden dependence on the batch
    cfg = (1010, 502, 1e3, 7, 0.5, 17, 2)
    loc = I.LocalInstance(*cfg[:6], rounds=cfg[6])
    js = np.array([501, 0, 17, 17, 250])
    o, i, v = loc.columns(js)
    oa, ia, va = loc.columns(np.arange(502))
    for q, j in enumerate(js):
        a = sorted(zip(i[o == q], v[o == q]))
        b = sorted(zip(ia[oa == j], va[oa == j]))
        assert a == b
    rs = np.array([1009, 3, 3, 600])
    assert np.array_equal(loc.b(rs), loc.b(np.arange(1010))[rs])
