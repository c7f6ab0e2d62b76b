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


def test_second_iterate_from_the_sampled_form():
    # tests/local_iterates.py: x_2 at sampled columns from the sampled form
    # equals the full oracle's FISTA (two iterations, L = 1), an FP32 run of
    # the same iteration (numpy float32, a rounding sequence of its own) stays
    # within the a-priori bound, and each planted mistake (x_1 reported, tau
    # or L off by 1%, the residual's sign flipped, a nonzero first momentum
    # step) leaves it somewhere.
    from oracle import fista as F
    from local_iterates import second_iterate, informative_columns, soft
    from fp32_bounds import fista_float32

    m, n, kappa, s, tau, seed = 1 << 15, 1 << 14, 1e6, 16, 1.0, 77
    loc = I.LocalInstance(m, n, kappa, s, tau, seed, rounds=2)
    full = I.Instance(m, n, kappa, s, tau, seed, rounds=2)
    A = full.sparse_A().tocsr()
    mv, rmv = (lambda v: A @ v), (lambda v: A.T @ v)
    js = informative_columns(loc, 48, 4)
    ref, bound = second_iterate(loc, js)
    assert np.count_nonzero(ref) >= 8
    x2 = F.fista(mv, rmv, full.b, tau, 1.0, 2)
    assert np.all(np.abs(x2[js] - ref) <= 1e-12 * np.maximum(1.0, np.abs(ref)))
    x2f = fista_float32(A, full.b, tau, 1.0, 2)
    assert np.all(np.abs(x2f[js] - ref) <= bound)
    x1 = F.fista(mv, rmv, full.b, tau, 1.0, 1)
    r = A @ x1 - full.b
    y = 1.01 * x1
    mistakes = {
        "x_1": x1,
        "tau": F.fista(mv, rmv, full.b, 0.99 * tau, 1.0, 2),
        "L": F.fista(mv, rmv, full.b, tau, 1.01, 2),
        "sign": soft(x1 + A.T @ r, tau),
        "momentum": soft(y - A.T @ (A @ y - full.b), tau),
    }
    for name, bad in mistakes.items():
        assert np.any(np.abs(bad[js] - ref) > bound), name
