"""Pins of the section 8.9 (Table 1) instance class in the CPU oracle.

Each pin checks the oracle against something other than itself: explicit
Givens matrices built from the display of section 4, LAPACK's SVD, the
optimality conditions IGen builds b to satisfy (section 3.1), the duality
gap, and the behaviour section 8.9 reports for CG-Newton on this class.
"""
import math

import numpy as np
import pytest

from oracle import fista as OF
from oracle import newton as ON
from oracle.huge import HugeInstance, b_at_pairs, planted_at

SEED = 1503035206
CASES = [(64, 6), (130, 9), (1024, 1)]


def givens_dense(n, i, j, theta):
    """G(i, j, theta) of section 4 as an explicit n x n matrix (0-based i, j)."""
    G = np.eye(n)
    c, s = math.cos(theta), math.sin(theta)
    G[i, i], G[i, j], G[j, i], G[j, j] = c, -s, s, c
    return G


def dense_definition(I):
    """A = Sigma G^T with G the product of G(2k-1, 2k, theta), k = 1..n/2."""
    n, m = I.n, I.m
    G = np.eye(n)
    for k in range(n // 2):
        G = G @ givens_dense(n, 2 * k, 2 * k + 1, I.theta)
    Sig = np.zeros((m, n))
    Sig[:n, :n] = np.diag(I.sigma)
    return Sig @ G.T


@pytest.mark.parametrize("n,s", CASES)
def test_operator_equals_definition(n, s):
    I = HugeInstance(n, s, SEED)
    Ad = dense_definition(I)
    assert np.abs(I.sparse_A().toarray() - Ad).max() <= 1e-13
    rng = np.random.default_rng(3)
    x = rng.standard_normal(n)
    y = rng.standard_normal(I.m)
    assert np.allclose(I.matvec(x), Ad @ x, rtol=0, atol=1e-12 * np.abs(Ad @ x).max())
    assert np.allclose(I.rmatvec(y), Ad.T @ y, rtol=0, atol=1e-12 * np.abs(Ad.T @ y).max())
    assert np.allclose(I.colnorm2(), (Ad * Ad).sum(0), rtol=1e-14, atol=0)
    # rows n..m-1 are zero, and each 2 x 2 block is full (theta = 2 pi / 3)
    assert not Ad[n:].any()
    assert I.sparse_A().nnz == 2 * n


@pytest.mark.parametrize("n,s", CASES[:2])
def test_singular_values_are_the_sigma_law(n, s):
    I = HugeInstance(n, s, SEED)
    sv = np.sort(np.linalg.svd(I.sparse_A().toarray(), compute_uv=False))
    want = np.sort(np.r_[np.full(n // 2, 0.1), np.full(n // 2, 100.0)])
    assert np.abs(sv - want).max() <= 1e-12 * 100
    assert I.L == 1e4


@pytest.mark.parametrize("n,s,tau", [(64, 6, 1.0), (130, 9, 0.37), (1024, 1, 2.5)])
def test_planted_solution_is_optimal(n, s, tau):
    # IGen builds b so that A^T (A x* - b) = -tau g with g in the
    # subdifferential of ||x*||_1 (section 3.1, eq. (11)): the prox-gradient
    # fixed point holds at x*, and the duality gap of x* is zero.
    I = HugeInstance(n, s, SEED, tau=tau)
    A = I.sparse_A()
    assert np.abs(A.T @ I.e[: I.m] - I.tau * I.g).max() <= 1e-12
    # through b: rounding of b (|b| up to sigma_even |x_neg|) times sigma_even
    grad = A.T @ (A @ I.xstar - I.b)
    slack = 16 * np.finfo(float).eps * np.abs(I.b).max() * math.sqrt(I.L)
    assert np.abs(grad + I.tau * I.g).max() <= slack
    L = I.L
    fixed = OF.soft_threshold(I.xstar - grad / L, I.tau / L)
    assert np.abs(fixed - I.xstar).max() <= 1e-9 * max(1.0, np.abs(I.xstar).max())
    P, D, gap = OF.duality_gap(lambda v: A @ v, lambda v: A.T @ v, I.b, I.tau, I.xstar)
    # the dual value sums b^T u with |b| up to sigma_even |x_neg| = 1e6 against
    # u = -e of size tau / sigma_odd: FP64 cancellation leaves ~1e-8 relative
    assert abs(gap) <= 1e-6
    assert P == pytest.approx(I.fstar, rel=1e-12)


@pytest.mark.parametrize("n,s", CASES)
def test_support_values_and_subgradient(n, s):
    I = HugeInstance(n, s, SEED)
    nz = np.flatnonzero(I.xstar)
    assert len(nz) == s and len(set(I.support.tolist())) == s
    assert (I.xstar == -1e4).sum() == s // 2 and (I.xstar == 0.1).sum() == s - s // 2
    assert np.array_equal(I.g[nz], np.sign(I.xstar[nz]))
    off = np.setdiff1d(np.arange(n), nz)
    assert np.all(np.abs(I.g[off]) <= 0.9)


@pytest.mark.parametrize("n,s", CASES + [(4098, 4)])
def test_sampled_values_equal_whole_construction(n, s):
    # planted_at / b_at_pairs go through the inverse bijection, the class
    # through the forward one: the two must name the same support and b.
    I = HugeInstance(n, s, SEED)
    idx = np.arange(n)
    xs, g = planted_at(n, s, SEED, idx)
    assert np.array_equal(xs, I.xstar) and np.array_equal(g, I.g)
    bi, bj = b_at_pairs(n, s, SEED, np.arange(n // 2))
    assert np.array_equal(bi, I.b[0:n:2]) and np.array_equal(bj, I.b[1:n:2])


def test_default_s_and_sizes_of_table_1():
    # section 8.9: s = n / 2^10 and m = 2n; the smallest instance of Table 1
    n = 2 ** 30
    assert n // 1024 == 2 ** 20
    I = HugeInstance(2048, 2048 // 1024, SEED)
    assert I.m == 4096 and I.s == 2


def test_cg_newton_reproduces_section_8_9_behaviour():
    # Section 8.9 reports 8 Newton steps with about 100 PCG iterations each
    # and a solution of relative error of order 1e-4 for this class.
    n = 2 ** 14
    I = HugeInstance(n, n // 1024, SEED)
    x, st = ON.newton_cg(I.matvec, I.rmatvec, I.colnorm2(), I.b, I.tau, max_newton=8)
    rel = np.linalg.norm(x - I.xstar) / np.linalg.norm(I.xstar)
    assert st["newton"] == 7                      # 8 steps taken, none converged yet
    assert rel <= 5e-4
    assert 8 * 20 <= st["pcg"] <= 8 * 200
