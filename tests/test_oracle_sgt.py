"""Pins of the section 8.9 (Table 1) instance class in the CPU oracle.

Each pin checks the oracle against something other than itself: explicit
Givens matrices built from the display of section 4, LAPACK's SVD, the
optimality conditions IGen builds b to satisfy (section 3.1), the duality
gap, and the behaviour section 8.9 reports for CG-Newton on this class.
"""
import math
import os

import numpy as np
import pytest

from oracle import fista as OF
from oracle import newton as ON
from oracle.sgt import SgtInstance, b_at_pairs, planted_at, uniform_sigmas

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
    I = SgtInstance(n, s, SEED)
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
    I = SgtInstance(n, s, SEED)
    sv = np.sort(np.linalg.svd(I.sparse_A().toarray(), compute_uv=False))
    want = np.sort(np.r_[np.full(n // 2, 0.1), np.full(n // 2, 100.0)])
    assert np.abs(sv - want).max() <= 1e-12 * 100
    assert I.L == 1e4


@pytest.mark.parametrize("n,s,tau", [(64, 6, 1.0), (130, 9, 0.37), (1024, 1, 2.5)])
def test_planted_solution_is_optimal(n, s, tau):
    # IGen builds b so that A^T (A x* - b) = -tau g with g in the
    # subdifferential of ||x*||_1 (section 3.1, eq. (11)): the prox-gradient
    # fixed point holds at x*, and the duality gap of x* is zero.
    I = SgtInstance(n, s, SEED, tau=tau)
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
    I = SgtInstance(n, s, SEED)
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
    I = SgtInstance(n, s, SEED)
    idx = np.arange(n)
    xs, g = planted_at(n, s, SEED, idx)
    assert np.array_equal(xs, I.xstar) and np.array_equal(g, I.g)
    bi, bj = b_at_pairs(n, s, SEED, np.arange(n // 2))
    assert np.array_equal(bi, I.b[0:n:2]) and np.array_equal(bj, I.b[1:n:2])


def test_default_s_and_sizes_of_table_1():
    # section 8.9: s = n / 2^10 and m = 2n; the smallest instance of Table 1
    n = 2 ** 30
    assert n // 1024 == 2 ** 20
    I = SgtInstance(2048, 2048 // 1024, SEED)
    assert I.m == 4096 and I.s == 2


def test_cg_newton_reproduces_section_8_9_behaviour():
    # Section 8.9 reports 8 Newton steps with about 100 PCG iterations each
    # and a solution of relative error of order 1e-4 for this class.
    n = 2 ** 14
    I = SgtInstance(n, n // 1024, SEED)
    x, st = ON.newton_cg(I.matvec, I.rmatvec, I.colnorm2(), I.b, I.tau, max_newton=8)
    rel = np.linalg.norm(x - I.xstar) / np.linalg.norm(I.xstar)
    assert st["newton"] == 7                      # 8 steps taken, none converged yet
    assert rel <= 5e-4
    assert 8 * 20 <= st["pcg"] <= 8 * 200


# ---- sigma and x* laws of sections 8.4 to 8.6 --------------------------------
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_conditioning_values.txt")


def golden():
    out = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        k, v = line.split()
        out[k] = float(v)
    return out


def test_uniform_sigma_law_gives_the_printed_condition_numbers():
    # section 8.4: sigma uniform on [0, 10^q] shifted by 0.1 at n = 2^22 gives
    # kappa(A^T A) from 1e2 to 1e12 in steps of x1e2
    n = 2 ** 22
    gv = golden()
    for q in range(6):
        sig = uniform_sigmas(n, 11, 10.0 ** q, 0.1)
        assert sig.min() >= 0.1 and sig.max() < 10.0 ** q + 0.1
        k = (sig.max() / sig.min()) ** 2
        assert abs(math.log10(k) - gv[f"kAtA_log10_q{q}"]) <= 0.15, (q, k)


@pytest.mark.parametrize("law", ["osgen", "osgen3"])
def test_laws_keep_igen_optimality(law):
    I = SgtInstance(130, 9, SEED, tau=0.37, sigma_law="uniform", sigma_scale=100.0, xstar_law=law, gamma=10.0)
    A = I.sparse_A()
    assert np.abs(A.T @ I.e[: I.m] - I.tau * I.g).max() <= 1e-12
    grad = A.T @ (A @ I.xstar - I.b)
    assert np.abs(grad + I.tau * I.g).max() <= 64 * np.finfo(float).eps * np.abs(I.b).max() * math.sqrt(I.L)
    nz = np.flatnonzero(I.xstar)
    assert np.array_equal(I.g[nz], np.sign(I.xstar[nz]))


def test_osgen_values_and_support():
    I = SgtInstance(512, 40, SEED, sigma_law="uniform", xstar_law="osgen", gamma=7.0)
    nz = np.flatnonzero(I.xstar)
    assert len(nz) == 40 and np.all(np.abs(I.xstar[nz]) <= 7.0)
    xs, g = planted_at(512, 40, SEED, np.arange(512), xstar_law="osgen", gamma=7.0)
    assert np.array_equal(xs, I.xstar) and np.array_equal(g, I.g)


@pytest.mark.parametrize("s1,s2", [(5, 5), (0, 7), (6, 0), (3, 4)])
def test_osgen3_solves_eq_19_and_keeps_extremes(s1, s2):
    # Procedure OsGen3: G^T x = gamma (Sigma^T Sigma)^{-1} 1_n exactly, then the
    # s1 smallest and s2 largest |x_i| are kept (ties by index).
    n = 256
    I = SgtInstance(n, s1 + s2, SEED, sigma_law="uniform", sigma_scale=10.0, xstar_law="osgen3", gamma=100.0,
                    s1=s1, s2=s2)
    rhs = 100.0 / I.sigma ** 2
    assert np.abs(I.apply_Gt(I.x_full) - rhs).max() <= 1e-13 * np.abs(rhs).max()
    ranked = sorted(range(n), key=lambda i: (abs(I.x_full[i]), i))
    keep = set(ranked[:s1]) | (set(ranked[n - s2:]) if s2 else set())
    assert set(np.flatnonzero(I.xstar).tolist()) <= keep
    for i in range(n):
        assert I.xstar[i] == (I.x_full[i] if i in keep else 0.0)


def test_kappa_rho_equals_eigenprojection():
    # eq. (17) with P_rho built from a dense eigendecomposition of A^T A
    I = SgtInstance(64, 8, SEED, sigma_law="uniform", sigma_scale=10.0, xstar_law="osgen3", gamma=100.0)
    Ad = I.sparse_A().toarray()
    lam, V = np.linalg.eigh(Ad.T @ Ad)
    for rho in (0.1, 1.0, 20.0):
        Vr = V[:, lam >= rho]
        den = np.linalg.norm(Vr @ (Vr.T @ I.xstar))
        want = np.linalg.norm(I.xstar) / den if den > 0 else math.inf
        assert I.kappa_rho(rho) == pytest.approx(want, rel=1e-9)


def test_printed_kappa_rho_of_sections_8_4_to_8_6():
    # the paper's kappa_0.1(x*) statements, reproduced at n = 2^20, s = n / 2^7
    n = 2 ** 20
    s = n // 2 ** 7
    gv = golden()
    k84 = [SgtInstance(n, s, 11, sigma_law="uniform", sigma_scale=10.0 ** q, xstar_law="osgen", gamma=g).kappa_rho(0.1)
           for q in (0, 2, 5) for g in (10.0, 1e3)]
    assert all(gv["kappa01_osgen"] <= k <= 1.2 * gv["kappa01_osgen"] for k in k84), k84
    assert k84[0] == pytest.approx(k84[1], rel=1e-12)   # gamma = 1e3 gives the kappa_0.1 of gamma = 10
    k85 = [SgtInstance(n, s, 11, theta=th, sigma_law="uniform", sigma_scale=10.0 ** q, xstar_law="osgen3",
                       gamma=100.0).kappa_rho(0.1)
           for th in (2 * math.pi / 10, 2 * math.pi / 1e3) for q in range(4)]
    assert 0.75 * gv["kappa01_osgen3_mean_8_5"] <= np.mean(k85) <= 1.25 * gv["kappa01_osgen3_mean_8_5"], k85
    k86 = SgtInstance(n, s, 11, theta=2 * math.pi / 10, sigma_law="uniform", sigma_scale=10.0, xstar_law="osgen3",
                      gamma=100.0).kappa_rho(0.1)
    assert 0.5 * gv["kappa01_osgen3_8_6"] <= k86 <= 1.5 * gv["kappa01_osgen3_8_6"], k86


# ---- PCDM (section 8.1) --------------------------------------------------------
def test_pcdm_single_coordinate_step_is_exact_minimisation():
    # with one coordinate sampled (p tiny, beta -> 1) the PCDM step minimises
    # f_tau exactly along that coordinate: compare with a fine 1-D search
    from oracle.sgt import pcdm
    I = SgtInstance(64, 6, SEED, sigma_law="uniform", sigma_scale=10.0, xstar_law="osgen", gamma=5.0)
    A = I.sparse_A().toarray()
    x0 = np.random.default_rng(1).standard_normal(64)
    i = 7
    Li = float(A[:, i] @ A[:, i])
    g = A[:, i] @ (A @ x0 - I.b)
    z = x0[i] - g / Li
    xi = np.sign(z) * max(abs(z) - I.tau / Li, 0.0)
    f = lambda t: I.tau * np.abs(np.r_[x0[:i], t, x0[i + 1:]]).sum() + 0.5 * np.sum(
        (A @ np.r_[x0[:i], t, x0[i + 1:]] - I.b) ** 2)
    grid = xi + np.linspace(-1e-3, 1e-3, 2001)
    assert f(xi) <= min(f(t) for t in grid) + 1e-12 * abs(f(xi))
    # beta = 1 + (omega - 1) p: p = 1 gives beta = 2, and the step is that of
    # the Jacobi splitting with 2 L_i
    x1 = pcdm(I, I.tau, 1, p=1.0, x0=x0)
    v = 2.0 * I.colnorm2()
    zz = x0 - (A.T @ (A @ x0 - I.b)) / v
    assert np.allclose(x1, np.sign(zz) * np.maximum(np.abs(zz) - I.tau / v, 0.0), rtol=0, atol=1e-12)


@pytest.mark.parametrize("p", [1.0, 0.5])
def test_pcdm_decreases_objective_and_reaches_minimiser(p):
    # PCDM with the ESO step (beta = 1 + (omega - 1) p) is a descent method in
    # expectation; on this small instance it reaches the planted x*
    from oracle.sgt import pcdm
    I = SgtInstance(256, 8, SEED, sigma_law="uniform", sigma_scale=1.0, xstar_law="osgen", gamma=5.0)
    f = lambda x: OF.primal(I.matvec, I.b, I.tau, x)
    x = pcdm(I, I.tau, 3000, p=p)
    assert f(x) <= f(np.zeros(256))
    assert np.linalg.norm(x - I.xstar) / np.linalg.norm(I.xstar) <= 1e-8


# ---- IGen2 (section 3.2, m < n) -------------------------------------------------
@pytest.mark.parametrize("m,n,s,law", [(64, 96, 6, "alternating"), (130, 260, 9, "uniform"), (128, 130, 3, "uniform")])
def test_igen2_optimality_conditions(m, n, s, law):
    from oracle.sgt import SgtIGen2Instance
    I = SgtIGen2Instance(m, n, s, SEED, tau=0.37, sigma_law=law, sigma_scale=10.0, xstar_law="osgen", gamma=3.0)
    A = I.sparse_A().toarray()
    B = A[:, :m]
    # step 3 against a dense solve: e = tau B^{-T} g
    assert np.allclose(I.e, I.tau * np.linalg.solve(B.T, I.g), rtol=1e-12, atol=1e-12 * np.abs(I.e).max())
    # eq. (15): N~^T e in tau [-1, 1], equal to xi tau sign(N^T e)
    nte = A[:, m:].T @ I.e
    assert np.all(np.abs(nte) <= I.tau * (1 + 1e-12))
    assert np.allclose(np.abs(nte), np.abs(I.xi) * I.tau, rtol=1e-12)
    # optimality of x*: A^T (A x* - b) in -tau d||x*||_1, zero duality gap
    grad = A.T @ (A @ I.xstar - I.b)
    nz = np.flatnonzero(I.xstar)
    assert len(nz) == s and np.all(nz < m)
    assert np.allclose(grad[nz], -I.tau * np.sign(I.xstar[nz]), rtol=0, atol=1e-9)
    assert np.all(np.abs(grad) <= I.tau * (1 + 1e-9))
    P, D, gap = OF.duality_gap(lambda v: A @ v, lambda v: A.T @ v, I.b, I.tau, I.xstar)
    assert abs(gap) <= 1e-9
    assert P == pytest.approx(I.fstar, rel=1e-12)
    # operator and diagonal against the explicit matrix
    x = np.random.default_rng(4).standard_normal(n)
    y = np.random.default_rng(5).standard_normal(m)
    assert np.allclose(I.matvec(x), A @ x, rtol=0, atol=1e-12 * np.abs(A @ x).max())
    assert np.allclose(I.rmatvec(y), A.T @ y, rtol=0, atol=1e-12 * np.abs(A.T @ y).max())
    assert np.allclose(I.colnorm2(), (A * A).sum(0), rtol=1e-13)


def test_igen2_fista_obeys_the_rate_towards_the_planted_optimum():
    # x* is the minimiser by construction, so FISTA from 0 obeys Beck and
    # Teboulle's f(x_k) - f* <= 2 L ||x*||^2 / (k + 1)^2 with f* = f(x*)
    from oracle.sgt import SgtIGen2Instance
    I = SgtIGen2Instance(256, 384, 8, SEED, sigma_law="uniform", sigma_scale=1.0, xstar_law="osgen", gamma=5.0)
    fstar = OF.primal(I.matvec, I.b, I.tau, I.xstar)
    for k in (10, 100, 1000):
        x = OF.fista(I.matvec, I.rmatvec, I.b, I.tau, I.L, k)
        gap = OF.primal(I.matvec, I.b, I.tau, x) - fstar
        assert -1e-9 * fstar <= gap <= 2 * I.L * float(I.xstar @ I.xstar) / (k + 1) ** 2
