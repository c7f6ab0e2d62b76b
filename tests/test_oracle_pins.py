"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test names what it pins.  None of them retypes the oracle's formula:
they compare against published values (Philox known answers, the sparsity
counts printed in section 4.2), against library routines that compute the
same object another way (LAPACK SVD / solve / eigvalsh, scipy minimisers),
against brute force, or against closed forms and invariants.
"""
import math
import os

import numpy as np
import pytest
import scipy.optimize

from oracle import bruteforce, fista as F, instance as I, newton, philox, polish

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_rows(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


# --------------------------------------------------------------------------
# Philox-4x32-10: published known-answer values
# --------------------------------------------------------------------------
def test_philox_known_answers():
    for row in _golden_rows("philox4x32_10_kat.txt"):
        v = [int(h, 16) for h in row]
        out = philox.philox4x32_10(v[0], v[1], v[2], v[3], (v[4], v[5]))
        assert [int(o) for o in out] == v[6:10]


def test_philox_vectorised_matches_scalar():
    ctr = np.arange(100, dtype=np.uint64)
    vec = philox.philox4x32_10(ctr, 7, 9, 11, (123, 456))
    for i in (0, 17, 99):
        sc = philox.philox4x32_10(i, 7, 9, 11, (123, 456))
        assert [int(a[i]) for a in vec] == [int(a) for a in sc]


# --------------------------------------------------------------------------
# Random bijections (Feistel + cycle walking)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("N", [2, 4, 6, 10, 1000, 1024, 2048, 4098])
def test_permutation_is_bijection_and_inverse(N):
    key = philox.seed_key(99)
    p = I.permutation(np.arange(N), N, I.TAG_PERM | 1, key)
    assert sorted(p.tolist()) == list(range(N))
    inv = I.permutation_inverse(p, N, I.TAG_PERM | 1, key)
    assert np.array_equal(inv, np.arange(N))


def test_permutation_depends_on_seed_and_tag():
    N = 1024
    a = I.permutation(np.arange(N), N, I.TAG_PERM, philox.seed_key(1))
    b = I.permutation(np.arange(N), N, I.TAG_PERM, philox.seed_key(2))
    c = I.permutation(np.arange(N), N, I.TAG_PERM | 1, philox.seed_key(1))
    assert not np.array_equal(a, b) and not np.array_equal(a, c)


# --------------------------------------------------------------------------
# Givens rotation convention (section 4, display of G(i, j, theta))
# --------------------------------------------------------------------------
def test_givens_quarter_turn_maps_ei_to_ej():
    # With theta = pi/2 (c = 0, s = 1) the display gives G e_i = e_j and
    # G e_j = -e_i: column i holds (c, s) in rows (i, j), column j (-s, c).
    for (i, j) in [(0, 3), (3, 0), (2, 5)]:
        ei = np.zeros(6)
        ei[i] = 1.0
        ej = np.zeros(6)
        ej[j] = 1.0
        one = np.array([1.0])
        zero = np.array([0.0])
        a = I.rotate(ei.copy(), np.array([i]), np.array([j]), zero, one)
        b = I.rotate(ej.copy(), np.array([i]), np.array([j]), zero, one)
        assert np.array_equal(a, ej) and np.array_equal(b, -ei)
        # transpose undoes it
        a2 = I.rotate(a, np.array([i]), np.array([j]), zero, one, transpose=True)
        assert np.array_equal(a2, ei)


def test_givens_explicit_matrix_entries():
    # theta = pi/6 on plane (1, 3) of R^4: the four nontrivial entries of
    # the display, row i = (c, -s), row j = (s, c), identity elsewhere.
    c, s = math.cos(math.pi / 6), math.sin(math.pi / 6)
    M = np.zeros((4, 4))
    for col in range(4):
        e = np.zeros(4)
        e[col] = 1.0
        M[:, col] = I.rotate(e, np.array([1]), np.array([3]), np.array([c]), np.array([s]))
    expect = np.eye(4)
    expect[1, 1], expect[1, 3], expect[3, 1], expect[3, 3] = c, -s, s, c
    assert np.array_equal(M, expect)


# --------------------------------------------------------------------------
# Generated instances: structure of eq. (16) and Procedure IGen
# --------------------------------------------------------------------------
SMALL = [  # (m, n, kappa, s, tau, seed, rounds)
    (32, 16, 10.0, 3, 0.7, 11, 1),
    (64, 24, 1e3, 5, 1.0, 12, 2),
    (40, 40, 1e2, 6, 2.0, 13, 3),
    (2048, 1024, 1e2, 10, 1.0, 1503035200, 1),
]


def _explicit_stage_product(N, stages, transpose_each, order):
    """Dense product of the stages' rotation matrices in the given order."""
    M = np.eye(N)
    for idx in order:
        st = stages[idx]
        R = np.eye(N)
        for i, j, c, s in zip(st.first, st.second, st.c, st.s):
            Gij = np.eye(N)
            Gij[i, i], Gij[i, j], Gij[j, i], Gij[j, j] = c, -s, s, c
            R = R @ Gij
        M = M @ (R.T if transpose_each else R)
    return M


@pytest.mark.parametrize("cfg", SMALL[:3])
def test_operator_equals_definition_by_matrix_products(cfg):
    # MvPA / MvPAt against A = Q Sigma G^T built from dense rotation
    # matrices multiplied in the composition order G = S_r ... S_1.
    m, n, kappa, s, tau, seed, r = cfg
    inst = I.Instance(m, n, kappa, s, tau, seed, rounds=r)
    G = _explicit_stage_product(n, inst.G_stages, False, list(reversed(range(r))))
    Q = _explicit_stage_product(m, inst.Q_stages, False, list(reversed(range(r))))
    Sig = np.zeros((m, n))
    Sig[np.arange(n), np.arange(n)] = inst.sigma
    A = Q @ Sig @ G.T
    x = np.random.default_rng(1).standard_normal(n)
    y = np.random.default_rng(2).standard_normal(m)
    assert np.allclose(inst.matvec(x), A @ x, rtol=0, atol=1e-13)
    assert np.allclose(inst.rmatvec(y), A.T @ y, rtol=0, atol=1e-13)
    assert np.allclose(inst.dense_A(), A, rtol=0, atol=1e-14)


@pytest.mark.parametrize("cfg", SMALL)
def test_singular_values_and_orthogonality(cfg):
    m, n, kappa, s, tau, seed, r = cfg
    inst = I.Instance(m, n, kappa, s, tau, seed, rounds=r)
    A = inst.dense_A()
    sv = np.linalg.svd(A, compute_uv=False)
    assert np.allclose(np.sort(sv), np.sort(inst.sigma), rtol=1e-12, atol=0)
    assert inst.sigma[0] == 1.0 and math.isclose(inst.sigma[-1], 1.0 / kappa, rel_tol=1e-14)
    x = np.random.default_rng(3).standard_normal(n)
    # ||A x|| = ||Sigma G^T x|| and ||G^T x|| = ||x||
    assert math.isclose(np.linalg.norm(inst.matvec(x)),
                        np.linalg.norm(inst.sigma * inst.apply_Gt(x)), rel_tol=1e-13)
    assert math.isclose(np.linalg.norm(inst.apply_Gt(x)), np.linalg.norm(x), rel_tol=1e-13)
    y = np.random.default_rng(4).standard_normal(m)
    assert math.isclose(np.linalg.norm(inst.apply_Qt(y)), np.linalg.norm(y), rel_tol=1e-13)
    assert math.isclose(inst.matvec(x) @ y, x @ inst.rmatvec(y), rel_tol=1e-12)


@pytest.mark.parametrize("cfg", SMALL)
def test_igen_noise_matches_literal_formula(cfg):
    # IGen step 3 written literally with a dense solve: e = tau A (A^T A)^{-1} g
    m, n, kappa, s, tau, seed, r = cfg
    inst = I.Instance(m, n, kappa, s, tau, seed, rounds=r)
    A = inst.dense_A()
    e_lit = tau * A @ np.linalg.solve(A.T @ A, inst.g)
    scale = np.abs(e_lit).max()
    assert np.abs(inst.e - e_lit).max() <= 1e-12 * kappa ** 2 * max(scale, 1.0) * 1e-2
    # eq. (11): A^T e = tau g, and b = A x* + e
    assert np.abs(A.T @ inst.e - tau * inst.g).max() <= 1e-10 * tau * max(1.0, kappa)
    assert np.abs(inst.b - (A @ inst.xstar + inst.e)).max() <= 1e-12 * max(1.0, np.abs(inst.b).max())


@pytest.mark.parametrize("cfg", SMALL)
def test_planted_solution_is_optimal(cfg):
    m, n, kappa, s, tau, seed, r = cfg
    inst = I.Instance(m, n, kappa, s, tau, seed, rounds=r)
    A = inst.dense_A()
    mv, rmv = (lambda v: A @ v), (lambda v: A.T @ v)
    grad = A.T @ (A @ inst.xstar - inst.b)
    # prox-gradient fixed point: x* = soft(x* - grad, tau)
    kkt = np.abs(inst.xstar - F.soft_threshold(inst.xstar - grad, tau)).max()
    assert kkt <= 1e-10 * max(1.0, kappa)
    P, D, gap = F.duality_gap(mv, rmv, inst.b, tau, inst.xstar)
    assert D <= P * (1 + 1e-13) and abs(gap) <= 1e-12
    assert math.isclose(P, inst.fstar, rel_tol=1e-12)
    # closed form f* = tau ||x*||_1 + 0.5 tau^2 sum_j (G^T g)_j^2 / sigma_j^2
    closed = tau * np.abs(inst.xstar).sum() + 0.5 * tau ** 2 * np.sum(
        (inst.apply_Gt(inst.g) / inst.sigma) ** 2)
    assert math.isclose(closed, inst.fstar, rel_tol=1e-12)


@pytest.mark.parametrize("cfg", SMALL)
def test_support_values_and_subgradient(cfg):
    m, n, kappa, s, tau, seed, r = cfg
    inst = I.Instance(m, n, kappa, s, tau, seed, rounds=r)
    sup = np.flatnonzero(inst.xstar)
    assert sup.size == s and np.array_equal(np.sort(inst.support), sup)
    off = np.setdiff1d(np.arange(n), sup)
    assert np.all(np.abs(inst.g[off]) <= 0.9)
    assert np.array_equal(inst.g[sup], np.sign(inst.xstar[sup]))


def test_nnz_bounds_per_row_and_column():
    for r in (1, 2):
        inst = I.Instance(4096, 2048, 1e3, 20, 1.0, 5, rounds=r)
        A = inst.sparse_A()
        assert np.diff(A.indptr).max() <= 4 ** r
        assert np.diff(A.tocsc().indptr).max() <= 4 ** r
        # almost every column is full (pair merges are rare)
        assert A.nnz >= 0.99 * (4 ** r) * 2048


def test_rotation_angles_unit_and_uniform():
    c, s = I.stage_angles(0, 1, 200000, philox.seed_key(3))
    assert np.abs(c * c + s * s - 1.0).max() <= 1e-15
    theta = np.mod(np.arctan2(s, c), 2 * np.pi)
    hist, _ = np.histogram(theta, bins=16, range=(0, 2 * np.pi))
    expected = 200000 / 16
    chi2 = np.sum((hist - expected) ** 2 / expected)
    assert chi2 < 45.0          # 15 dof, p ~ 1e-4


# --------------------------------------------------------------------------
# Paper's printed sparsity counts (section 4.2), n = 8
# --------------------------------------------------------------------------
def _paper_stage(kind, N, theta):
    if kind == "adj":     # 1-based (2k-1, 2k), k = 1..N/2
        f, g = np.arange(0, N, 2), np.arange(1, N, 2)
    else:                 # 1-based (2k, 2k+1), k = 1..N/2-1
        f, g = np.arange(1, N - 1, 2), np.arange(2, N, 2)
    return I.Stage(f, g, np.full(f.size, math.cos(theta)), np.full(f.size, math.sin(theta)))


def _compose(N, kinds, theta):
    M = np.eye(N)
    for kind in reversed(kinds):          # rightmost factor acts first
        st = _paper_stage(kind, N, theta)
        for j in range(N):
            M[:, j] = I.rotate(M[:, j].copy(), st.first, st.second, st.c, st.s)
    return M


N_SIDE = {1: ["adj"], 2: ["sh", "adj"], 3: ["adj", "sh", "adj"], 4: ["sh", "adj", "sh", "adj"]}
M_SIDE = {1: ["adj"], 2: ["adj", "sh"], 3: ["adj", "sh", "adj"], 4: ["sh", "adj", "sh", "adj"]}


def test_paper_sparsity_counts_n8():
    rows = _golden_rows("paper_sparsity_n8.txt")
    n, m, theta = 8, 16, 2 * math.pi / 10
    sig = np.linspace(0.3, 7.0, n)
    rng = np.random.default_rng(0)
    for row in rows:
        k, nnz_ata, nnz_a = int(row[0]), int(row[1]), int(row[2])
        G = _compose(n, N_SIDE[k], theta)
        ata = G @ np.diag(sig ** 2) @ G.T
        assert np.count_nonzero(np.abs(ata) > 1e-12) == nnz_ata
        # nnz(A) was one random draw of P: it must be a reachable count
        Gm = _compose(m, M_SIDE[k], theta)
        Sig = np.zeros((m, n))
        Sig[np.arange(n), np.arange(n)] = sig
        counts = []
        for _ in range(400):
            P = np.eye(m)[rng.permutation(m)]
            A = P @ Gm @ P @ Sig @ G.T
            counts.append(np.count_nonzero(np.abs(A) > 1e-12))
        assert min(counts) <= nnz_a <= max(counts)


# --------------------------------------------------------------------------
# FISTA and the duality gap
# --------------------------------------------------------------------------
def test_fista_one_step_exact_for_orthonormal_columns():
    # kappa = 1: A^T A = I, the minimiser is soft(A^T b, tau) (textbook) and
    # the generator planted x*, so one FISTA step from 0 must return x*.
    inst = I.Instance(64, 32, 1.0, 5, 0.8, 21, rounds=2)
    A = inst.dense_A()
    assert np.allclose(A.T @ A, np.eye(32), atol=1e-14)
    x1 = F.fista(lambda v: A @ v, lambda v: A.T @ v, inst.b, inst.tau, 1.0, 1)
    assert np.abs(x1 - inst.xstar).max() <= 1e-14
    assert np.abs(x1 - F.soft_threshold(A.T @ inst.b, inst.tau)).max() <= 1e-15


def test_fista_zero_when_tau_dominates():
    inst = I.Instance(64, 32, 10.0, 5, 1.0, 22, rounds=1)
    A = inst.dense_A()
    tau = 1.0001 * np.abs(A.T @ inst.b).max()
    x = F.fista(lambda v: A @ v, lambda v: A.T @ v, inst.b, tau, 1.0, 50)
    assert np.array_equal(x, np.zeros(32))


def test_fista_beck_teboulle_rate():
    # Beck & Teboulle, Theorem 4.4: f(x_k) - f* <= 2 L ||x_0 - x*||^2 / (k+1)^2
    inst = I.Instance(512, 256, 1e2, 6, 1.0, 23, rounds=2)
    A = inst.sparse_A()
    mv, rmv = (lambda v: A @ v), (lambda v: A.T @ v)
    x0 = np.zeros(256)
    bound0 = 2.0 * inst.L * np.sum((x0 - inst.xstar) ** 2)
    for k in (1, 2, 5, 10, 50, 200):
        xk = F.fista(mv, rmv, inst.b, inst.tau, inst.L, k)
        assert F.primal(mv, inst.b, inst.tau, xk) - inst.fstar <= bound0 / (k + 1) ** 2 + 1e-9 * inst.fstar


def test_fista_lyapunov_nonincreasing():
    # Beck & Teboulle, Lemma 4.1 (the step behind Theorem 4.4): with
    # v_k = f(x_k) - f* and u_k = t_k x_k - (t_k - 1) x_{k-1} - x*, the
    # quantity (2/L) t_k^2 v_k + ||u_k||^2 never increases along FISTA.
    inst = I.Instance(128, 64, 30.0, 5, 1.0, 28, rounds=2)
    A = inst.dense_A()
    mv, rmv = (lambda v: A @ v), (lambda v: A.T @ v)
    t = F.momentum_sequence(60)
    xs = [np.zeros(64)] + [F.fista(mv, rmv, inst.b, inst.tau, inst.L, k) for k in range(1, 61)]
    E = []
    for k in range(1, 61):
        v = F.primal(mv, inst.b, inst.tau, xs[k]) - inst.fstar
        u = t[k - 1] * xs[k] - (t[k - 1] - 1.0) * xs[k - 1] - inst.xstar
        E.append(2.0 / inst.L * t[k - 1] ** 2 * v + u @ u)
    for k in range(len(E) - 1):
        assert E[k + 1] <= E[k] * (1 + 1e-10) + 1e-9


@pytest.mark.parametrize("seed", [31, 32])
def test_fista_reaches_bruteforce_solution(seed):
    inst = I.Instance(16, 8, 5.0, 3, 0.5, seed, rounds=2)
    A = inst.dense_A()
    xb, fb = bruteforce.lasso_bruteforce(A, inst.b, inst.tau)
    assert np.abs(xb - inst.xstar).max() <= 1e-12
    x = F.fista(lambda v: A @ v, lambda v: A.T @ v, inst.b, inst.tau, 1.0, 3000)
    assert np.abs(x - xb).max() <= 1e-9


def test_bruteforce_on_non_planted_tau():
    # tau different from the generating one: the optimum is no longer x*;
    # brute force and scipy's bounded split formulation must agree.
    inst = I.Instance(20, 10, 3.0, 4, 1.0, 41, rounds=1)
    A = inst.dense_A()
    tau = 0.3
    xb, fb = bruteforce.lasso_bruteforce(A, inst.b, tau)
    # x = u - v, u, v >= 0: smooth bound-constrained problem
    def fun(z):
        u, v = z[:10], z[10:]
        r = A @ (u - v) - inst.b
        g = A.T @ r
        return tau * z.sum() + 0.5 * r @ r, np.concatenate([tau + g, tau - g])
    res = scipy.optimize.minimize(fun, np.zeros(20), jac=True, method="L-BFGS-B",
                                  bounds=[(0, None)] * 20, options=dict(ftol=1e-15, gtol=1e-12, maxiter=5000))
    assert res.fun >= fb - 1e-9 and abs(res.fun - fb) <= 1e-7 * max(1.0, abs(fb))
    assert np.abs((res.x[:10] - res.x[10:]) - xb).max() <= 1e-5


def test_duality_gap_brackets_optimum():
    inst = I.Instance(256, 128, 1e2, 4, 1.0, 24, rounds=2)
    A = inst.sparse_A()
    mv, rmv = (lambda v: A @ v), (lambda v: A.T @ v)
    rng = np.random.default_rng(5)
    for _ in range(5):
        x = inst.xstar + 0.1 * rng.standard_normal(128)
        P, D, gap = F.duality_gap(mv, rmv, inst.b, inst.tau, x)
        assert D <= inst.fstar * (1 + 1e-14) and inst.fstar <= P * (1 + 1e-14) and gap >= 0
    # equality at (x*, u = A x* - b = -e)
    assert math.isclose(F.dual_value(rmv, inst.b, inst.tau, -inst.e), inst.fstar, rel_tol=1e-12)


def test_power_iteration_reaches_sigma1_squared():
    inst = I.Instance(256, 128, 4.0, 4, 1.0, 25, rounds=2)
    A = inst.dense_A()
    lam = F.power_iteration(lambda v: A @ v, lambda v: A.T @ v, 128, 1000)
    assert math.isclose(lam, np.linalg.eigvalsh(A.T @ A).max(), rel_tol=1e-6)
    assert math.isclose(lam, 1.0, rel_tol=1e-6)


def test_momentum_sequence_properties():
    t = F.momentum_sequence(50)
    assert t[0] == 1.0
    for k in range(50):   # t_{k+1}^2 - t_{k+1} = t_k^2 and t_k >= (k+2)/2
        assert math.isclose(t[k + 1] ** 2 - t[k + 1], t[k] ** 2, rel_tol=1e-12)
        assert t[k] >= (k + 2) / 2.0 - 1e-12


# --------------------------------------------------------------------------
# Smoothed Newton-CG and polish
# --------------------------------------------------------------------------
@pytest.mark.parametrize("hessian", ["primal", "primal_dual"])
def test_newton_cg_minimises_smoothed_problem(hessian):
    inst = I.Instance(64, 32, 1e2, 4, 1.0, 26, rounds=2)
    A = inst.dense_A()
    mv, rmv = (lambda v: A @ v), (lambda v: A.T @ v)
    mu = 1e-3
    cn = (A * A).sum(0)
    x, st = newton.newton_cg(mv, rmv, cn, inst.b, inst.tau, mu=mu, hessian=hessian, grad_tol=1e-10)
    # independent minimiser of problem (8): scipy BFGS on the smooth objective
    fun = lambda v: newton.smoothed_objective(mv, inst.b, inst.tau, mu, v)
    jac = lambda v: inst.tau * v / np.sqrt(mu * mu + v * v) + A.T @ (A @ v - inst.b)
    ref = scipy.optimize.minimize(fun, np.zeros(32), jac=jac, method="BFGS",
                                  options=dict(gtol=1e-11, maxiter=20000))
    assert fun(x) <= ref.fun + 1e-9
    assert np.abs(x - ref.x).max() <= 1e-4
    # O(mu) distance to the l1 minimiser
    assert np.abs(x - inst.xstar).max() <= 50 * mu


@pytest.mark.parametrize("kappa,tol", [(1e2, 1e-11), (1e4, 1e-8)])
def test_polish_recovers_planted_solution(kappa, tol):
    inst = I.Instance(4096, 2048, kappa, 20, 1.0, 27, rounds=2)
    A = inst.sparse_A()
    # perturbed guess: one true support index missing, one wrong one present
    guess = inst.xstar.copy()
    guess[inst.support[0]] = 0.0
    wrong = np.setdiff1d(np.arange(2048), inst.support)[5]
    guess[wrong] = 0.3
    x, rounds = polish.polish(A, inst.b, inst.tau, guess)
    assert np.linalg.norm(x - inst.xstar) <= tol * np.linalg.norm(inst.xstar)
    assert rounds >= 2
