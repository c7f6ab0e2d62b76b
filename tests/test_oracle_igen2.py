"""Pins of the oracle's Procedure IGen2 (section 3.2, m < n) on the
generator's matrices: the optimality conditions the procedure builds in,
step 3 against a dense solve, the unique minimiser by sign enumeration, and
the bound used for L."""
import numpy as np
import pytest

from oracle import bruteforce as BF
from oracle import fista as F
from oracle import instance as OI

CASES = [(512, 700, 1e2, 8, 1.0, 1503035230), (64, 90, 10.0, 3, 0.5, 1503035231), (6, 10, 3.0, 2, 0.3, 41)]


@pytest.mark.parametrize("cfg", CASES)
def test_planted_x_satisfies_the_optimality_conditions(cfg):
    o = OI.IGen2Instance(*cfg)
    A = o.dense_A()
    grad = A.T @ (A @ o.xstar - o.b)           # A^T (A x* - b) = -A^T e
    S = o.xstar != 0
    assert S.sum() == cfg[3]
    assert np.all(~S[o.m:])                    # x* lies in B's columns
    assert np.abs(grad[S] + o.tau * np.sign(o.xstar[S])).max() <= 1e-12 * o.tau
    assert np.abs(grad[~S]).max() < o.tau      # strictly inside off S
    assert np.abs(-grad / o.tau - o.g).max() <= 1e-12
    P, D, gap = F.duality_gap(lambda v: A @ v, lambda v: A.T @ v, o.b, o.tau, o.xstar)
    assert abs(P - o.fstar) <= 1e-12 * abs(P) and abs(gap) <= 1e-12


@pytest.mark.parametrize("cfg", CASES)
def test_step3_and_step4_against_dense_algebra(cfg):
    o = OI.IGen2Instance(*cfg)
    A = o.dense_A()
    B, Nt = A[:, : o.m], A[:, o.m:]
    # step 3: e = tau B^{-T} g on the first m components
    assert np.allclose(np.linalg.solve(B.T, o.tau * o.g[: o.m]), o.e, rtol=0, atol=1e-12 * max(1, np.abs(o.e).max()))
    # step 4: N~_k = xi_k tau / |N_k^T e| N_k with N_k = B e_{p(k)}, so |N~_k^T e| = |xi_k| tau <= tau
    assert len(set(o.p.tolist())) == o.n - o.m and np.all(np.abs(o.Bi.g[o.p]) >= 0.5)
    for k in range(o.n - o.m):
        Nk = B[:, o.p[k]]
        assert np.allclose(Nt[:, k], o.xi[k] * o.tau / abs(Nk @ o.e) * Nk, rtol=1e-14, atol=0)
    assert np.allclose(np.abs(Nt.T @ o.e), np.abs(o.xi) * o.tau, rtol=1e-12, atol=0)
    assert np.allclose(o.b, A @ o.xstar + o.e, rtol=0, atol=1e-12 * np.abs(o.b).max())


def test_unique_minimiser_by_sign_enumeration():
    o = OI.IGen2Instance(*CASES[2])
    x, f = BF.lasso_bruteforce(o.dense_A(), o.b, o.tau)
    assert np.abs(x - o.xstar).max() <= 1e-10
    assert abs(f - o.fstar) <= 1e-10 * abs(o.fstar)


@pytest.mark.parametrize("cfg", CASES)
def test_lipschitz_bound(cfg):
    o = OI.IGen2Instance(*cfg)
    A = o.dense_A()
    lam = float(np.linalg.eigvalsh(A @ A.T).max())
    assert lam <= o.L * (1 + 1e-12)
    assert o.L == 1.0 + float(np.max(o.c ** 2)) and np.abs(o.c).max() <= 2.0


def test_fista_reaches_the_planted_solution():
    o = OI.IGen2Instance(*CASES[1])
    A = o.sparse_A()
    x = F.fista(lambda v: A @ v, lambda v: A.T @ v, o.b, o.tau, o.L, 20000)
    assert np.linalg.norm(x - o.xstar) / np.linalg.norm(o.xstar) <= 1e-6


def test_argument_checks():
    with pytest.raises(ValueError):
        OI.IGen2Instance(64, 64, 10.0, 3, 1.0, 1)            # m < n required
    with pytest.raises(ValueError):
        OI.IGen2Instance(64, 90, 10.0, 3, 1.0, 1, rounds=2)  # one stage
    with pytest.raises(ValueError):
        OI.IGen2Instance(8, 40, 10.0, 3, 1.0, 1)             # more N columns than eligible B columns
