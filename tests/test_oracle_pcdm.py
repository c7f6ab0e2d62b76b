"""Pins of the PCDM oracle (section 8.1 item PCDM, section 8.3) on the
generator's instances, against what the method's definition fixes."""
import numpy as np
import pytest

from oracle import instance as OI
from oracle import pcdm as P
from oracle.philox import seed_key


def _inst(m, n, kappa, s, tau, seed, rounds):
    o = OI.Instance(m, n, kappa, s, tau, seed, rounds=rounds)
    return o, o.sparse_A()


def _f(A, b, tau, x):
    r = A @ x - b
    return tau * np.abs(x).sum() + 0.5 * r @ r


@pytest.mark.parametrize("n,varpi", [(64, 1), (64, 40), (1000, 40), (1000, 7), (6, 6)])
def test_tau_nice_sets_are_distinct_and_an_epoch_is_a_permutation(n, varpi):
    key = seed_key(11)
    q = n // varpi
    seen = []
    for k in range(2 * q):
        S = P.tau_nice_set(n, varpi, k, key)
        assert S.size == varpi and np.unique(S).size == varpi
        assert S.min() >= 0 and S.max() < n
        seen.append(S)
    for e in range(2):
        ep = np.concatenate(seen[e * q:(e + 1) * q])
        assert np.unique(ep).size == q * varpi            # no coordinate twice in an epoch
    assert not np.array_equal(seen[0], seen[q])            # each epoch draws its own bijection


def test_single_coordinate_step_is_the_exact_minimiser_along_it():
    # varpi = 1 gives beta = 1, and the shrinkage step minimises f along the
    # chosen coordinate exactly (the model Q^i is f restricted to it)
    o, A = _inst(256, 128, 10.0, 5, 0.7, 3, 2)
    key = seed_key(5)
    x = 0.3 * np.sin(np.arange(o.n))
    for k in range(20):
        i = int(P.tau_nice_set(o.n, 1, k, key)[0])
        y = P.pcdm(A, o.b, o.tau, 1, 1, key, x0=x) if k == 0 else None
        # one step from x at coordinate i, taken directly
        Ai = A[:, i].toarray().ravel()
        r = A @ x - o.b
        L = Ai @ Ai
        z = x[i] - (Ai @ r) / L
        xi = np.sign(z) * max(abs(z) - o.tau / L, 0.0)
        if k == 0:
            assert np.isclose(y[i], xi) and np.array_equal(np.delete(y, i), np.delete(x, i))
        fx = _f(A, o.b, o.tau, np.where(np.arange(o.n) == i, xi, x))
        for t in np.linspace(-2.0, 2.0, 801):
            xt = x.copy()
            xt[i] = xi + t
            assert _f(A, o.b, o.tau, xt) >= fx - 1e-12 * abs(fx)
        x[i] = xi


def test_beta_and_separability_degree():
    for rounds, bound in ((1, 4), (2, 16)):
        o, A = _inst(512, 256, 100.0, 5, 1.0, 7, rounds)
        w = P.separability_degree(A)
        rows = np.diff(A.tocsr().indptr)
        assert w == rows.max() and 1 <= w <= bound
    assert P.pcdm_beta(16, 1, 1000) == 1.0
    assert P.pcdm_beta(16, 1000, 1000) == 16.0
    assert np.isclose(P.pcdm_beta(16, 40, 2 ** 20), 1.0 + 15 * 39 / (2 ** 20 - 1))


@pytest.mark.parametrize("varpi,epochs", [(1, 15), (8, 40), (40, 200)])
def test_pcdm_reaches_the_planted_minimiser(varpi, epochs):
    # Procedure IGen makes x* the minimiser (section 3.1); PCDM converges to it
    o, A = _inst(256, 128, 2.0, 4, 1.0, 1503035210, 2)
    key = seed_key(o.seed)
    steps = epochs * (o.n // varpi)
    x = P.pcdm(A, o.b, o.tau, steps, varpi, key)
    err = np.linalg.norm(x - o.xstar) / np.linalg.norm(o.xstar)
    assert err <= 1e-8, err


def test_pcdm_decreases_the_objective_from_zero():
    o, A = _inst(2048, 1024, 1e2, 10, 1.0, 1503035200, 1)
    key = seed_key(o.seed)
    f0 = _f(A, o.b, o.tau, np.zeros(o.n))
    fs = [_f(A, o.b, o.tau, P.pcdm(A, o.b, o.tau, k * (o.n // 40), 40, key)) for k in (1, 4, 16)]
    assert f0 > fs[0] > fs[1] > fs[2] >= o.fstar * (1 - 1e-12)
