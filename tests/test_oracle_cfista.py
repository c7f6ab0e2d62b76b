"""The C/OpenMP FISTA of the oracle (used by the bench's CPU baseline at all
host cores) against the numpy oracle and against what the paper fixes."""
import numpy as np
import pytest

from oracle import cfista as C
from oracle import fista as F
from oracle import instance as OI


@pytest.fixture(scope="module")
def inst():
    o = OI.Instance(4096, 2048, 1e3, 20, 1.0, 1503035221, rounds=2)
    return o, o.sparse_A()


@pytest.mark.parametrize("threads", [1, 3, 8])
def test_equals_numpy_oracle_bit_for_bit(inst, threads):
    o, A = inst
    At = A.T.tocsr()
    ref = F.fista(lambda v: A @ v, lambda v: At @ v, o.b, o.tau, o.L, 60)
    x = C.fista(C.CsrPair(A), o.b, o.tau, o.L, 60, threads=threads)
    assert np.array_equal(x, ref)


def test_warm_start_continues_the_iteration(inst):
    # from x0 the iteration restarts its momentum (t_1 = 1), as oracle.fista
    o, A = inst
    At = A.T.tocsr()
    x0 = F.fista(lambda v: A @ v, lambda v: At @ v, o.b, o.tau, o.L, 7)
    ref = F.fista(lambda v: A @ v, lambda v: At @ v, o.b, o.tau, o.L, 9, x0=x0)
    x = C.fista(C.CsrPair(A), o.b, o.tau, o.L, 9, x0=x0, threads=4)
    assert np.array_equal(x, ref)


def test_kappa_one_is_solved_in_one_step():
    # kappa = 1: A has orthonormal columns and L = 1, so the first step
    # soft(A^T b, tau) is the minimiser, which IGen plants at x*
    o = OI.Instance(512, 256, 1.0, 9, 0.7, 1503035222, rounds=2)
    x = C.fista(C.CsrPair(o.sparse_A()), o.b, o.tau, 1.0, 1, threads=2)
    assert np.abs(x - o.xstar).max() <= 1e-12 * max(1.0, np.abs(o.xstar).max())


def test_reaches_the_planted_minimiser():
    o = OI.Instance(1024, 512, 10.0, 5, 1.0, 1503035223, rounds=2)
    A = o.sparse_A()
    x = C.fista(C.CsrPair(A), o.b, o.tau, o.L, 3000, threads=4)
    assert np.linalg.norm(x - o.xstar) / np.linalg.norm(o.xstar) <= 1e-9
    P, D, gap = F.duality_gap(lambda v: A @ v, lambda v: A.T @ v, o.b, o.tau, x)
    assert gap <= 1e-12
