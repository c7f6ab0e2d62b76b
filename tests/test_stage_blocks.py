"""The structure the blocked stored operator relies on (two Givens stages,
eq. (16), section 4.2 pairs): with G = S_2 S_1 and Q = S~_2 S~_1,

    A = Q Sigma G^T = sum_{i < n} sigma_i (Q e_i)(G e_i)^T,

and in stage order (position p holds index pi(p)) G e_i is supported on the
four consecutive positions 2k-1 .. 2k+2 (mod n) around i's stage-1 pair k,
with values (-v0 s2, v0 c2, v1 c2', v1 s2') from the pair's rotation
(v0, v1) and the two stage-2 rotations that meet it; the same holds for
Q e_i on the m side.  Checked on the CPU against the oracle's A, including
the smallest sides (4 and 6 positions, where the runs wrap), and with the
sum of term magnitudes |Q| Sigma |G|^T that bounds the FP32 rounding of the
blocked products.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import instance as I


def stage_run(perm, stages, i):
    """(indices, values) of S_2 S_1 e_i on one side, in run order."""
    N = len(perm)
    pinv = np.argsort(perm)
    a = int(pinv[i])
    k = a >> 1
    c1, s1 = stages[0].c[k], stages[0].s[k]
    v0, v1 = (-s1, c1) if (a & 1) else (c1, s1)
    ka = (k - 1) % (N // 2)
    c2a, s2a = stages[1].c[ka], stages[1].s[ka]
    c2b, s2b = stages[1].c[k], stages[1].s[k]
    vals = [-(v0 * s2a), v0 * c2a, v1 * c2b, v1 * s2b]
    pos = [(2 * k - 1 + t) % N for t in range(4)]
    return [int(perm[p]) for p in pos], vals


CASES = [(16, 8), (8, 8), (6, 4), (4, 4), (64, 32), (1010, 502)]


@pytest.mark.parametrize("m,n", CASES)
def test_rank_one_runs_sum_to_A(m, n):
    inst = I.Instance(m, n, 1e2, 2, 1.0, 7, rounds=2)
    A = inst.dense_A()
    B = np.zeros((m, n))
    T = np.zeros((m, n))
    for i in range(n):
        ri, u = stage_run(inst.perm_m, inst.Q_stages, i)
        ci, w = stage_run(inst.perm_n, inst.G_stages, i)
        assert len(set(ri)) == 4 and len(set(ci)) == 4      # four distinct positions, also when wrapping
        for r in range(4):
            for c in range(4):
                B[ri[r], ci[c]] += inst.sigma[i] * u[r] * w[c]
                T[ri[r], ci[c]] += abs(inst.sigma[i] * u[r] * w[c])
    assert np.abs(A - B).max() <= 1e-15 * max(1.0, np.abs(A).max())
    # the magnitudes of the terms sum to |Q| Sigma |G|^T: with two stages each
    # entry of Q and G is one product of stage coefficients
    Gt = sp.identity(n, format="csr")
    for st in inst.G_stages:
        Gt = Gt @ abs(I.Instance._stage_matrix(n, st, transpose=True))
    Q = sp.identity(m, format="csr")
    for st in inst.Q_stages:
        Q = abs(I.Instance._stage_matrix(m, st)) @ Q
    Sig = sp.csr_matrix((inst.sigma, (np.arange(n), np.arange(n))), shape=(m, n))
    assert np.abs((Q @ (Sig @ Gt)).toarray() - T).max() <= 1e-15 * max(1.0, T.max())


@pytest.mark.parametrize("m,n", [(16, 8), (1010, 502), (8, 8)])
def test_rows_hold_at_most_four_runs_and_columns_exactly_four(m, n):
    # row p is covered by the runs of the (at most four) middle indices at the
    # m-positions of its two covering stage-1 pairs; column a by exactly four
    inst = I.Instance(m, n, 1e2, 2, 1.0, 11, rounds=2)
    rows = np.zeros(m, dtype=int)
    cols = np.zeros(n, dtype=int)
    for i in range(n):
        ri, _ = stage_run(inst.perm_m, inst.Q_stages, i)
        ci, _ = stage_run(inst.perm_n, inst.G_stages, i)
        rows[ri] += 1
        cols[ci] += 1
    assert rows.max() <= 4 and rows.sum() == 4 * n
    assert np.all(cols == 4)
