"""FP64 polish on the reduced problem (13), with a KKT add/drop loop.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Given an approximate minimiser (from FP32 FISTA or from the smoothed Newton
method), take its support S and signs, solve the stationarity condition of
the reduced problem (13) of section 3.2,
    A_S^T A_S x_S = A_S^T b - tau*sign_S,
with a direct sparse solver, then check the optimality conditions of (1):
entries whose sign disagrees with sign_S leave S; coordinates j outside S
with |A_j^T (A x - b)| > tau enter S with sign -sign(A_j^T (A x - b)).
Repeat until no change (at most ``max_rounds`` times).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def polish(A, b, tau, x_init, support_tol=0.0, max_rounds=10, kkt_slack=1e-9):
    A = sp.csc_matrix(A)
    n = A.shape[1]
    S = np.flatnonzero(np.abs(x_init) > support_tol)
    sgn = np.sign(x_init[S])
    x = np.zeros(n)
    rounds = 0
    for rounds in range(1, max_rounds + 1):
        x = np.zeros(n)
        if S.size:
            AS = A[:, S]
            M = (AS.T @ AS).tocsc()
            rhs = AS.T @ b - tau * sgn
            xs = spla.spsolve(M, rhs) if S.size > 1 else rhs / M.toarray()[0, 0]
            xs = np.atleast_1d(xs)
            bad = np.sign(xs) != sgn
            if np.any(bad):
                S, sgn = S[~bad], sgn[~bad]
                continue
            x[S] = xs
        g = A.T @ (A @ x - b)
        off = np.ones(n, dtype=bool)
        off[S] = False
        viol = np.flatnonzero(off & (np.abs(g) > tau * (1.0 + kkt_slack)))
        if viol.size == 0:
            return x, rounds
        S = np.concatenate([S, viol])
        sgn = np.concatenate([sgn, -np.sign(g[viol])])
        order = np.argsort(S)
        S, sgn = S[order], sgn[order]
    return x, rounds
