"""Exact l1-LS solution by enumeration of sign patterns (n <= 12).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Section 3.2 reduces problem (1), once the support S and the signs of x* are
known, to the smooth problem (13) whose stationary points satisfy
A_S^T A_S x_S = A_S^T b - tau*sign(x*_S).  Enumerating every sign pattern
in {-1, 0, +1}^n, solving that system and keeping the patterns that satisfy
the optimality conditions of (1) (sign(x_S) = pattern on S and
|A_j^T (A x - b)| <= tau off S, the subdifferential form quoted before
eq. (11)) gives every minimiser; with A of full column rank the minimiser is
unique.  3^12 = 531441 small solves at most.
"""
import itertools

import numpy as np


def lasso_bruteforce(A, b, tau, tol=1e-9):
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    if n > 12:
        raise ValueError("brute force is for n <= 12")
    AtA = A.T @ A
    Atb = A.T @ b
    best_x, best_f = None, np.inf
    for pattern in itertools.product((-1, 0, 1), repeat=n):
        sgn = np.array(pattern, dtype=np.float64)
        S = np.flatnonzero(sgn)
        x = np.zeros(n)
        if S.size:
            M = AtA[np.ix_(S, S)]
            try:
                xs = np.linalg.solve(M, Atb[S] - tau * sgn[S])
            except np.linalg.LinAlgError:
                continue
            if np.any(np.sign(xs) != sgn[S]):
                continue
            x[S] = xs
        g = AtA @ x - Atb                    # A^T (A x - b)
        off = np.setdiff1d(np.arange(n), S)
        if off.size and np.abs(g[off]).max() > tau * (1.0 + tol):
            continue
        r = A @ x - b
        f = tau * np.abs(x).sum() + 0.5 * r @ r
        if f < best_f:
            best_x, best_f = x, f
    return best_x, best_f
