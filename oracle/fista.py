"""FISTA, soft-thresholding, duality gap and power iteration (plain FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

FISTA is the first-order method of section 8.1 (Beck & Teboulle's FISTA, the
paper's reference [fista]): at the current point y it minimises the
separable model Q_tau(.; y) of eq. (4) with H = L*I, L >= lambda_max(A^T A),
whose exact minimiser is the shrinkage-thresholding (soft-threshold) step
(section 2), then extrapolates with the t_k momentum sequence.  Operators
are passed as callables so that the same loop runs on a dense matrix, a
scipy matrix or the MvPA/MvPAt products of ``oracle.instance``.
"""
import math

import numpy as np


def soft_threshold(z, thr):
    """argmin_u thr*|u| + 0.5*(u - z)^2 = sign(z) * max(|z| - thr, 0)."""
    return np.sign(z) * np.maximum(np.abs(z) - thr, 0.0)


def momentum_sequence(k):
    """t_1..t_{k+1} with t_1 = 1, t_{j+1} = (1 + sqrt(1 + 4 t_j^2)) / 2."""
    t = [1.0]
    for _ in range(k):
        t.append((1.0 + math.sqrt(1.0 + 4.0 * t[-1] * t[-1])) / 2.0)
    return t


def fista(A_mv, At_mv, b, tau, L, iters, x0=None, return_y=False):
    """Run ``iters`` FISTA iterations from x0 (default 0).

    x_0 = x0, y_1 = x_0, t_1 = 1; for k = 1, 2, ...:
      x_k     = soft(y_k - A^T(A y_k - b)/L, tau/L)
      t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2
      y_{k+1} = x_k + ((t_k - 1)/t_{k+1}) (x_k - x_{k-1})
    Returns x_iters (and y_iters, the point the last step was taken from).
    """
    n = At_mv(np.zeros_like(b)).shape[0]
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    y = x.copy()
    y_used = y
    t = 1.0
    for _ in range(iters):
        y_used = y
        grad = At_mv(A_mv(y) - b)
        x_new = soft_threshold(y - grad / L, tau / L)
        t_new = (1.0 + math.sqrt(1.0 + 4.0 * t * t)) / 2.0
        y = x_new + ((t - 1.0) / t_new) * (x_new - x)
        x, t = x_new, t_new
    if return_y:
        return x, y_used
    return x


def primal(A_mv, b, tau, x):
    """f_tau(x) = tau ||x||_1 + 0.5 ||A x - b||^2 (problem (1))."""
    r = A_mv(x) - b
    return tau * np.abs(x).sum() + 0.5 * float(r @ r)


def dual_value(At_mv, b, tau, r):
    """Lasso dual at the scaled residual u = theta*r.

    The dual of problem (1) is  max_u -0.5 ||u||^2 - b^T u  s.t.
    ||A^T u||_inf <= tau; u = theta*r with theta = min(1, tau/||A^T r||_inf)
    is feasible for any r.  (The paper states no dual; this is the standard
    Lagrange dual of (1), as used for gap certificates of l1-LS solvers.)
    """
    g_inf = float(np.abs(At_mv(r)).max()) if r.size else 0.0
    theta = 1.0 if g_inf <= tau else tau / g_inf
    u = theta * r
    return -0.5 * float(u @ u) - float(b @ u)


def duality_gap(A_mv, At_mv, b, tau, x, r_dual=None):
    """(P, D, rel_gap) with P = f_tau(x), D from r_dual (default A x - b)."""
    r = A_mv(x) - b
    P = tau * np.abs(x).sum() + 0.5 * float(r @ r)
    D = dual_value(At_mv, b, tau, r if r_dual is None else r_dual)
    return P, D, (P - D) / abs(P)


def power_iteration(A_mv, At_mv, n, iters, seed=0):
    """lambda_max(A^T A) by the power method on A^T A from a seeded start."""
    v = np.random.default_rng(seed).standard_normal(n)
    v /= np.linalg.norm(v)
    lam = 0.0
    for _ in range(iters):
        w = At_mv(A_mv(v))
        lam = float(v @ w)
        v = w / np.linalg.norm(w)
    return lam
