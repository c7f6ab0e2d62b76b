"""Tolerance of an FP32 FISTA trajectory against the FP64 oracle.

The FP32 path rounds A and b once and then every product, sum and stored
iterate.  The rounding that dominates is that of the residual r = A x - b,
whose entries start at the size of b: it is of the order of rounding b
itself.  FISTA's momentum step y = x_k + beta (x_k - x_{k-1}) makes the
iteration map expansive (up to 1 + 2 beta per step), so a linear-growth
argument does not bound how such perturbations propagate.  Instead the
exact FP64 trajectory's response to perturbations of that kind is measured
twice on the host: the oracle's FISTA on A and b rounded to FP32 (FP64
arithmetic), and the same iteration carried out in FP32 arithmetic (numpy
float32 products, sums and iterates, a different rounding sequence from the
device's).  The bound is a multiple of the larger response, with a floor of
a few FP32 units in the last place of the iterate.
"""
import numpy as np

from oracle import fista as F

EPS32 = float(np.finfo(np.float32).eps)


def fista_float32(A, b, tau, L, iters, x0=None):
    """The FISTA iteration of oracle.fista carried out in FP32 (an
    instrument for the size of FP32 rounding effects, not a reference)."""
    A32 = A.astype(np.float32)
    At32 = A32.T.tocsr() if hasattr(A32, "tocsr") else A32.T
    b32 = np.asarray(b, dtype=np.float32)
    n = At32.shape[0]
    x = np.zeros(n, np.float32) if x0 is None else np.asarray(x0, dtype=np.float32)
    y = x.copy()
    thr, Lf = np.float32(tau / L), np.float32(L)
    t = 1.0
    for _ in range(iters):
        z = y - (At32 @ ((A32 @ y) - b32)) / Lf
        xn = (np.sign(z) * np.maximum(np.abs(z) - thr, np.float32(0.0))).astype(np.float32)
        tn = (1.0 + np.sqrt(1.0 + 4.0 * t * t)) / 2.0
        y = (xn + np.float32((t - 1.0) / tn) * (xn - x)).astype(np.float32)
        x, t = xn, tn
    return x.astype(np.float64)


def fp32_trajectory_bound(A, b, tau, L, iters, factor=8.0, x_ref=None, x0=None):
    """(x_ref, bound): the FP64 oracle iterate after `iters` steps (from x0,
    default 0) and the tolerance for an FP32 run of the same iteration."""
    if x_ref is None:
        x_ref = F.fista(lambda v: A @ v, lambda v: A.T @ v, b, tau, L, iters, x0=x0)
    A32 = A.astype(np.float32).astype(np.float64)
    At32 = A32.T.tocsr() if hasattr(A32, "tocsr") else A32.T
    b32 = np.asarray(b, dtype=np.float32).astype(np.float64)
    x_data = F.fista(lambda v: A32 @ v, lambda v: At32 @ v, b32, tau, L, iters, x0=x0)
    x_arith = fista_float32(A, b, tau, L, iters, x0=x0)
    sens = max(float(np.abs(x_data - x_ref).max()), float(np.abs(x_arith - x_ref).max()))
    floor = 16.0 * EPS32 * max(1.0, float(np.abs(x_ref).max()))
    return x_ref, factor * sens + floor
