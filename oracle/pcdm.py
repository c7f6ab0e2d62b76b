"""PCDM on the generator's instances (plain FP64 numpy / scipy.sparse).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Section 8.1 (item PCDM): at a point x the method builds, for each of the
coordinates it updates in parallel, the separable model
    Q^i(y_i; x) = tau |y_i| + 0.5 ||A x - b||^2 + (A_i^T (A x - b)) (y_i - x_i)
                  + (beta L_i / 2) (y_i - x_i)^2,
with L_i = (A^T A)_ii, and minimises it exactly by shrinkage:
    y_i = soft(x_i - A_i^T (A x - b) / (beta L_i), tau / (beta L_i)).
Section 8.3 fixes beta = 1 + (omega - 1)(varpi - 1)/(n - 1), omega the
degree of partial separability of 0.5 ||A x - b||^2 (the largest number of
nonzeros in a row of A) and varpi the number of coordinates updated together
(40 there).  The residual r = A x - b is kept and updated by A_S dx_S after
each step.

The paper runs the varpi updates asynchronously; here a step updates its
varpi coordinates synchronously from the same x.  The coordinates of a step
are a uniformly random varpi-subset (tau-nice sampling): step k of epoch
e = k // q (q = floor(n / varpi) steps per epoch) takes positions
[(k mod q) varpi, (k mod q + 1) varpi) of a random bijection pi_e of
{0..n-1} (the Feistel bijection of oracle.instance with tag 0x10000 + e).
"""
import numpy as np
import scipy.sparse as sp

from .instance import permutation

TAG_PCDM_EPOCH = 0x10000


def tau_nice_set(n, varpi, step, key):
    """The coordinates (original indices) updated by step `step`."""
    q = n // varpi
    e, i = divmod(int(step), q)
    return permutation(np.arange(i * varpi, (i + 1) * varpi), n, TAG_PCDM_EPOCH + e, key)


def separability_degree(A):
    """omega: the largest number of nonzeros in a row of A."""
    A = sp.csr_matrix(A)
    return int(np.diff(A.indptr).max()) if A.shape[0] else 0


def pcdm_beta(omega, varpi, n):
    """beta = 1 + (omega - 1)(varpi - 1)/(n - 1) (section 8.3)."""
    return 1.0 + (omega - 1) * (varpi - 1) / max(n - 1, 1)


def pcdm(A, b, tau, steps, varpi, key, x0=None, beta=None):
    """x after `steps` PCDM steps of `varpi` coordinates each."""
    A = sp.csc_matrix(A)
    n = A.shape[1]
    L = np.asarray(A.multiply(A).sum(axis=0)).ravel()
    if beta is None:
        beta = pcdm_beta(separability_degree(A), varpi, n)
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    r = A @ x - b
    for k in range(steps):
        S = tau_nice_set(n, varpi, k, key)
        AS = A[:, S]
        g = AS.T @ r
        v = beta * L[S]
        z = x[S] - g / v
        y = np.sign(z) * np.maximum(np.abs(z) - tau / v, 0.0)
        dx = y - x[S]
        x[S] = y
        r = r + AS @ dx
    return x
