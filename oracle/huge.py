"""Huge-scale instance class of section 8.9 (Table 1), plain FP64 numpy.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Section 8.9 builds its instances as A = Sigma G^T with m = 2n rows and rank
n: no left rotations and no permutation (the construction of section 4.1
with Q = I), G one stage of n/2 Givens rotations G(2k-1, 2k, theta) on
adjacent pairs, all with the same angle theta = 2 pi / 3, sigma_i = 0.1 for
odd i and 100 for even i (1-based), and x* with s = n / 2^10 nonzeros, half
of them -1e4 and the rest 0.1.  b comes from Procedure IGen (section 3.1)
with tau = 1 (section 8.3).

Readings where the section leaves a choice:

* Support positions: the first s outputs of the support bijection of
  ``oracle.instance`` (random positions); the first floor(s/2) draws get
  x_neg, the others x_pos.
* Subgradient off the support: U[-0.9, 0.9] from the same counters as
  ``oracle.instance`` (a strict interior choice of eq. (10)'s [-1, 1]).
* Rotation convention: G(i, j, theta) maps (z_i, z_j) to
  (c z_i - s z_j, s z_i + c z_j) (section 4), c = cos theta, s = sin theta.

Because Sigma's bottom m - n rows are zero and the rotations pair
neighbours, A is block diagonal with 2 x 2 blocks: everything here is
written as plain whole-vector numpy on the pair arrays, and ``sparse_A``
gives the explicit matrix for tests.
"""
import math

import numpy as np
import scipy.sparse as sp

from .instance import SIDE_SUPPORT, TAG_PERM, TAG_SUBGRAD, permutation, permutation_inverse, rotate
from .philox import philox4x32_10, seed_key, unit_double


class HugeInstance:
    """One instance of the section 8.9 class (FP64, 0-based indices)."""

    def __init__(self, n, s, seed, m=None, theta=2.0 * math.pi / 3.0, sigma_odd=0.1, sigma_even=100.0,
                 x_neg=-1.0e4, x_pos=0.1, tau=1.0):
        m = 2 * n if m is None else m
        if not (n >= 2 and n % 2 == 0 and m >= n and m % 2 == 0):
            raise ValueError("need n >= 2 even, m >= n even")
        if not (0 <= s <= n) or not tau > 0.0 or not (sigma_odd > 0.0 and sigma_even > 0.0):
            raise ValueError("need 0 <= s <= n, tau > 0, sigma > 0")
        self.n, self.m, self.s, self.seed = int(n), int(m), int(s), int(seed)
        self.theta, self.tau = float(theta), float(tau)
        self.c, self.sn = math.cos(self.theta), math.sin(self.theta)
        # sigma_i for i = 1..n: odd i (0-based even positions) sigma_odd
        self.sigma = np.where(np.arange(n) % 2 == 0, float(sigma_odd), float(sigma_even))
        self.L = float(max(sigma_odd, sigma_even)) ** 2
        self.first = np.arange(0, n, 2)
        self.second = np.arange(1, n, 2)
        key = seed_key(seed)
        self.support = permutation(np.arange(s), n, TAG_PERM | SIDE_SUPPORT, key)
        vals = np.where(np.arange(s) < s // 2, float(x_neg), float(x_pos))
        self.xstar = np.zeros(n)
        self.xstar[self.support] = vals
        w0, w1, _, _ = philox4x32_10(np.arange(n), 0, TAG_SUBGRAD, 0, key)
        g = 0.9 * (2.0 * unit_double(w0, w1) - 1.0)
        g[self.support] = np.sign(vals)
        self.g = g
        # IGen step 3 with the SVD-known inverse: e = tau Sigma^{+T} G^T g
        self.e = np.zeros(m)
        self.e[:n] = self.tau * self.apply_Gt(g) / self.sigma
        # IGen step 4
        self.b = self.matvec(self.xstar) + self.e
        self.fstar = self.tau * np.abs(self.xstar).sum() + 0.5 * float(self.e @ self.e)

    def apply_Gt(self, x):
        z = np.array(x, dtype=np.float64, copy=True)
        return rotate(z, self.first, self.second, self.c, self.sn, transpose=True)

    def apply_G(self, x):
        z = np.array(x, dtype=np.float64, copy=True)
        return rotate(z, self.first, self.second, self.c, self.sn)

    def matvec(self, x):
        """A x (Algorithm MvPA with Q = I): G^T, then Sigma (n -> m)."""
        out = np.zeros(self.m)
        out[: self.n] = self.sigma * self.apply_Gt(x)
        return out

    def rmatvec(self, y):
        """A^T y (Algorithm MvPAt with Q = I): Sigma^T (m -> n), then G."""
        return self.apply_G(self.sigma * np.asarray(y, dtype=np.float64)[: self.n])

    def colnorm2(self):
        """diag(A^T A): squared norms of the columns of A."""
        a = np.zeros(self.n)
        a[self.first] = self.sigma[self.first] ** 2 * self.c ** 2 + self.sigma[self.second] ** 2 * self.sn ** 2
        a[self.second] = self.sigma[self.first] ** 2 * self.sn ** 2 + self.sigma[self.second] ** 2 * self.c ** 2
        return a

    def sparse_A(self):
        """A = Sigma G^T as a scipy CSR matrix."""
        n, m = self.n, self.m
        i, j = self.first, self.second
        # G^T restricted to the pair: rows (i, j) = [[c, s], [-s, c]]
        rows = np.concatenate([i, i, j, j])
        cols = np.concatenate([i, j, i, j])
        vals = np.concatenate([np.full(len(i), self.c), np.full(len(i), self.sn),
                               np.full(len(i), -self.sn), np.full(len(i), self.c)])
        Gt = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
        Sig = sp.csr_matrix((self.sigma, (np.arange(n), np.arange(n))), shape=(m, n))
        A = (Sig @ Gt).tocsr()
        A.sort_indices()
        return A


def planted_at(n, s, seed, idx, x_neg=-1.0e4, x_pos=0.1):
    """(x*_i, g_i) at the indices idx alone, without building the instance.

    i lies in supp(x*) exactly when its position q = psi^{-1}(i) under the
    support bijection is < s, since the support is the first s outputs of
    psi; q < floor(s/2) gives x_neg.  Used for sampled checks at sizes the
    whole-vector construction cannot reach.
    """
    key = seed_key(seed)
    idx = np.asarray(idx, dtype=np.int64)
    q = permutation_inverse(idx, n, TAG_PERM | SIDE_SUPPORT, key) if s > 0 else np.full(idx.shape, n)
    on = q < s
    xs = np.where(on, np.where(q < s // 2, float(x_neg), float(x_pos)), 0.0)
    w0, w1, _, _ = philox4x32_10(idx, 0, TAG_SUBGRAD, 0, key)
    g = np.where(on, np.sign(xs), 0.9 * (2.0 * unit_double(w0, w1) - 1.0))
    return xs, g


def b_at_pairs(n, s, seed, pairs, theta=2.0 * math.pi / 3.0, sigma_odd=0.1, sigma_even=100.0,
               x_neg=-1.0e4, x_pos=0.1, tau=1.0):
    """b at the two rows of each pair k in `pairs` (rows 2k, 2k+1), by IGen
    steps 3 and 4 on that pair alone: e = tau Sigma^{-1} G^T g, b = A x* + e."""
    pairs = np.asarray(pairs, dtype=np.int64)
    i, j = 2 * pairs, 2 * pairs + 1
    xi, gi = planted_at(n, s, seed, i, x_neg, x_pos)
    xj, gj = planted_at(n, s, seed, j, x_neg, x_pos)
    c, sn = math.cos(theta), math.sin(theta)
    ei = tau * (c * gi + sn * gj) / sigma_odd
    ej = tau * (-sn * gi + c * gj) / sigma_even
    bi = sigma_odd * (c * xi + sn * xj) + ei
    bj = sigma_even * (-sn * xi + c * xj) + ej
    return bi, bj
