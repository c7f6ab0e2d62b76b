"""The A = Sigma G^T instance class of sections 8.4 to 8.9, plain FP64 numpy.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The experiments of sections 8.4, 8.5, 8.6 and 8.9 all use A = Sigma G^T
with m = 2n rows and rank n: Sigma carries sigma_1..sigma_n on its top
n x n diagonal (section 4), and G is one stage of n/2 Givens rotations
G(2k-1, 2k, theta) on adjacent pairs, all with the same angle (section 4.1
with Q = I and no permutation).  They differ in the singular values, the
angle and the planted x*:

* sigma law "alternating" (section 8.9): sigma_i = sigma_odd for odd i and
  sigma_even for even i (1-based); 0.1 and 100 in Table 1.
* sigma law "uniform" (sections 8.4 to 8.6): sigma_i uniform on [0, 10^q],
  then shifted by 0.1 (scale = 10^q, shift = 0.1).
* x* law "table1" (section 8.9): s nonzeros, half -1e4 and the rest 0.1.
* x* law "osgen" (section 6, Procedure OsGen): s positions, values uniform
  on [-gamma, gamma].
* x* law "osgen3" (section 6, Procedure OsGen3): x = G gamma (Sigma^T
  Sigma)^{-1} 1_n solves eq. (19) exactly; the s1 smallest and the s2
  largest components in absolute value are kept, the rest set to zero.

b comes from Procedure IGen (section 3.1).  kappa_rho(x*) is eq. (17) of
section 5.

Readings where the sections leave a choice:

* Random positions (table1, osgen): the first s outputs of the support
  bijection of ``oracle.instance``; table1 gives the first floor(s/2) draws
  x_neg and the others x_pos.
* osgen values: gamma (2u - 1) with u from the x* counter (q, 0, 0x300, 0)
  of support draw q.
* uniform sigma: pair k (elements 2k, 2k+1) draws Philox counter
  (k, 0, 0x500, 0); the words (0, 1) give sigma_{2k} and (2, 3)
  sigma_{2k+1}, each u * scale + shift.
* osgen3 ranks components by (|x_i|, i): equal magnitudes are taken in
  index order.
* Subgradient off the support: U[-0.9, 0.9] from the counters of
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

from .instance import SIDE_SUPPORT, TAG_PERM, TAG_SUBGRAD, TAG_XSTAR, permutation, permutation_inverse, rotate
from .philox import philox4x32_10, seed_key, unit_double


TAG_SIGMA = 0x500


def uniform_sigmas(n, seed, scale, shift):
    """sigma_i = u_i * scale + shift, u_i uniform on [0, 1), drawn per pair."""
    key = seed_key(seed)
    w0, w1, w2, w3 = philox4x32_10(np.arange(n // 2), 0, TAG_SIGMA, 0, key)
    sig = np.empty(n)
    sig[0::2] = unit_double(w0, w1) * scale + shift
    sig[1::2] = unit_double(w2, w3) * scale + shift
    return sig


class SgtInstance:
    """One instance of the A = Sigma G^T class (FP64, 0-based indices)."""

    def __init__(self, n, s, seed, m=None, theta=2.0 * math.pi / 3.0, sigma_odd=0.1, sigma_even=100.0,
                 x_neg=-1.0e4, x_pos=0.1, tau=1.0, sigma_law="alternating", sigma_scale=1.0, sigma_shift=0.1,
                 xstar_law="table1", gamma=1.0, s1=None, s2=None):
        m = 2 * n if m is None else m
        if not (n >= 2 and n % 2 == 0 and m >= n and m % 2 == 0):
            raise ValueError("need n >= 2 even, m >= n even")
        if not (0 <= s <= n) or not tau > 0.0:
            raise ValueError("need 0 <= s <= n, tau > 0")
        self.n, self.m, self.s, self.seed = int(n), int(m), int(s), int(seed)
        self.theta, self.tau = float(theta), float(tau)
        self.c, self.sn = math.cos(self.theta), math.sin(self.theta)
        if sigma_law == "alternating":
            # sigma_i for i = 1..n: odd i (0-based even positions) sigma_odd
            self.sigma = np.where(np.arange(n) % 2 == 0, float(sigma_odd), float(sigma_even))
        elif sigma_law == "uniform":
            self.sigma = uniform_sigmas(n, seed, float(sigma_scale), float(sigma_shift))
        else:
            raise ValueError(sigma_law)
        if not np.all(self.sigma > 0.0):
            raise ValueError("singular values must be positive")
        self.L = float(self.sigma.max()) ** 2
        self.first = np.arange(0, n, 2)
        self.second = np.arange(1, n, 2)
        key = seed_key(seed)
        w0, w1, _, _ = philox4x32_10(np.arange(n), 0, TAG_SUBGRAD, 0, key)
        g = 0.9 * (2.0 * unit_double(w0, w1) - 1.0)
        self.xstar = np.zeros(n)
        if xstar_law in ("table1", "osgen"):
            self.support = permutation(np.arange(s), n, TAG_PERM | SIDE_SUPPORT, key)
            if xstar_law == "table1":
                vals = np.where(np.arange(s) < s // 2, float(x_neg), float(x_pos))
            else:
                u0, u1, _, _ = philox4x32_10(np.arange(s), 0, TAG_XSTAR, 0, key)
                vals = float(gamma) * (2.0 * unit_double(u0, u1) - 1.0)
            self.xstar[self.support] = vals
        elif xstar_law == "osgen3":
            s1 = s // 2 if s1 is None else int(s1)
            s2 = s - s1 if s2 is None else int(s2)
            if s1 < 0 or s2 < 0 or s1 + s2 != s:
                raise ValueError("need s1 + s2 = s")
            # eq. (19): G^T x = gamma (Sigma^T Sigma)^{-1} 1_n, solved exactly by x = G (...)
            self.x_full = self.apply_G(float(gamma) / (self.sigma * self.sigma))
            order = np.lexsort((np.arange(n), np.abs(self.x_full)))   # by |x|, then index
            self.support = np.r_[order[:s1], order[n - s2:]] if s2 > 0 else order[:s1]
            self.xstar[self.support] = self.x_full[self.support]
        else:
            raise ValueError(xstar_law)
        nz = np.flatnonzero(self.xstar)
        g[self.support] = np.sign(self.xstar[self.support])
        self.g = g
        # IGen step 3 with the SVD-known inverse: e = tau Sigma^{+T} G^T g
        self.e = np.zeros(m)
        self.e[:n] = self.tau * self.apply_Gt(g) / self.sigma
        # IGen step 4
        self.b = self.matvec(self.xstar) + self.e
        self.fstar = self.tau * np.abs(self.xstar).sum() + 0.5 * float(self.e @ self.e)
        self.nnz_xstar = len(nz)

    def kappa_AtA(self):
        """kappa(A^T A) = (sigma_max / sigma_min)^2 (section 5)."""
        return float((self.sigma.max() / self.sigma.min()) ** 2)

    def kappa_rho(self, rho, x=None):
        """kappa_rho(x) of eq. (17): ||x|| / ||P_rho x||, P_rho the projection on
        the eigenvectors of A^T A = G Sigma^2 G^T (the columns of G) with
        eigenvalue sigma_i^2 >= rho."""
        x = self.xstar if x is None else x
        u = self.apply_Gt(x)
        den = float(np.linalg.norm(u[self.sigma * self.sigma >= rho]))
        return float(np.linalg.norm(x)) / den if den > 0.0 else math.inf

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


def planted_at(n, s, seed, idx, x_neg=-1.0e4, x_pos=0.1, xstar_law="table1", gamma=1.0):
    """(x*_i, g_i) at the indices idx alone, without building the instance
    (x* laws "table1" and "osgen").

    i lies in supp(x*) exactly when its position q = psi^{-1}(i) under the
    support bijection is < s, since the support is the first s outputs of
    psi; the value is then that of support draw q.  Used for sampled checks
    at sizes the whole-vector construction cannot reach.
    """
    key = seed_key(seed)
    idx = np.asarray(idx, dtype=np.int64)
    q = permutation_inverse(idx, n, TAG_PERM | SIDE_SUPPORT, key) if s > 0 else np.full(idx.shape, n)
    on = q < s
    if xstar_law == "table1":
        vals = np.where(q < s // 2, float(x_neg), float(x_pos))
    elif xstar_law == "osgen":
        u0, u1, _, _ = philox4x32_10(np.where(on, q, 0), 0, TAG_XSTAR, 0, key)
        vals = float(gamma) * (2.0 * unit_double(u0, u1) - 1.0)
    else:
        raise ValueError(xstar_law)
    xs = np.where(on, vals, 0.0)
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


TAG_PCDM = 0x600


def pcdm(I, tau, iters, p=1.0, x0=None, omega=2):
    """PCDM (section 8.1 item PCDM, section 8.3) on an SgtInstance.

    Step k updates, in parallel and from the same x, every coordinate i of
    the sampled set S_k: x_i <- soft(x_i - A_i^T (A x - b) / (beta L_i),
    tau / (beta L_i)), L_i = (A^T A)_ii.  S_k holds each coordinate
    independently with probability p (a doubly uniform sampling); for it
    beta = 1 + (omega - 1) (E|S|^2 / E|S| - 1) / (n - 1) = 1 + (omega - 1) p,
    omega the largest number of nonzeros in a row of A (2 in this class).
    Coordinate 2k + e is in S_j when word e of Philox counter (k, j, 0x600, 0)
    is below p 2^32 (every coordinate when p >= 1).
    """
    n = I.n
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    beta = 1.0 + (omega - 1) * min(p, 1.0)
    v = beta * I.colnorm2()
    key = seed_key(I.seed)
    thr = min(int(p * 4294967296.0), 4294967296)
    for step in range(iters):
        g = I.rmatvec(I.matvec(x) - I.b)
        z = x - g / v
        upd = np.sign(z) * np.maximum(np.abs(z) - tau / v, 0.0)
        if p >= 1.0:
            x = upd
        else:
            w0, w1, _, _ = philox4x32_10(np.arange(n // 2), step, TAG_PCDM, 0, key)
            take = np.empty(n, dtype=bool)
            take[0::2] = w0 < thr
            take[1::2] = w1 < thr
            x = np.where(take, upd, x)
    return x


TAG_XI = 0x700


class SgtIGen2Instance:
    """Procedure IGen2 (section 3.2) for m < n on the A = Sigma G^T class.

    B (m x m) = Sigma_B G_B^T with the class's sigma law on the m columns
    and the adjacent-pair rotations of angle theta; N (m x (n-m)), n - m <= m,
    is [Sigma_N G_N^T; 0]: its column pair k couples the rows of B's pair k,
    with singular values from the same law (uniform: Philox counter
    (k, 1, 0x500, 0); alternating: the same two values) and the same angle.
    x* has s <= m nonzeros among the first m components (positions and values
    as in SgtInstance with "table1" or "osgen" over [0, m)); g is sign(x*)
    on the support and U[-0.9, 0.9] elsewhere among the first m (eq. (14)).
    IGen2: e = tau B^{-T} g (step 3), N~_j = xi_j tau / |N_j^T e| N_j with
    xi_j = 2u - 1 from Philox counter (j, 0, 0x700, 0) (step 4, xi uniform on
    [-1, 1]), A = [B, N~], b = A x* + e (step 5).
    """

    def __init__(self, m, n, s, seed, theta=2.0 * math.pi / 3.0, sigma_odd=0.1, sigma_even=100.0, x_neg=-1.0e4,
                 x_pos=0.1, tau=1.0, sigma_law="alternating", sigma_scale=1.0, sigma_shift=0.1,
                 xstar_law="table1", gamma=1.0):
        if not (m >= 2 and m % 2 == 0 and n > m and (n - m) % 2 == 0 and n - m <= m):
            raise ValueError("need m even, n > m, n - m even and <= m")
        if not (0 <= s <= m) or not tau > 0.0:
            raise ValueError("need 0 <= s <= m, tau > 0")
        self.m, self.n, self.s, self.seed = int(m), int(n), int(s), int(seed)
        self.nn = n - m
        self.theta, self.tau = float(theta), float(tau)
        self.c, self.sn = math.cos(self.theta), math.sin(self.theta)
        key = seed_key(seed)
        if sigma_law == "alternating":
            self.sigma_b = np.where(np.arange(m) % 2 == 0, float(sigma_odd), float(sigma_even))
            self.sigma_n = np.where(np.arange(self.nn) % 2 == 0, float(sigma_odd), float(sigma_even))
        elif sigma_law == "uniform":
            self.sigma_b = uniform_sigmas(m, seed, float(sigma_scale), float(sigma_shift))
            w0, w1, w2, w3 = philox4x32_10(np.arange(self.nn // 2), 1, TAG_SIGMA, 0, key)
            self.sigma_n = np.empty(self.nn)
            self.sigma_n[0::2] = unit_double(w0, w1) * float(sigma_scale) + float(sigma_shift)
            self.sigma_n[1::2] = unit_double(w2, w3) * float(sigma_scale) + float(sigma_shift)
        else:
            raise ValueError(sigma_law)
        # x* among the first m components
        self.support = permutation(np.arange(s), m, TAG_PERM | SIDE_SUPPORT, key)
        if xstar_law == "table1":
            vals = np.where(np.arange(s) < s // 2, float(x_neg), float(x_pos))
        elif xstar_law == "osgen":
            u0, u1, _, _ = philox4x32_10(np.arange(s), 0, TAG_XSTAR, 0, key)
            vals = float(gamma) * (2.0 * unit_double(u0, u1) - 1.0)
        else:
            raise ValueError(xstar_law)
        self.xstar = np.zeros(n)
        self.xstar[self.support] = vals
        w0, w1, _, _ = philox4x32_10(np.arange(m), 0, TAG_SUBGRAD, 0, key)
        g = 0.9 * (2.0 * unit_double(w0, w1) - 1.0)
        g[self.support] = np.sign(vals)
        self.g = g
        # IGen2 step 3: e = tau B^{-T} g = tau Sigma_B^{-1} G_B^T g
        self.e = self.tau * self._rot(g, transpose=True) / self.sigma_b
        # IGen2 step 4: N~_j = xi_j tau / |N_j^T e| N_j
        ntE = self._rot(self.sigma_n * self.e[: self.nn], transpose=False)   # N^T e = G_N Sigma_N e_top
        u0, u1, _, _ = philox4x32_10(np.arange(self.nn), 0, TAG_XI, 0, key)
        self.xi = 2.0 * unit_double(u0, u1) - 1.0
        self.colscale = self.xi * self.tau / np.abs(ntE)
        # IGen2 step 5
        self.b = self.matvec(self.xstar) + self.e
        self.fstar = self.tau * np.abs(self.xstar).sum() + 0.5 * float(self.e @ self.e)
        A = self.sparse_A().toarray() if n <= 4096 else None
        self.L = float(np.linalg.eigvalsh(A @ A.T).max()) if A is not None else None

    def _rot(self, z, transpose):
        z = np.array(z, dtype=np.float64, copy=True)
        k = len(z)
        return rotate(z, np.arange(0, k, 2), np.arange(1, k, 2), self.c, self.sn, transpose=transpose)

    def matvec(self, x):
        """A x = B x_B + N~ x_N (m entries)."""
        x = np.asarray(x, dtype=np.float64)
        m, nn = self.m, self.nn
        y = self.sigma_b * self._rot(x[:m], transpose=True)
        y[:nn] += self.sigma_n * self._rot(self.colscale * x[m:], transpose=True)
        return y

    def rmatvec(self, y):
        """A^T y = [B^T y; N~^T y] (n entries)."""
        y = np.asarray(y, dtype=np.float64)
        m, nn = self.m, self.nn
        out = np.empty(self.n)
        out[:m] = self._rot(self.sigma_b * y, transpose=False)
        out[m:] = self.colscale * self._rot(self.sigma_n * y[:nn], transpose=False)
        return out

    def colnorm2(self):
        """diag(A^T A)."""
        out = np.empty(self.n)
        c2, s2 = self.c ** 2, self.sn ** 2
        sb, sn_ = self.sigma_b, self.sigma_n
        out[0:self.m:2] = sb[0::2] ** 2 * c2 + sb[1::2] ** 2 * s2
        out[1:self.m:2] = sb[0::2] ** 2 * s2 + sb[1::2] ** 2 * c2
        cs = self.colscale
        out[self.m::2] = cs[0::2] ** 2 * (sn_[0::2] ** 2 * c2 + sn_[1::2] ** 2 * s2)
        out[self.m + 1::2] = cs[1::2] ** 2 * (sn_[0::2] ** 2 * s2 + sn_[1::2] ** 2 * c2)
        return out

    def sparse_A(self):
        """A = [B, N~] as a scipy CSR matrix, from the explicit 2 x 2 blocks."""
        m, nn = self.m, self.nn
        rows, cols, vals = [], [], []
        c, s = self.c, self.sn
        for k in range(m // 2):
            i, j = 2 * k, 2 * k + 1
            # B block: Sigma_B G_B^T on columns (i, j): rows i: sigma_i (c, s); j: sigma_j (-s, c)
            rows += [i, i, j, j]
            cols += [i, j, i, j]
            vals += [self.sigma_b[i] * c, self.sigma_b[i] * s, -self.sigma_b[j] * s, self.sigma_b[j] * c]
            if j < nn:
                a, bb = self.colscale[i], self.colscale[j]
                rows += [i, i, j, j]
                cols += [m + i, m + j, m + i, m + j]
                vals += [self.sigma_n[i] * c * a, self.sigma_n[i] * s * bb, -self.sigma_n[j] * s * a,
                         self.sigma_n[j] * c * bb]
        A = sp.csr_matrix((vals, (rows, cols)), shape=(m, self.n))
        A.sort_indices()
        return A
