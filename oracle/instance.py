"""Instance generator of the l1-LS problem, plain FP64 numpy.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

What is generated (Fountoulakis & Gondzio, arXiv:1503.03520):

* Problem (1), section 1: minimise  tau*||x||_1 + 0.5*||A x - b||^2.
* A is built with a known SVD as in eq. (16) of section 4,
  A = Q Sigma G^T, where Sigma (m x n) carries sigma_1..sigma_n on its top
  diagonal and zeros below (section 4, the display of Sigma), and G, Q are
  products of Givens rotations G(i,j,theta) whose (i,j) block is
  [[c, -s], [s, c]] (section 4, the display of G(i,j,theta)).
* b comes from Procedure IGen (section 3.1): pick a subgradient g of
  ||x*||_1 (eq. (10)), set e = tau*A(A^T A)^{-1} g (step 3) and b = A x* + e
  (step 4).  With the SVD known, (A^T A)^{-1} = G (Sigma^T Sigma)^{-1} G^T
  (section 4), so e = tau * Q Sigma^{+T} G^T g.
* Operator products follow Algorithms MvPA / MvPAt (section 4): A x applies
  the factors of G^T, then Sigma, then the factors of Q; A^T y the reverse.

Readings where the paper leaves a choice (each one is listed with its reason
in the design notes of the repository):

* Rotation stages.  Section 4.2 builds denser A by alternating a stage of
  rotations on adjacent pairs (2k-1, 2k) with a stage on shifted pairs
  (2k, 2k+1), both under a random permutation P (section 4.1).  Here each
  side (n for G, m for Q) draws one random bijection pi; stage t pairs
  (pi(2k), pi(2k+1)) for odd t and (pi(2k+1), pi(2k+2 mod N)) for even t
  (0-based positions; the shifted stage wraps around so that every stage is
  a perfect matching of N/2 rotations).  Each rotation gets its own angle,
  uniform on [0, 2 pi).
* Composition order.  G = S_r ... S_2 S_1 and Q = S~_r ... S~_1, so stage 1
  sits next to Sigma on both sides (as in the paper's n-side compositions
  G, G_2 G, G G_2 G, G_2 G G_2 G of section 4.2).  Within a pair (i, j) the
  rotation is G(i, j, theta) with i the first element.
* sigma_j = kappa^(-(j-1)/(n-1)), j = 1..n, so cond(A) = kappa and
  kappa(A^T A) = kappa^2 in the sense of section 5; L = sigma_1^2 = 1.
* x*: support = first s outputs of a third random bijection of {0..n-1},
  values N(0,1) (Box-Muller); g_i = sign(x*_i) on the support and
  U[-0.9, 0.9] off it (a strict interior choice of the [-1,1] case of
  eq. (10)).

Every random draw comes from Philox-4x32-10 (``oracle.philox``) under the
counter layout documented on each function, so that an independent
implementation reproduces the same instance.
"""
import math

import numpy as np
import scipy.sparse as sp

from .philox import philox4x32_10, seed_key, unit_double

SIDE_N = 0          # G acts on R^n
SIDE_M = 1          # Q acts on R^m
SIDE_SUPPORT = 2    # bijection that picks supp(x*)
TAG_PERM = 0x100    # | side
TAG_ANGLE = 0x200   # | side
TAG_XSTAR = 0x300
TAG_SUBGRAD = 0x400
TAG_IGEN2_PICK = 0x900   # bijection choosing the columns of B that N copies
TAG_IGEN2_XI = 0xA00     # counter (k, 0, tag, 0): xi_k of N column k
ANGLE_MAX_ATTEMPTS = 32
FEISTEL_ROUNDS = 4


# ----------------------------------------------------------------------------
# Random bijection of {0..N-1}: balanced Feistel network (Luby-Rackoff) on
# 2*h bits, round function = low h bits of the first Philox word of counter
# (R, round, tag, 0); cycle-walking maps the 2^(2h) domain back onto [0, N).
# ----------------------------------------------------------------------------
def feistel_half_bits(N):
    bits = max(1, (int(N) - 1).bit_length())
    return (bits + 1) // 2


def _round_fn(t, R, tag, key, mask):
    w0, _, _, _ = philox4x32_10(R, t, tag, 0, key)
    return w0 & mask


def feistel_encrypt(x, half, tag, key):
    mask = np.uint64((1 << half) - 1)
    x = np.asarray(x, dtype=np.uint64)
    L, R = x >> np.uint64(half), x & mask
    for t in range(FEISTEL_ROUNDS):
        L, R = R, L ^ _round_fn(t, R, tag, key, mask)
    return (L << np.uint64(half)) | R


def feistel_decrypt(y, half, tag, key):
    mask = np.uint64((1 << half) - 1)
    y = np.asarray(y, dtype=np.uint64)
    L, R = y >> np.uint64(half), y & mask
    for t in reversed(range(FEISTEL_ROUNDS)):
        L, R = R ^ _round_fn(t, L, tag, key, mask), L
    return (L << np.uint64(half)) | R


def permutation(a, N, tag, key):
    """pi(a) for positions a in [0, N): encrypt, re-encrypt while >= N."""
    half = feistel_half_bits(N)
    y = feistel_encrypt(a, half, tag, key)
    out = np.asarray(y).copy()
    todo = out >= N
    while np.any(todo):
        out[todo] = feistel_encrypt(out[todo], half, tag, key)
        todo = out >= N
    return out.astype(np.int64)


def permutation_inverse(i, N, tag, key):
    """pi^{-1}(i) for indices i in [0, N)."""
    half = feistel_half_bits(N)
    out = np.asarray(feistel_decrypt(i, half, tag, key)).copy()
    todo = out >= N
    while np.any(todo):
        out[todo] = feistel_decrypt(out[todo], half, tag, key)
        todo = out >= N
    return out.astype(np.int64)


# ----------------------------------------------------------------------------
# Givens stages (section 4 and 4.2)
# ----------------------------------------------------------------------------
def stage_pairs(perm, t):
    """(first, second) index arrays of the N/2 rotations of stage t >= 1."""
    N = len(perm)
    k = np.arange(N // 2)
    if t % 2 == 1:          # adjacent positions (2k, 2k+1)
        return perm[2 * k], perm[2 * k + 1]
    return perm[2 * k + 1], perm[(2 * k + 2) % N]   # shifted, cyclic


def stage_angles(side, t, npairs, key):
    """(c, s) = (cos theta, sin theta), theta uniform on [0, 2 pi).

    Rotation k of stage t on ``side`` draws attempt a = 0, 1, ... from
    Philox counter (k, a, TAG_ANGLE|side, t): U, V uniform on [-1, 1) from
    words (0,1) and (2,3); the first attempt with 0 < U*U + V*V <= 1 gives
    c = U/r, s = V/r, r = sqrt(U*U + V*V) (uniform direction in the disc).
    Only IEEE-exact operations are used, so the values are reproducible.
    """
    return stage_angles_at(side, t, np.arange(npairs, dtype=np.int64), key)


def stage_angles_at(side, t, pairs, key):
    """(c, s) of the rotations ``pairs`` (pair indices k) of stage t, drawn
    as in ``stage_angles`` (each rotation's draws depend on k only)."""
    pairs = np.asarray(pairs, dtype=np.int64)
    c = np.full(pairs.size, np.nan)
    s = np.full(pairs.size, np.nan)
    pending = np.arange(pairs.size, dtype=np.int64)
    for a in range(ANGLE_MAX_ATTEMPTS):
        if pending.size == 0:
            break
        w0, w1, w2, w3 = philox4x32_10(pairs[pending], a, TAG_ANGLE | side, t, key)
        U = 2.0 * unit_double(w0, w1) - 1.0
        V = 2.0 * unit_double(w2, w3) - 1.0
        q = U * U + V * V
        ok = (q > 0.0) & (q <= 1.0)
        r = np.sqrt(q[ok])
        c[pending[ok]] = U[ok] / r
        s[pending[ok]] = V[ok] / r
        pending = pending[~ok]
    c[pending] = 1.0
    s[pending] = 0.0
    return c, s


def sigma_values(n, kappa):
    """sigma_j = kappa^(-(j-1)/(n-1)), j = 1..n (0-based j here)."""
    j = np.arange(n, dtype=np.float64)
    return np.power(float(kappa), -(j / float(n - 1)))


def rotate(z, first, second, c, s, transpose=False):
    """Apply all rotations G(i, j, theta) of one stage to z (in place).

    G(i, j, theta) maps (z_i, z_j) to (c z_i - s z_j, s z_i + c z_j)
    (section 4); its transpose maps them to (c z_i + s z_j, -s z_i + c z_j).
    The pairs of a stage are disjoint, so the rotations commute.
    """
    zi = z[first].copy()
    zj = z[second].copy()
    if transpose:
        z[first] = c * zi + s * zj
        z[second] = -s * zi + c * zj
    else:
        z[first] = c * zi - s * zj
        z[second] = s * zi + c * zj
    return z


class Stage:
    def __init__(self, first, second, c, s):
        self.first, self.second, self.c, self.s = first, second, c, s


class Instance:
    """One generated instance (all arrays FP64 / int64, 0-based indices)."""

    def __init__(self, m, n, kappa, s, tau, seed, rounds=1):
        if not (n >= 2 and m >= n and m % 2 == 0 and n % 2 == 0):
            raise ValueError("need m >= n >= 2, m and n even")
        if not (0 <= s <= n) or not kappa >= 1.0 or not tau > 0.0:
            raise ValueError("need 0 <= s <= n, kappa >= 1, tau > 0")
        if rounds < 1:
            raise ValueError("rounds >= 1")
        self.m, self.n, self.kappa, self.s = int(m), int(n), float(kappa), int(s)
        self.tau, self.seed, self.rounds = float(tau), int(seed), int(rounds)
        key = seed_key(seed)
        self.key = key
        self.perm_n = permutation(np.arange(n), n, TAG_PERM | SIDE_N, key)
        self.perm_m = permutation(np.arange(m), m, TAG_PERM | SIDE_M, key)
        self.G_stages = []
        self.Q_stages = []
        for t in range(1, rounds + 1):
            f, g = stage_pairs(self.perm_n, t)
            c, sn = stage_angles(SIDE_N, t, n // 2, key)
            self.G_stages.append(Stage(f, g, c, sn))
            f, g = stage_pairs(self.perm_m, t)
            c, sn = stage_angles(SIDE_M, t, m // 2, key)
            self.Q_stages.append(Stage(f, g, c, sn))
        self.sigma = sigma_values(n, kappa)
        self.L = float(np.max(self.sigma) ** 2)
        self._make_solution(key)

    # -- operator products: Algorithms MvPA and MvPAt (section 4) ----------
    def apply_Gt(self, x):
        z = np.array(x, dtype=np.float64, copy=True)
        for st in reversed(self.G_stages):      # G^T = S_1^T ... S_r^T
            rotate(z, st.first, st.second, st.c, st.s, transpose=True)
        return z

    def apply_G(self, x):
        z = np.array(x, dtype=np.float64, copy=True)
        for st in self.G_stages:                # G = S_r ... S_1
            rotate(z, st.first, st.second, st.c, st.s)
        return z

    def apply_Q(self, z):
        z = np.array(z, dtype=np.float64, copy=True)
        for st in self.Q_stages:                # Q = S~_r ... S~_1
            rotate(z, st.first, st.second, st.c, st.s)
        return z

    def apply_Qt(self, y):
        z = np.array(y, dtype=np.float64, copy=True)
        for st in reversed(self.Q_stages):
            rotate(z, st.first, st.second, st.c, st.s, transpose=True)
        return z

    def matvec(self, x):
        """A x (Algorithm MvPA): G^T, then Sigma (n -> m), then Q."""
        w = self.apply_Gt(x)
        z = np.zeros(self.m)
        z[: self.n] = self.sigma * w
        return self.apply_Q(z)

    def rmatvec(self, y):
        """A^T y (Algorithm MvPAt): Q^T, then Sigma^T (m -> n), then G."""
        z = self.apply_Qt(y)
        return self.apply_G(self.sigma * z[: self.n])

    # -- Procedure OsGen-style x*, subgradient g, Procedure IGen ------------
    def _make_solution(self, key):
        n, s = self.n, self.s
        sup_perm_tag = TAG_PERM | SIDE_SUPPORT
        self.support = permutation(np.arange(s), n, sup_perm_tag, key)
        q = np.arange(s)
        w0, w1, w2, w3 = philox4x32_10(q, 0, TAG_XSTAR, 0, key)
        u1 = unit_double(w0, w1)
        u2 = unit_double(w2, w3)
        vals = np.sqrt(-2.0 * np.log(1.0 - u1)) * np.cos(2.0 * math.pi * u2)
        self.xstar = np.zeros(n)
        self.xstar[self.support] = vals
        w0, w1, _, _ = philox4x32_10(np.arange(n), 0, TAG_SUBGRAD, 0, key)
        g = 0.9 * (2.0 * unit_double(w0, w1) - 1.0)
        g[self.support] = np.sign(vals)
        self.g = g
        # IGen step 3 with the SVD-known inverse: e = tau Q Sigma^{+T} G^T g
        z = np.zeros(self.m)
        z[:n] = self.tau * self.apply_Gt(g) / self.sigma
        self.e = self.apply_Q(z)
        # IGen step 4
        self.b = self.matvec(self.xstar) + self.e
        self.fstar = self.tau * np.abs(self.xstar).sum() + 0.5 * self.e @ self.e

    # -- explicit matrices (tests and scipy-based products) ----------------
    @staticmethod
    def _stage_matrix(N, st, transpose=False):
        sgn = -1.0 if not transpose else 1.0
        rows = np.concatenate([st.first, st.first, st.second, st.second])
        cols = np.concatenate([st.first, st.second, st.first, st.second])
        vals = np.concatenate([st.c, sgn * st.s, -sgn * st.s, st.c])
        return sp.csr_matrix((vals, (rows, cols)), shape=(N, N))

    def sparse_A(self):
        """A = Q Sigma G^T as a scipy CSR matrix with sorted indices."""
        n, m = self.n, self.m
        Gt = sp.identity(n, format="csr")
        for st in self.G_stages:            # G^T = S_1^T S_2^T ... S_r^T
            Gt = Gt @ self._stage_matrix(n, st, transpose=True)
        Sig = sp.csr_matrix((self.sigma, (np.arange(n), np.arange(n))), shape=(m, n))
        Q = sp.identity(m, format="csr")
        for st in self.Q_stages:            # Q = S~_r ... S~_1
            Q = self._stage_matrix(m, st) @ Q
        A = (Q @ (Sig @ Gt)).tocsr()
        A.sort_indices()
        return A

    def dense_A(self):
        return self.sparse_A().toarray()


class IGen2Instance:
    """Procedure IGen2 (section 3.2): an instance with m < n.

    Inputs of the procedure and the readings taken here:
    * B (m x m, rank m) is the generator's square A = Q Sigma G^T (eq. (16)
      with n = m), one rotation stage per side; x* lies in its columns (the
      procedure's S within the first m components): support, values, g and
      e = tau B^{-T} g are those of ``Instance(m, m, ...)`` (step 3 with the
      SVD-known inverse, B^{-T} = Q Sigma^{-1} G^T).
    * N (m x (n - m)): column k is a copy of column p(k) of B, p injective,
      drawn among the columns j with |g_j| >= 1/2 (positions 0..n-m-1 of a
      random bijection of that list, tag TAG_IGEN2_PICK).  Then
      N_k^T e = tau g_p and the rescaled column of step 4,
      N~_k = xi_k tau / |N_k^T e| N_k, has scale |xi_k| / |g_p| <= 2;
      xi_k = 2u - 1 from counter (k, 0, TAG_IGEN2_XI, 0).
    * A = [B, N~], b = A x* + e = B x*_B + e (x* is zero on N~), and
      A^T e = tau g with g_{m+k} = xi_k sign(N_k^T e), so x* is optimal
      (eq. (15)); with |xi_k| < 1 the condition off S is strict and x* is
      the unique minimiser when B_S has full rank.
    * lambda_max(A A^T) = lambda_max(B (I + P D^2 P^T) B^T) <= 1 + max_k c_k^2
      (sigma_1 = 1, P D the placement and scales of N~): the L used here.
    """

    def __init__(self, m, n, kappa, s, tau, seed, rounds=1):
        if not (m >= 2 and m % 2 == 0 and n > m):
            raise ValueError("IGen2 needs n > m >= 2, m even")
        if rounds != 1:
            raise ValueError("IGen2 is built with one rotation stage per side")
        if not (0 <= s <= m):
            raise ValueError("need 0 <= s <= m")
        self.m, self.n, self.kappa, self.s = int(m), int(n), float(kappa), int(s)
        self.tau, self.seed, self.rounds = float(tau), int(seed), int(rounds)
        Bi = Instance(m, m, kappa, s, tau, seed, rounds=rounds)
        self.Bi = Bi
        key = Bi.key
        elig = np.flatnonzero(np.abs(Bi.g) >= 0.5)
        k = np.arange(n - m)
        if n - m > elig.size:
            raise ValueError("IGen2: n - m exceeds the columns of B eligible for N")
        self.p = elig[permutation(k, elig.size, TAG_IGEN2_PICK, key)]
        w0, w1, w2, w3 = philox4x32_10(k, 0, TAG_IGEN2_XI, 0, key)
        self.xi = 2.0 * unit_double(w0, w1) - 1.0
        B = Bi.sparse_A()
        Bc = B.tocsc()
        dots = (Bc.T @ Bi.e)[self.p]            # N_k^T e, k = 0 .. n-m-1
        self.c = self.xi * tau / np.abs(dots)
        self.N_tilde = (Bc[:, self.p] @ sp.diags(self.c)).tocsc()
        A = sp.hstack([B, self.N_tilde], format="csr")
        A.sort_indices()
        self._A = A
        self.support = Bi.support
        self.xstar = np.concatenate([Bi.xstar, np.zeros(n - m)])
        self.g = np.concatenate([Bi.g, self.xi * np.sign(dots)])
        self.e = Bi.e
        self.b = Bi.b
        self.fstar = Bi.fstar
        self.L = float(1.0 + np.max(self.c ** 2)) if n > m else 1.0

    def sparse_A(self):
        return self._A.copy()

    def dense_A(self):
        return self._A.toarray()

    def matvec(self, x):
        return self._A @ x

    def rmatvec(self, y):
        return self._A.T @ y


class LocalInstance:
    """The instance of ``Instance(m, n, kappa, s, tau, seed, rounds)``
    evaluated at chosen indices only, for sizes where the O(n) arrays of
    ``Instance`` are too large to build in a test (n = 2^26).

    Every quantity is computed from the same definitions and draws:
    the bijections and angles (sections 4 and 4.2) at the positions and pairs
    that are touched, A's columns A e_j = Q Sigma G^T e_j and rows
    A^T e_i = G Sigma^T Q^T e_i by Algorithms MvPA / MvPAt applied to sparse
    vectors (a stage rotates only the pairs that hold an entry), and b_i of
    Procedure IGen (section 3.1): (A x*)_i + e_i with
    e_i = tau sum_k Q[i, k] (G^T g)_k / sigma_k over k < n (step 3 with the
    SVD-known inverse of section 4).  Entries that land on the same index
    are summed, so floating-point values agree with ``Instance`` up to the
    order of the additions.

    A batch of sparse vectors is kept as parallel arrays (owner, index,
    value); ``owner`` says which vector of the batch an entry belongs to.
    """

    def __init__(self, m, n, kappa, s, tau, seed, rounds=1):
        if not (n >= 2 and m >= n and m % 2 == 0 and n % 2 == 0):
            raise ValueError("need m >= n >= 2, m and n even")
        self.m, self.n, self.kappa, self.s = int(m), int(n), float(kappa), int(s)
        self.tau, self.seed, self.rounds = float(tau), int(seed), int(rounds)
        self.key = seed_key(seed)

    def _N(self, side):
        return self.n if side == SIDE_N else self.m

    def position(self, side, i):
        """pi^{-1}(i): the position of index i on ``side``."""
        return permutation_inverse(np.asarray(i, dtype=np.int64), self._N(side), TAG_PERM | side, self.key)

    def index(self, side, p):
        """pi(p): the index at position p on ``side``."""
        return permutation(np.asarray(p, dtype=np.int64), self._N(side), TAG_PERM | side, self.key)

    def sigma(self, j):
        """sigma_j = kappa^(-(j-1)/(n-1)) (0-based j), as ``sigma_values``."""
        j = np.asarray(j, dtype=np.float64)
        return np.power(self.kappa, -(j / float(self.n - 1)))

    def _stage(self, side, t, owner, idx, val, transpose):
        """Stage t of ``side`` (or its transpose) applied to a batch of sparse
        vectors.  Odd t pairs positions (2k, 2k+1), even t (2k+1, 2k+2 mod N);
        G(f, g, theta) maps (z_f, z_g) to (c z_f - s z_g, s z_f + c z_g)."""
        N = self._N(side)
        a = self.position(side, idx)
        if t % 2 == 1:
            f = a - (a & 1)
        else:
            f = np.where(a & 1, a, (a - 1) % N)
        g = (f + 1) % N
        k = f // 2
        first = a == f
        c, s = stage_angles_at(side, t, k, self.key)
        partner = self.index(side, np.where(first, g, f))
        # z at f feeds (c, s) to (f, g); z at g feeds (-s, c); the transpose
        # swaps the signs of s
        sgn = np.where(first, 1.0, -1.0) * (-1.0 if transpose else 1.0)
        owner2 = np.concatenate([owner, owner])
        idx2 = np.concatenate([idx, partner])
        val2 = np.concatenate([c * val, sgn * s * val])
        return self._combine(owner2, idx2, val2)

    @staticmethod
    def _combine(owner, idx, val):
        key = owner.astype(np.int64) * (1 << 34) + idx.astype(np.int64)
        uk, inv = np.unique(key, return_inverse=True)
        out = np.zeros(uk.size)
        np.add.at(out, inv, val)
        return uk >> 34, uk & ((1 << 34) - 1), out

    def columns(self, js):
        """A e_j for each j in ``js``: (owner, row index, value) sorted."""
        js = np.asarray(js, dtype=np.int64)
        o, i, v = np.arange(js.size), js.copy(), np.ones(js.size)
        for t in range(self.rounds, 0, -1):          # G^T = S_1^T ... S_r^T
            o, i, v = self._stage(SIDE_N, t, o, i, v, transpose=True)
        v = v * self.sigma(i)                         # Sigma: index i of R^n -> i of R^m
        for t in range(1, self.rounds + 1):           # Q = S~_r ... S~_1
            o, i, v = self._stage(SIDE_M, t, o, i, v, transpose=False)
        return o, i, v

    def rows(self, rs):
        """A^T e_i for each i in ``rs``: (owner, column index, value) sorted."""
        rs = np.asarray(rs, dtype=np.int64)
        o, i, v = np.arange(rs.size), rs.copy(), np.ones(rs.size)
        for t in range(self.rounds, 0, -1):          # Q^T
            o, i, v = self._stage(SIDE_M, t, o, i, v, transpose=True)
        keep = i < self.n                             # Sigma^T drops indices >= n
        o, i, v = o[keep], i[keep], v[keep] * self.sigma(i[keep])
        for t in range(1, self.rounds + 1):           # G
            o, i, v = self._stage(SIDE_N, t, o, i, v, transpose=False)
        return o, i, v

    def xstar(self, js):
        """x*_j: N(0,1) (Box-Muller) at support rank q if pi_sup^{-1}(j) < s."""
        js = np.asarray(js, dtype=np.int64)
        q = permutation_inverse(js, self.n, TAG_PERM | SIDE_SUPPORT, self.key)
        w0, w1, w2, w3 = philox4x32_10(q, 0, TAG_XSTAR, 0, self.key)
        u1 = unit_double(w0, w1)
        u2 = unit_double(w2, w3)
        vals = np.sqrt(-2.0 * np.log(1.0 - u1)) * np.cos(2.0 * math.pi * u2)
        return np.where(q < self.s, vals, 0.0)

    def subgradient(self, js):
        """g_j: sign(x*_j) on the support, 0.9 (2u - 1) off it (eq. (10))."""
        js = np.asarray(js, dtype=np.int64)
        w0, w1, _, _ = philox4x32_10(js, 0, TAG_SUBGRAD, 0, self.key)
        g = 0.9 * (2.0 * unit_double(w0, w1) - 1.0)
        q = permutation_inverse(js, self.n, TAG_PERM | SIDE_SUPPORT, self.key)
        xs = self.xstar(js)
        return np.where(q < self.s, np.sign(xs), g)

    def e(self, rs):
        """e_i = tau (Q Sigma^{+T} G^T g)_i (IGen step 3)."""
        rs = np.asarray(rs, dtype=np.int64)
        o, k, q = np.arange(rs.size), rs.copy(), np.ones(rs.size)
        for t in range(self.rounds, 0, -1):          # row i of Q: Q^T e_i
            o, k, q = self._stage(SIDE_M, t, o, k, q, transpose=True)
        keep = k < self.n
        o, k, q = o[keep], k[keep], q[keep]
        # (G^T g)_k = (G e_k)^T g
        oo, l, gv = np.arange(k.size), k.copy(), np.ones(k.size)
        for t in range(1, self.rounds + 1):
            oo, l, gv = self._stage(SIDE_N, t, oo, l, gv, transpose=False)
        gtg = np.zeros(k.size)
        np.add.at(gtg, oo, gv * self.subgradient(l))
        out = np.zeros(rs.size)
        np.add.at(out, o, q * (self.tau * gtg / self.sigma(k)))
        return out

    def b(self, rs):
        """b_i = (A x*)_i + e_i (IGen step 4)."""
        rs = np.asarray(rs, dtype=np.int64)
        o, j, a = self.rows(rs)
        ax = np.zeros(rs.size)
        np.add.at(ax, o, a * self.xstar(j))
        return ax + self.e(rs)


def objective(A_mv, b, tau, x):
    """f_tau(x) of problem (1); A_mv is a callable x -> A x."""
    r = A_mv(x) - b
    return tau * np.abs(x).sum() + 0.5 * r @ r


def default_s(n, divisor):
    """Support size of the workloads: max(1, floor(n / divisor))."""
    return max(1, n // divisor)
