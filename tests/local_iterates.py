"""The second FISTA iterate at sampled columns from the oracle's sampled
form (``oracle.instance.LocalInstance``), with an a-priori bound on the
error of an FP32 computation of it.

FISTA (section 8.1) from x_0 = 0 with t_1 = 1 has beta_1 = 0, so y_2 = x_1
and, with L = 1 (sigma_1^2 = 1 for the generator's A),

    x_1 = soft(A^T b, tau),   x_2 = soft(x_1 - A^T (A x_1 - b), tau).

x_2 at columns J needs A's rows touching J, every column of those rows
(x_1 there) and b at the rows of those columns: a two-hop neighbourhood
that the sampled form evaluates without building A.

Bound (FP32 values of A and b, FP32 products, sums and iterates, each sum
of at most 16 + 1 terms, u = eps32 / 2):
  - x_1: |x_1' - x_1| <= d_c = 20 eps32 sum_r |a_rc b_r|;
  - r' = A' x_1' - b': |r' - r| <= sum_c |a_rc| d_c + 10 eps32 (|A| |x_1| + |b|)_r;
  - g' = A'^T r': |g' - g| <= (|A|^T |A| d)_j + 20 eps32 (|A|^T (|A| |x_1| + |b|))_j;
  - z = x_1 - g and soft() is 1-Lipschitz, one more rounding of z.
The bound used is d_j + (|A|^T |A| d)_j + 40 eps32 ((|A|^T (|A| |x_1| + |b|))_j
+ |x_1|_j): twice the rounding terms above.
"""
import numpy as np

from oracle import instance as OI

EPS32 = float(np.finfo(np.float32).eps)


def soft(z, tau):
    return np.sign(z) * np.maximum(np.abs(z) - tau, 0.0)


def second_iterate(loc, js):
    """(x_2 at js in FP64, the FP32 error bound at js)."""
    js = np.asarray(js)
    o, ri, rv = loc.columns(js)
    rows = np.unique(ri)
    ro, rc, rval = loc.rows(rows)
    cols = np.union1d(np.unique(rc), js)
    co, cri, crv = loc.columns(cols)
    cb = loc.b(cri)
    atb = np.zeros(cols.size)
    mag = np.zeros(cols.size)
    np.add.at(atb, co, crv * cb)
    np.add.at(mag, co, np.abs(crv * cb))
    x1 = soft(atb, loc.tau)
    d1 = 20 * EPS32 * mag
    at_c = np.searchsorted(cols, rc)
    ax = np.zeros(rows.size)
    axm = np.zeros(rows.size)
    ad = np.zeros(rows.size)
    np.add.at(ax, ro, rval * x1[at_c])
    np.add.at(axm, ro, np.abs(rval * x1[at_c]))
    np.add.at(ad, ro, np.abs(rval) * d1[at_c])
    bv = loc.b(rows)
    res = ax - bv
    at_r = np.searchsorted(rows, ri)
    g = np.zeros(js.size)
    gm = np.zeros(js.size)
    gd = np.zeros(js.size)
    np.add.at(g, o, rv * res[at_r])
    np.add.at(gm, o, np.abs(rv) * (axm[at_r] + np.abs(bv[at_r])))
    np.add.at(gd, o, np.abs(rv) * ad[at_r])
    at_j = np.searchsorted(cols, js)
    x1j, d1j = x1[at_j], d1[at_j]
    x2 = soft(x1j - g, loc.tau)
    bound = d1j + gd + 40 * EPS32 * (gm + np.abs(x1j)) + 1e-30
    return x2, bound


def informative_columns(loc, count, seed, candidates=4096, support=16):
    """Columns where the early iterates are not all zero: the `count`
    largest |A^T b| among random candidates, and sampled support columns."""
    rng = np.random.default_rng(seed)
    cand = np.unique(rng.integers(0, loc.n, candidates))
    o, ri, rv = loc.columns(cand)
    atb = np.zeros(cand.size)
    np.add.at(atb, o, rv * loc.b(ri))
    big = cand[np.argsort(-np.abs(atb))[:count]]
    sup = OI.permutation(np.arange(loc.s), loc.n, OI.TAG_PERM | OI.SIDE_SUPPORT, loc.key)
    pick = rng.choice(sup, min(support, sup.size), replace=False) if sup.size else sup
    return np.unique(np.concatenate([big, pick, rng.integers(0, loc.n, count)]))
