"""GPU parity of the blocked stored operator (runs of four stage positions,
L1LS_STORE_BLK32 / L1LS_OP_BLOCKED) against the CPU oracle.

The blocked form stores A = sum_i sigma_i (Q e_i)(G e_i)^T term by term in
FP32 (two Givens stages, eq. (16)), so its products carry one FP32 rounding
per stored value plus the FP32 sums, like the FP32 CSR/CSC: the tolerances
are those of the FP32 stored operator.
"""
import ctypes

import numpy as np
import pytest
import scipy.sparse as sp

torch = pytest.importorskip("torch")

import paper_1503_03520_amd as L  # noqa: E402
import seeded_inputs as SI  # noqa: E402
from fp32_bounds import fp32_trajectory_bound  # noqa: E402
from oracle import fista as F  # noqa: E402
from oracle import instance as OI  # noqa: E402

pytestmark = pytest.mark.gpu

STORE_ALL = L.STORE_F32 | L.STORE_F64 | L.STORE_BLK32

# (m, n, kappa, s, tau, seed): two stages throughout.  Ragged with respect to
# the 64-row tiles and 256-column workgroups, square (every row holds four
# runs, so row tiles exceed the branch-free rounds), the smallest sizes the
# runs allow (n = 4: the four positions of a run are the whole side) and a
# case spanning many tiles.
CASES = [
    (1010, 502, 1e3, 7, 0.5, 17),
    (1000, 1000, 1e2, 9, 1.0, 21),
    (4, 4, 3.0, 1, 1.0, 5),
    (6, 4, 10.0, 2, 2.0, 6),
    (600, 300, 1.0, 5, 1.0, 8),
    (8192, 4096, 1e4, 41, 1.0, 1503035201),
    (130, 4, 10.0, 1, 1.0, 12),        # m >> n: most rows hold no run at all
]
# the FP64 workload's sizes and conditioning with two stages
C1_TWO_STAGES = (2048, 1024, 1e2, 10, 1.0, 1503035200)

_cache = {}


def pair(cfg):
    if cfg not in _cache:
        m, n, kappa, s, tau, seed = cfg
        print(f"\n[case] blocked m={m} n={n} kappa={kappa} s={s} tau={tau} seed={seed}", flush=True)
        g = L.l1ls_generate(m, n, kappa, s, tau, seed, rounds=2, storage=STORE_ALL)
        o = OI.Instance(m, n, kappa, s, tau, seed, rounds=2)
        _cache[cfg] = (g, o, o.sparse_A())
    return _cache[cfg]


def term_magnitudes(o):
    """sum_i sigma_i |Q e_i| |G e_i|^T = |Q| Sigma |G|^T: the sum of the
    magnitudes of the terms that make up each entry of A.  With two stages
    every entry of Q (and of G) is a single product of stage coefficients
    (a stage-2 pair meets a stage-1 pair in one position), so |Q| is the
    product of the stages' magnitudes."""
    Gt = sp.identity(o.n, format="csr")
    for st in o.G_stages:
        Gt = Gt @ abs(OI.Instance._stage_matrix(o.n, st, transpose=True))
    Q = sp.identity(o.m, format="csr")
    for st in o.Q_stages:
        Q = abs(OI.Instance._stage_matrix(o.m, st)) @ Q
    Sig = sp.csr_matrix((o.sigma, (np.arange(o.n), np.arange(o.n))), shape=(o.m, o.n))
    return (Q @ (Sig @ Gt)).tocsr()


def _dev(v, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(v), dtype=dtype, device="cuda")


def _apply(g, trans, v, size, op=L.OP_BLOCKED):
    out = torch.empty(size, dtype=torch.float32, device="cuda")
    L.l1ls_apply(g, trans, op, L.F32, _dev(v, torch.float32), out)
    torch.cuda.synchronize()
    return out.double().cpu().numpy()


@pytest.mark.parametrize("cfg", CASES)
def test_blocked_products_match_oracle(cfg):
    g, o, A = pair(cfg)
    x = SI.normal_vector(o.n, 201)
    y = SI.normal_vector(o.m, 202)
    ax, aty = o.matvec(x), o.rmatvec(y)
    xr = x.astype(np.float32).astype(np.float64)
    yr = y.astype(np.float32).astype(np.float64)
    # On the FP32-rounded inputs: one rounding per stored term value, one per
    # product and at most 8 additions deep (4 within a run, 4 runs), so
    # |err| <= 10 eps32 sum_terms |term| |x_j|; 20 leaves room.
    T = term_magnitudes(o)
    eps = np.finfo(np.float32).eps
    bx = 20 * eps * (T @ np.abs(xr)) + 1e-30
    by = 20 * eps * (T.T @ np.abs(yr)) + 1e-30
    assert np.all(np.abs(_apply(g, 0, x, o.m) - A @ xr) <= bx)
    assert np.all(np.abs(_apply(g, 1, y, o.n) - A.T @ yr) <= by)
    # and against the oracle's rotations on the unrounded vectors
    assert np.abs(_apply(g, 0, x, o.m) - ax).max() <= 2e-6 * max(1.0, np.abs(ax).max())
    assert np.abs(_apply(g, 1, y, o.n) - aty).max() <= 2e-6 * max(1.0, np.abs(aty).max())


@pytest.mark.parametrize("cfg", [c for c in CASES if c[1] <= 1000])
def test_blocked_rows_and_columns_store_the_same_matrix(cfg):
    # A e_j through the row runs and A^T e_i through the column runs give
    # columns and rows of A; both equal the oracle's A to the FP32 rounding
    # of each term (and of the sums of terms that share an entry).
    g, o, A = pair(cfg)
    Ad = A.toarray()
    Td = term_magnitudes(o).toarray()
    by_rows = np.stack([_apply(g, 0, np.eye(o.n)[j], o.m) for j in range(min(o.n, 64))], axis=1)
    by_cols = np.stack([_apply(g, 1, np.eye(o.m)[i], o.n) for i in range(min(o.m, 64))], axis=0)
    eps = np.finfo(np.float32).eps
    k, c = by_cols.shape[0], by_rows.shape[1]
    assert np.all(np.abs(by_rows - Ad[:, :c]) <= 4 * eps * Td[:, :c])
    assert np.all(np.abs(by_cols - Ad[:k, :]) <= 4 * eps * Td[:k, :])
    assert np.all(np.abs(by_rows[:k, :] - by_cols[:, :c]) <= 8 * eps * Td[:k, :c])
    # the sparsity pattern is A's: no entry outside the runs' coverage
    assert np.all(by_rows[Td[:, :c] == 0] == 0) and np.all(by_cols[Td[:k, :] == 0] == 0)


@pytest.mark.parametrize("cfg", CASES)
def test_blocked_fista_trajectory_fp32(cfg):
    # The bound of the FP32 stored path (tests/fp32_bounds.py): the blocked
    # values are rounded once per term instead of once per entry, the same
    # order of perturbation.
    g, o, A = pair(cfg)
    iters = 50
    ref, bound = fp32_trajectory_bound(A, o.b, o.tau, 1.0, iters)
    x, rep, _ = L.l1ls_solve_fista(g, max_iter=iters, rel_gap_tol=0.0, check_every=5, precision=L.F32,
                                   op=L.OP_BLOCKED)
    assert np.abs(x.cpu().numpy() - ref).max() <= bound
    xs, _, _ = L.l1ls_solve_fista(g, max_iter=iters, rel_gap_tol=0.0, check_every=5, precision=L.F32)
    assert np.abs(x.cpu().numpy() - xs.cpu().numpy()).max() <= 2 * bound


@pytest.mark.parametrize("cfg", CASES)
def test_blocked_device_gap_matches_oracle_at_its_iterate(cfg):
    # The FP32 passes' FP64 statistics give P and D at the iterate they
    # produce; the oracle's objective at that iterate agrees to the FP32
    # rounding of r_x (relative eps32-scale terms of ||r||^2 and ||x||_1).
    g, o, A = pair(cfg)
    k = 40
    fs = L.Fista(g, rel_gap_tol=0.0, check_every=k, precision=L.F32, op=L.OP_BLOCKED)
    fs.iterate(k)
    rep = fs.report()
    x = fs.get_x().cpu().numpy()
    fs.destroy()
    r = A @ x - o.b
    P = o.tau * np.abs(x).sum() + 0.5 * r @ r
    assert abs(rep["primal"] - P) <= 1e-5 * max(1.0, abs(P))


def test_blocked_stepping_and_repeat_are_bitwise():
    g, o, A = pair(CASES[0])
    a, _, _ = L.l1ls_solve_fista(g, max_iter=64, rel_gap_tol=0.0, check_every=16, precision=L.F32, op=L.OP_BLOCKED)
    b, _, _ = L.l1ls_solve_fista(g, max_iter=64, rel_gap_tol=0.0, check_every=16, precision=L.F32, op=L.OP_BLOCKED)
    fs = L.Fista(g, rel_gap_tol=0.0, check_every=16, precision=L.F32, op=L.OP_BLOCKED)
    for _ in range(4):
        fs.iterate(16)
    c = fs.get_x()
    fs.destroy()
    assert torch.equal(a, b) and torch.equal(a, c)


def test_blocked_warm_start_stays_at_the_planted_solution():
    # x* is optimal, so FISTA from x* moves only by the FP32 gradient
    # rounding (the trajectory bound above, started from x*)
    g, o, A = pair(CASES[0])
    iters = 10
    x, rep, _ = L.l1ls_solve_fista(g, x0=_dev(o.xstar), max_iter=iters, rel_gap_tol=0.0, check_every=1,
                                   precision=L.F32, op=L.OP_BLOCKED)
    _, bound = fp32_trajectory_bound(A, o.b, o.tau, 1.0, iters, x_ref=o.xstar, x0=o.xstar)
    assert np.abs(x.cpu().numpy() - o.xstar).max() <= bound


def test_blocked_fp32_then_polish_recovers_planted():
    g, o, A = pair(C1_TWO_STAGES)
    x, rep, _ = L.l1ls_solve_fista(g, max_iter=3000, rel_gap_tol=1e-7, check_every=32, precision=L.F32,
                                   op=L.OP_BLOCKED, polish=1)
    err = np.linalg.norm(x.cpu().numpy() - o.xstar) / np.linalg.norm(o.xstar)
    assert err <= 1e-10 and abs(rep["rel_gap"]) <= 1e-12


def test_blocked_requires_its_storage_and_fp32():
    g = L.l1ls_generate(600, 300, 1.0, 5, 1.0, 8, rounds=2)   # CSR/CSC only
    out = torch.empty(600, dtype=torch.float32, device="cuda")
    x = torch.zeros(300, dtype=torch.float32, device="cuda")
    st = L.lib().l1ls_apply(g.handle, 0, L.OP_BLOCKED, L.F32, L._ptr(x), L._ptr(out), L._stream(None))
    assert st == -6
    o = L.solve_opts(precision=L.F32, op=L.OP_BLOCKED)
    h = ctypes.c_void_p()
    assert L.lib().l1ls_fista_create(g.handle, ctypes.byref(o), ctypes.byref(h)) == -6
    gb, _, _ = pair(CASES[0])
    o = L.solve_opts(precision=L.F64, op=L.OP_BLOCKED)
    assert L.lib().l1ls_fista_create(gb.handle, ctypes.byref(o), ctypes.byref(h)) == -6
