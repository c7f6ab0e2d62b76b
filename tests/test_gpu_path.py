"""Regularisation path (64 tau values as one sparse-times-dense iteration).

Each column is FISTA at its own tau on the shared instance; it is compared
with the oracle's FP64 FISTA at the same tau and iteration count (the FP32
bound of tests/fp32_bounds.py), the path endpoint tau >= ||A^T b||_inf gives x = 0,
and columns solved to tolerance carry FP64 certificates.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1503_03520_amd as L  # noqa: E402
from fp32_bounds import fp32_trajectory_bound  # noqa: E402
from oracle import fista as F  # noqa: E402
from oracle import instance as OI  # noqa: E402

pytestmark = pytest.mark.gpu

CFG = (8192, 4096, 1e3, 40, 1.0, 1503035203, 2)
_c = {}


def pair():
    if "p" not in _c:
        m, n, kappa, s, tau, seed, r = CFG
        print(f"\n[case] path instance m={m} n={n} kappa={kappa} seed={seed}", flush=True)
        g = L.l1ls_generate(m, n, kappa, s, tau, seed, rounds=r)
        o = OI.Instance(m, n, kappa, s, tau, seed, rounds=r)
        _c["p"] = (g, o, o.sparse_A())
    return _c["p"]


def taus_for(o, A, k):
    tmax = float(np.abs(A.T @ o.b).max())
    return np.geomspace(1e-3, 1.0, k) * tmax, tmax


@pytest.mark.parametrize("k", [64, 7])
def test_path_columns_match_oracle(k):
    g, o, A = pair()
    taus, tmax = taus_for(o, A, k)
    iters = 30
    X, reps, _ = L.l1ls_solve_fista_path(g, taus, max_iter=iters, rel_gap_tol=0.0, check_every=10)
    Xh = X.cpu().numpy()
    for c in sorted({0, 1, k // 2, k - 1}):
        ref, bound = fp32_trajectory_bound(A, o.b, float(taus[c]), 1.0, iters)
        assert np.abs(Xh[c] - ref).max() <= bound, c
        assert reps[c]["iterations"] == iters


def test_path_endpoint_is_zero():
    g, o, A = pair()
    taus, tmax = taus_for(o, A, 64)
    X, reps, _ = L.l1ls_solve_fista_path(g, [tmax * 1.0001, tmax * 2.0], max_iter=50, rel_gap_tol=0.0,
                                         check_every=10)
    assert np.array_equal(X.cpu().numpy(), np.zeros((2, o.n)))


def test_path_to_tolerance_with_fp64_certificates():
    # kappa = 10: the oracle's FP64 FISTA reaches rel gap 1e-5 within 2000
    # iterations for every tau of geomspace(1e-3, 1, 16) * ||A^T b||_inf.
    # FP32 bulk has a floor: for small tau (good fits) FP32 FISTA stalls near
    # rel gap 2e-3 (an FP32 numpy run of the same iteration stalls at the same
    # level), which the FP64 polish is for.  Columns that report convergence
    # must carry an FP64 certificate <= 3e-5; the others stop at max_iter with
    # an FP64 gap below 5e-3; every tau >= 0.1 tau_max converges.
    m, n, kappa, s, tau, seed, r = (8192, 4096, 10.0, 40, 1.0, 1503035204, 2)
    g = L.l1ls_generate(m, n, kappa, s, tau, seed, rounds=r)
    o = OI.Instance(m, n, kappa, s, tau, seed, rounds=r)
    A = o.sparse_A()
    taus, tmax = taus_for(o, A, 16)
    X, reps, st = L.l1ls_solve_fista_path(g, taus, max_iter=6000, rel_gap_tol=1e-5, check_every=16)
    for c, tau in enumerate(taus):
        P, D, gap = L.l1ls_objective_gap(g, float(tau), X[c].contiguous())
        print(c, tau / tmax, reps[c]["iterations"], reps[c]["rel_gap"], gap)
        if reps[c]["converged"] == 1:
            assert gap <= 3e-5, (c, gap)
        else:
            # stalled at the FP32 floor: both gaps above the tolerance, bounded
            assert reps[c]["rel_gap"] > 1e-5 and gap <= 5e-3, (c, reps[c]["rel_gap"], gap)
        if tau >= 0.1 * tmax:
            assert reps[c]["converged"] == 1 and reps[c]["iterations"] <= 4000


def test_path_fp64_finish_reports_fp64_certificates():
    # polish = 2: each column's FP32 result is finished in FP64 at its own
    # tau (the polish of the reduced problem (13) runs where the FP64 gap
    # misses the tolerance), and each report carries the FP64 gap of the
    # returned column.  The polish starts from the FP32 iterate's support, so
    # after 300 iterations at kappa = 1e3 it certifies only some columns;
    # what is checked is that every report tells the truth.
    g, o, A = pair()
    taus, tmax = taus_for(o, A, 16)
    taus = np.concatenate([taus, [o.tau]])
    kw = dict(max_iter=300, rel_gap_tol=1e-8, check_every=10)
    X32, r32, _ = L.l1ls_solve_fista_path(g, taus, **kw)
    X, reps, st = L.l1ls_solve_fista_path(g, taus, polish=2, **kw)
    done = 0
    for c, t in enumerate(taus):
        P, D, gap = L.l1ls_objective_gap(g, float(t), X[c].contiguous())
        assert reps[c]["rel_gap"] == gap, c
        assert reps[c]["converged"] == (1 if gap <= 1e-8 else 0), c
        P32, _, g32 = L.l1ls_objective_gap(g, float(t), X32[c].contiguous())
        if g32 <= 1e-8:
            assert torch.equal(X[c], X32[c]) and reps[c]["polish_rounds"] == 0, c   # nothing to finish
        else:
            assert reps[c]["polish_rounds"] >= 1, c
        # the finish never returns a column with a larger objective f_tau
        # (a polish that does not improve leaves the FP32 column)
        assert P <= P32 * (1 + 1e-12), (c, P, P32)
        done += reps[c]["converged"]
    print(f"FP64-finished columns within 1e-8: {done} of {len(taus)}", flush=True)
    assert reps[-1]["converged"] == 1
    assert (st == L.L1LS_OK) == (done == len(taus))


def test_path_polish_every_column_reaches_planted_solution():
    # polish = 1 polishes every column: at the planted tau the FP32 path's
    # column, finished in FP64, is x* (Procedure IGen) to the FP64 floor, as
    # the single-instance solve with polish = 1 from the same iterations
    g, o, A = pair()
    taus = np.array([o.tau, 0.5 * o.tau])
    X, reps, _ = L.l1ls_solve_fista_path(g, taus, max_iter=300, rel_gap_tol=1e-8, check_every=10, polish=1)
    assert reps[0]["polish_rounds"] >= 1 and reps[1]["polish_rounds"] >= 1
    err = np.linalg.norm(X[0].cpu().numpy() - o.xstar) / np.linalg.norm(o.xstar)
    x1, r1, _ = L.l1ls_solve_fista(g, max_iter=300, rel_gap_tol=1e-8, check_every=10, precision=L.F32, polish=1)
    err1 = np.linalg.norm(x1.cpu().numpy() - o.xstar) / np.linalg.norm(o.xstar)
    print(f"planted tau: path polish rel err {err:.3e}, single solve {err1:.3e}", flush=True)
    assert reps[0]["converged"] == 1 and err <= 1e-9
    assert err1 <= 1e-9
    for c in range(2):
        assert reps[c]["rel_gap"] == L.l1ls_objective_gap(g, float(taus[c]), X[c].contiguous())[2]
