"""FISTA in one workgroup (small FP64 instances whose stored operator and
iterates fit in one compute unit's LDS): l1ls_solve_fista takes that path
by itself; it must produce the multi-kernel iteration bit for bit (the
stepping interface always runs the multi-kernel passes), stop at the same
gap check, and match the oracle.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1503_03520_amd as L  # noqa: E402
from oracle import fista as F  # noqa: E402
from oracle import instance as OI  # noqa: E402

pytestmark = pytest.mark.gpu

# (m, n, kappa, s, tau, seed, rounds): all fit in 160 KB (FP64 CSR + CSC,
# two x slots, r_y): the FP64 workload (n = 1024, one stage), two-stage,
# tiny, square, s = 0, and m spanning more than one row per thread
FITS = [
    (2048, 1024, 1e2, 10, 1.0, 1503035200, 1),
    (600, 300, 1.0, 5, 1.0, 8, 2),
    (4, 2, 3.0, 1, 1.0, 5, 1),
    (6, 6, 10.0, 2, 2.0, 6, 2),
    (512, 256, 1e4, 0, 1.0, 9, 2),
    (3000, 600, 1e3, 6, 0.5, 31, 1),
]

_cache = {}


def pair(cfg):
    if cfg not in _cache:
        m, n, kappa, s, tau, seed, r = cfg
        print(f"\n[case] on-chip m={m} n={n} kappa={kappa} s={s} tau={tau} seed={seed} rounds={r}", flush=True)
        g = L.l1ls_generate(m, n, kappa, s, tau, seed, rounds=r)
        _cache[cfg] = g
    return _cache[cfg]


def _stepping(g, iters, check, tol=0.0):
    fs = L.Fista(g, precision=L.F64, rel_gap_tol=tol, check_every=check, max_iter=iters)
    fs.iterate(iters)
    rep = fs.report()
    x = fs.get_x()
    fs.destroy()
    return x, rep


@pytest.mark.parametrize("cfg", FITS)
@pytest.mark.parametrize("iters,check", [(1, 1), (2, 1), (37, 8), (200, 32)])
def test_onchip_equals_multikernel_bitwise(cfg, iters, check):
    g = pair(cfg)
    x, rep, _ = L.l1ls_solve_fista(g, max_iter=iters, rel_gap_tol=0.0, check_every=check, precision=L.F64)
    xs, rs = _stepping(g, iters, check)
    assert torch.equal(x, xs)
    assert rep["iterations"] == iters
    # the report's certificate is the FP64 gap at x (l1ls_objective_gap); its
    # primal value is the one the stepping run's device statistics give
    if iters % check == 0:
        assert math.isclose(rep["primal"], rs["primal"], rel_tol=1e-12)


@pytest.mark.parametrize("cfg", FITS[:2])
def test_onchip_stops_at_the_same_check_and_matches_the_oracle(cfg):
    g = pair(cfg)
    m, n, kappa, s, tau, seed, r = cfg
    x, rep, st = L.l1ls_solve_fista(g, max_iter=20000, rel_gap_tol=1e-10, check_every=32, precision=L.F64)
    assert st == L.L1LS_OK and rep["converged"] == 1
    fs = L.Fista(g, precision=L.F64, rel_gap_tol=1e-10, check_every=32)
    it = 0
    while it < 20000:
        fs.iterate(128)
        it += 128
        if fs.report()["converged"]:
            break
    rs = fs.report()
    xs = fs.get_x()
    fs.destroy()
    assert rs["converged"] == 1 and rs["iterations"] == rep["iterations"]
    assert torch.equal(x, xs)
    o = OI.Instance(m, n, kappa, s, tau, seed, rounds=r)
    A = o.sparse_A()
    ref = F.fista(lambda v: A @ v, lambda v: A.T @ v, o.b, o.tau, 1.0, rep["iterations"])
    assert np.abs(x.cpu().numpy() - ref).max() <= 1e-9 * max(1.0, np.abs(ref).max())


def test_onchip_final_gap_when_max_iter_is_not_a_check():
    # max_iter % check != 0: the gap is evaluated at the last iterate too,
    # and a tolerance met there counts as converged
    g = pair(FITS[0])
    x, rep, _ = L.l1ls_solve_fista(g, max_iter=45, rel_gap_tol=0.0, check_every=32, precision=L.F64)
    xs, rs = _stepping(g, 45, 32)
    assert torch.equal(x, xs)
    P, D, gap = L.l1ls_objective_gap(g, 1.0, x)
    assert math.isclose(rep["primal"], P, rel_tol=1e-9)
