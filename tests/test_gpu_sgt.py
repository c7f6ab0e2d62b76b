"""Section 8.9 (Table 1) instance class on the GPU against the CPU oracle.

Generation is compared bit for bit (the device evaluates IGen steps 3 and
4 in the oracle's operation order without contraction); operator products,
the duality gap and CG-Newton trajectories within FP64 rounding bounds.  At
the Table 1 size n = 2^30 the checks are sampled b values (the oracle
computes single pairs through the inverse support bijection) and properties
of the solve.
"""
import ctypes
import math

import numpy as np
import pytest
import torch

import paper_1503_03520_amd as L
from oracle import fista as OF
from oracle import newton as ON
from oracle.sgt import SgtInstance, b_at_pairs, planted_at

pytestmark = pytest.mark.gpu

SEED = 1503035206
# (n, s, m, overrides): one block, ragged against the 256-pair blocks,
# several blocks, the minimum size, square A, non-default parameters
CASES = [
    (64, 6, None, {}),
    (4098, 4, None, {}),
    (2 ** 16, 64, None, {}),
    (2, 1, None, {}),
    (1030, 3, 1030, {}),
    (2050, 7, 4100, dict(theta=0.3, sigma_odd=2.0, sigma_even=0.5, x_neg=-3.0, x_pos=7.5, tau=0.37)),
]
# the laws of sections 8.4 to 8.6: uniform singular values, OsGen and OsGen3
LAW_CASES = [
    (4098, 32, None, dict(sigma_law="uniform", sigma_scale=1e3, xstar_law="osgen", gamma=10.0)),
    (4098, 32, None, dict(theta=2 * math.pi / 10, sigma_law="uniform", sigma_scale=10.0, xstar_law="osgen3",
                          gamma=100.0)),
    (2050, 9, None, dict(theta=2 * math.pi / 1e3, sigma_law="uniform", sigma_scale=100.0, xstar_law="osgen3",
                         gamma=100.0, s1=0, s2=9)),
    (1030, 5, 2060, dict(sigma_law="uniform", sigma_scale=1.0, xstar_law="osgen3", gamma=3.0, s1=5, s2=0,
                         tau=0.5)),
    (64, 10, None, dict(xstar_law="osgen", gamma=2.0)),
]
_SIGMA = {"alternating": L.SIGMA_ALTERNATING, "uniform": L.SIGMA_UNIFORM}
_XSTAR = {"table1": L.XSTAR_TABLE1, "osgen": L.XSTAR_OSGEN, "osgen3": L.XSTAR_OSGEN3}


def make(n, s, m, kw):
    dev_kw = dict(kw)
    if "sigma_law" in dev_kw:
        dev_kw["sigma_law"] = _SIGMA[dev_kw["sigma_law"]]
    if "xstar_law" in dev_kw:
        dev_kw["xstar_law"] = _XSTAR[dev_kw["xstar_law"]]
    p = L.sgt_params(n, SEED, s=s, **({} if m is None else {"m": m}), **dev_kw)
    H = L.SgtInstance(p)
    O = SgtInstance(n, s, SEED, m=m, **kw)
    return H, O


def dev(v):
    return torch.from_numpy(np.ascontiguousarray(v, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("case", CASES + LAW_CASES)
def test_generation_is_bitwise_the_oracle(case):
    n, s, m, kw = case
    H, O = make(n, s, m, kw)
    d = H.describe()
    xs = torch.empty(n, dtype=torch.float64, device="cuda")
    g = torch.empty(n, dtype=torch.float64, device="cuda")
    H.planted(xs, g)
    assert np.array_equal(host(xs), O.xstar)
    assert np.array_equal(host(g), O.g)
    b = L.device_to_numpy(d.b_dev, n, np.float64)
    diff = np.flatnonzero(b != O.b[:n])
    assert diff.size == 0, (diff[:8], b[diff[:8]], O.b[:n][diff[:8]], np.spacing(O.b[:n][diff[:8]]))
    assert not O.b[n:].any()
    assert d.f_star == pytest.approx(O.fstar, rel=1e-13)
    assert d.L == O.L and d.c == O.c and d.s_rot == O.sn
    assert d.sigma_min == O.sigma.min() and d.sigma_max == O.sigma.max()
    H.free()


@pytest.mark.parametrize("case", CASES + LAW_CASES[:2])
def test_operator_products_match_oracle(case):
    n, s, m, kw = case
    H, O = make(n, s, m, kw)
    rng = np.random.default_rng(11)
    x = rng.standard_normal(n)
    y = rng.standard_normal(O.m)
    ax = torch.full((O.m,), float("nan"), dtype=torch.float64, device="cuda")
    aty = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    H.apply(0, dev(x), ax)
    H.apply(1, dev(y), aty)
    ref_ax, ref_aty = O.matvec(x), O.rmatvec(y)
    tol = 4 * np.finfo(float).eps * max(O.sigma.max(), 1.0)
    assert np.abs(host(ax) - ref_ax).max() <= tol * np.abs(x).max() * 2
    assert np.abs(host(aty) - ref_aty).max() <= tol * np.abs(y).max() * 2
    H.free()


@pytest.mark.parametrize("case", CASES[:3] + CASES[5:] + LAW_CASES[:2])
def test_gap_matches_oracle(case):
    n, s, m, kw = case
    H, O = make(n, s, m, kw)
    A = O.sparse_A()
    rng = np.random.default_rng(5)
    eps = np.finfo(float).eps
    for x in (O.xstar, O.xstar + 0.01 * rng.standard_normal(n), np.zeros(n)):
        P, D, gap = H.objective_gap(O.tau, dev(x))
        Po, Do, go = OF.duality_gap(lambda v: A @ v, lambda v: A.T @ v, O.b, O.tau, x)
        # r = A x - b is formed from terms of size |A x| + |b| (up to 1e6 on the
        # support), so each side's sums carry rounding of that size
        ax = np.abs(A @ x)
        scale = float(np.sum((ax + np.abs(O.b[: O.m])) * (ax + np.abs(O.b[: O.m]))))
        assert abs(P - Po) <= 8 * eps * (scale + abs(Po))
        assert abs(D - Do) <= 8 * eps * (scale + abs(Do))
    H.free()


def newton_pair(H, O, steps, **kw):
    x, rep, st = H.solve_cg_newton(max_iter=steps, **kw)
    hess = "primal" if kw.get("hessian", 0) == 1 else "primal_dual"
    xo, sto = ON.newton_cg(O.matvec, O.rmatvec, O.colnorm2(), O.b, O.tau, max_newton=steps, hessian=hess)
    return host(x), rep, st, xo, sto


@pytest.mark.parametrize("steps", [1, 2, 3, 8])
def test_cg_newton_trajectory_matches_oracle(steps):
    n, s = 4098, 4
    H, O = make(n, s, None, {})
    x, rep, st, xo, sto = newton_pair(H, O, steps)
    assert st == L.L1LS_NOT_CONVERGED and rep["iterations"] == steps
    assert abs(rep["inner"] - sto["pcg"]) <= 2 * steps
    scale = np.abs(xo).max()
    assert np.abs(x - xo).max() <= 1e-6 * scale
    rel = np.linalg.norm(x - O.xstar) / np.linalg.norm(O.xstar)
    assert rep["rel_err"] == pytest.approx(rel, rel=1e-6)
    H.free()


def test_cg_newton_primal_hessian_matches_oracle():
    H, O = make(2050, 7, 4100, CASES[5][3])
    x, rep, st, xo, sto = newton_pair(H, O, 3, hessian=1)
    assert rep["iterations"] == 3
    assert np.abs(x - xo).max() <= 1e-6 * np.abs(xo).max()
    H.free()


def test_cg_newton_converges_to_oracle_minimiser():
    n, s = 4098, 4
    H, O = make(n, s, None, {})
    # the FP64 floor of ||grad f_mu||_inf here is about eps sigma_even max|b| = 2e-8
    x, rep, st = H.solve_cg_newton(max_iter=300, rel_gap_tol=1e-7)
    xo, sto = ON.newton_cg(O.matvec, O.rmatvec, O.colnorm2(), O.b, O.tau, max_newton=300, grad_tol=1e-7)
    assert sto["grad_inf"] <= 1e-7
    assert st == L.L1LS_OK and rep["converged"] == 1
    x = host(x)
    assert np.abs(x - xo).max() <= 1e-7 * np.abs(xo).max()
    # the smoothed minimiser sits within O(mu) of x*: relative error far below 1e-4
    assert rep["rel_err"] <= 1e-6
    H.free()


def test_cg_newton_edge_cases():
    H, O = make(64, 6, None, {})
    n = 64
    # no Newton step: x stays at the start
    x, rep, st = H.solve_cg_newton(max_iter=0)
    assert rep["iterations"] == 0 and not host(x).any()
    # warm start at x* in place: one gradient evaluation, few steps
    xs = torch.empty(n, dtype=torch.float64, device="cuda")
    H.planted(xs)
    x, rep, st = H.solve_cg_newton(x_out=xs, x0=xs, max_iter=50)
    assert rep["rel_err"] <= 1e-6
    # options this class does not build, misaligned vectors
    buf = torch.zeros(n + 1, dtype=torch.float64, device="cuda")
    o = L.solve_opts(max_iter=1)
    rep = L.Report()
    assert L.lib().l1ls_sgt_solve_cg_newton(H.handle, ctypes.byref(o), ctypes.c_void_p(buf.data_ptr() + 8),
                                             ctypes.byref(rep)) == -1
    for kw in (dict(precision=L.F32), dict(polish=1)):
        o = L.solve_opts(max_iter=1, **kw)
        assert L.lib().l1ls_sgt_solve_cg_newton(H.handle, ctypes.byref(o), ctypes.c_void_p(buf.data_ptr()),
                                                 ctypes.byref(rep)) == -6
    assert L.lib().l1ls_sgt_apply(H.handle, 2, ctypes.c_void_p(buf.data_ptr()), ctypes.c_void_p(buf.data_ptr()),
                                   None) == -1
    H.free()


def test_stepping_object_equals_one_solve():
    # l1ls_sgt_newton_*: 3 + 5 Newton steps give the bits of one 8-step solve
    H, O = make(4098, 4, None, {})
    x1, rep1, _ = H.solve_cg_newton(max_iter=8)
    N = H.newton()
    r3, st3 = N.step(3)
    assert r3["iterations"] == 3 and st3 == L.L1LS_NOT_CONVERGED
    r8, _ = N.step(5)
    assert r8["iterations"] == 8 and r8["inner"] == rep1["inner"]
    assert np.array_equal(host(N.x), host(x1))
    assert r8["rel_err"] == rep1["rel_err"] and r8["primal"] == rep1["primal"]
    N.destroy()
    H.free()


def test_s_zero_gives_zero_planted_solution():
    H, O = make(256, 0, None, {})
    xs = torch.full((256,), 1.0, dtype=torch.float64, device="cuda")
    H.planted(xs)
    assert not host(xs).any()
    assert H.describe().f_star == pytest.approx(O.fstar, rel=1e-13)
    H.free()


def test_table_1_size_sampled_generation_and_solve():
    # n = 2^30, m = 2^31, s = 2^20: the smallest instance of Table 1.  b is
    # checked on sampled pairs (first, last, random) against the oracle's
    # single-pair construction, the planted x* against the inverse bijection,
    # and the 8-Newton-step solve against the behaviour section 8.9 reports.
    n = 2 ** 30
    p = L.sgt_params(n, SEED)
    H = L.SgtInstance(p)
    d = H.describe()
    rng = np.random.default_rng(2)
    pairs = np.unique(np.r_[0, 1, n // 2 - 1, n // 4, rng.integers(0, n // 2, 60)])
    bi, bj = b_at_pairs(n, p.s, SEED, pairs)
    base = d.b_dev
    for k, ei, ej in zip(pairs, bi, bj):
        got = L.device_to_numpy(base + 16 * int(k), 2, np.float64)
        assert got[0] == ei and got[1] == ej, int(k)
    x, rep, st = H.solve_cg_newton(max_iter=8)
    assert rep["iterations"] == 8
    assert rep["rel_err"] <= 5e-4
    # the total PCG count of the 8 Newton steps: section 8.9 reports about
    # 100 per step; this reading of CG-Newton needs more at this size (the
    # oracle's counts grow from 2^14 to 2^18), and the later steps' PCG runs
    # reach their 1000-iteration cap (4,224 = 1 + 1 + 6 + 216 + 4 x 1000 in
    # the measured run), so only the total is bounded here
    assert 8 <= rep["inner"] <= 8 * 1000
    # the planted values of the sampled indices, one by one
    idx = np.unique(np.r_[2 * pairs, 2 * pairs + 1])
    xs_ref, _ = planted_at(n, p.s, SEED, idx)
    xs = torch.empty(n, dtype=torch.float64, device="cuda")
    H.planted(xs)
    got = host(xs[torch.from_numpy(idx).cuda()])
    assert np.array_equal(got, xs_ref)
    assert int(torch.count_nonzero(xs)) == p.s
    del xs, x
    H.free()


@pytest.mark.parametrize("case", LAW_CASES + CASES[:1])
def test_kappa_rho_matches_oracle(case):
    n, s, m, kw = case
    H, O = make(n, s, m, kw)
    for rho in (0.1, 1.0, 50.0):
        want = O.kappa_rho(rho)
        got = H.kappa_rho(rho)
        if math.isinf(want):
            assert math.isinf(got)
        else:
            assert got == pytest.approx(want, rel=1e-12)
    H.free()


@pytest.mark.parametrize("case", [CASES[1], CASES[5], LAW_CASES[0], LAW_CASES[1]])
@pytest.mark.parametrize("iters", [1, 2, 10, 100])
def test_fista_trajectory_matches_oracle(case, iters):
    n, s, m, kw = case
    H, O = make(n, s, m, kw)
    x, rep, st = H.solve_fista(max_iter=iters, rel_gap_tol=0.0, check_every=7)
    assert rep["iterations"] == iters and st == L.L1LS_NOT_CONVERGED
    xo = OF.fista(O.matvec, O.rmatvec, O.b, O.tau, O.L, iters)
    assert np.abs(host(x) - xo).max() <= 1e-11 * max(1.0, np.abs(xo).max())
    P, D, gap = OF.duality_gap(O.matvec, O.rmatvec, O.b, O.tau, xo)
    assert rep["primal"] == pytest.approx(P, rel=1e-9)
    H.free()


def test_fista_stops_at_objective_target():
    # section 8.3's protocol: run until f_tau falls to a target value; the
    # test is evaluated every check_every iterations
    n, s, m, kw = LAW_CASES[0]
    H, O = make(n, s, m, kw)
    x50 = OF.fista(O.matvec, O.rmatvec, O.b, O.tau, O.L, 50)
    target = OF.primal(O.matvec, O.b, O.tau, x50)
    x, rep, st = H.solve_fista(max_iter=1000, rel_gap_tol=0.0, f_target=target * (1 + 1e-12), check_every=10)
    assert st == L.L1LS_OK and rep["converged"] == 1
    k = rep["iterations"]
    assert k % 10 == 0 and rep["primal"] <= target * (1 + 1e-12)
    # the first check at which the objective passed: the one before had not
    if k > 10:
        prev = OF.primal(O.matvec, O.b, O.tau, OF.fista(O.matvec, O.rmatvec, O.b, O.tau, O.L, k - 10))
        assert prev > target * (1 + 1e-12)
    H.free()


@pytest.mark.parametrize("steps", [3, 8])
def test_cg_newton_on_section_8_5_law_matches_oracle(steps):
    # Early steps agree to 1e-6.  Later, a PCG that ends one iteration apart
    # on the two sides (its stop test compares ||r|| with 0.1 ||rhs||, and
    # the two sides round the sums differently) gives a different inexact
    # Newton direction: both are valid, so from there the check is the
    # objective and a looser bound on x.
    n, s, m, kw = LAW_CASES[1]
    H, O = make(n, s, m, kw)
    x, rep, st = H.solve_cg_newton(max_iter=steps)
    xo, sto = ON.newton_cg(O.matvec, O.rmatvec, O.colnorm2(), O.b, O.tau, max_newton=steps)
    assert rep["iterations"] == steps
    assert abs(rep["inner"] - sto["pcg"]) <= 2 * steps
    x = host(x)
    scale = np.abs(xo).max()
    if steps <= 3:
        assert np.abs(x - xo).max() <= 1e-6 * scale
    else:
        assert np.abs(x - xo).max() <= 1e-4 * scale
        fo = OF.primal(O.matvec, O.b, O.tau, xo)
        assert rep["primal"] == pytest.approx(fo, rel=1e-6)
    H.free()


def test_cg_newton_on_section_8_5_law_reaches_oracle_minimiser():
    n, s, m, kw = LAW_CASES[1]
    H, O = make(n, s, m, kw)
    x, rep, st = H.solve_cg_newton(max_iter=300, rel_gap_tol=1e-7)
    xo, sto = ON.newton_cg(O.matvec, O.rmatvec, O.colnorm2(), O.b, O.tau, max_newton=300, grad_tol=1e-7)
    assert st == L.L1LS_OK and sto["grad_inf"] <= 1e-7
    assert np.abs(host(x) - xo).max() <= 1e-7 * np.abs(xo).max()
    H.free()


def test_section_8_5_instance_at_paper_size():
    # n = 2^22, m = 2n, s = n / 2^7, OsGen3 with gamma = 100, s1 = s2 = s/2,
    # sigma uniform on [0, 100] + 0.1, theta = 2 pi / 10: the radix selection
    # on the device picks exactly the oracle's components and b is bitwise equal
    n = 2 ** 22
    kw = dict(theta=2 * math.pi / 10, sigma_law="uniform", sigma_scale=100.0, xstar_law="osgen3", gamma=100.0)
    H, O = make(n, n // 128, None, kw)
    xs = torch.empty(n, dtype=torch.float64, device="cuda")
    H.planted(xs)
    assert np.array_equal(host(xs), O.xstar)
    d = H.describe()
    assert np.array_equal(L.device_to_numpy(d.b_dev, n, np.float64), O.b[:n])
    assert H.kappa_rho(0.1) == pytest.approx(O.kappa_rho(0.1), rel=1e-12)
    H.free()


@pytest.mark.parametrize("case", [CASES[1], LAW_CASES[0], LAW_CASES[1]])
@pytest.mark.parametrize("p", [1.0, 0.5, 0.05])
@pytest.mark.parametrize("steps", [1, 5, 50])
def test_pcdm_trajectory_matches_oracle(case, p, steps):
    from oracle.sgt import pcdm
    n, s, m, kw = case
    H, O = make(n, s, m, kw)
    x, rep, st = H.solve_pcdm(max_iter=steps, rel_gap_tol=0.0, check_every=16, pcdm_p=p)
    assert rep["iterations"] == steps and st == L.L1LS_NOT_CONVERGED
    xo = pcdm(O, O.tau, steps, p=p)
    assert np.abs(host(x) - xo).max() <= 1e-11 * max(1.0, np.abs(xo).max())
    H.free()


def test_pcdm_reaches_objective_target():
    from oracle.sgt import pcdm
    n, s, m, kw = LAW_CASES[0]
    H, O = make(n, s, m, kw)
    target = OF.primal(O.matvec, O.b, O.tau, pcdm(O, O.tau, 40))
    x, rep, st = H.solve_pcdm(max_iter=5000, rel_gap_tol=0.0, f_target=target * (1 + 1e-12), check_every=8)
    assert st == L.L1LS_OK and rep["iterations"] % 8 == 0 and rep["primal"] <= target * (1 + 1e-12)
    H.free()


# ---- IGen2 (section 3.2, m < n) -------------------------------------------------
IGEN2_CASES = [
    (64, 96, 6, dict()),
    (130, 260, 9, dict(sigma_law="uniform", sigma_scale=10.0, xstar_law="osgen", gamma=3.0, tau=0.37)),
    (1026, 1030, 5, dict(sigma_law="uniform", sigma_scale=100.0, xstar_law="osgen", gamma=10.0)),
    (4098, 6000, 40, dict(theta=2 * math.pi / 10, sigma_law="uniform", sigma_scale=1.0, xstar_law="osgen",
                          gamma=5.0)),
]


def make_igen2(m, n, s, kw):
    from oracle.sgt import SgtIGen2Instance
    dev_kw = dict(kw)
    if "sigma_law" in dev_kw:
        dev_kw["sigma_law"] = _SIGMA[dev_kw["sigma_law"]]
    if "xstar_law" in dev_kw:
        dev_kw["xstar_law"] = _XSTAR[dev_kw["xstar_law"]]
    H = L.SgtInstance(L.sgt_params(n, SEED, m=m, s=s, **dev_kw))
    O = SgtIGen2Instance(m, n, s, SEED, **kw)
    return H, O


@pytest.mark.parametrize("case", IGEN2_CASES)
def test_igen2_generation_is_bitwise_the_oracle(case):
    m, n, s, kw = case
    H, O = make_igen2(m, n, s, kw)
    d = H.describe()
    torch.cuda.synchronize()
    assert np.array_equal(L.device_to_numpy(d.b_dev, m, np.float64), O.b)
    assert np.array_equal(L.device_to_numpy(d.colscale_dev, n - m, np.float64), O.colscale)
    xs = torch.empty(n, dtype=torch.float64, device="cuda")
    g = torch.empty(n, dtype=torch.float64, device="cuda")
    H.planted(xs, g)
    assert np.array_equal(host(xs), O.xstar)
    assert np.array_equal(host(g)[:m], O.g) and not host(g)[m:].any()
    assert d.f_star == pytest.approx(O.fstar, rel=1e-13)
    if O.L is not None:
        assert d.L == pytest.approx(O.L, rel=1e-13)
    with pytest.raises(L.L1lsError):
        H.kappa_rho(0.1)
    H.free()


@pytest.mark.parametrize("case", IGEN2_CASES[:3])
def test_igen2_products_and_gap_match_oracle(case):
    m, n, s, kw = case
    H, O = make_igen2(m, n, s, kw)
    rng = np.random.default_rng(8)
    x = rng.standard_normal(n)
    y = rng.standard_normal(m)
    ax = torch.full((m,), float("nan"), dtype=torch.float64, device="cuda")
    aty = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    H.apply(0, dev(x), ax)
    H.apply(1, dev(y), aty)
    A = O.sparse_A()
    scale = np.abs(A.data).max()
    assert np.abs(host(ax) - O.matvec(x)).max() <= 16 * np.finfo(float).eps * scale * np.abs(x).max()
    assert np.abs(host(aty) - O.rmatvec(y)).max() <= 16 * np.finfo(float).eps * scale * np.abs(y).max()
    P, D, gap = H.objective_gap(O.tau, dev(O.xstar))
    Po, Do, go = OF.duality_gap(lambda v: A @ v, lambda v: A.T @ v, O.b, O.tau, O.xstar)
    assert P == pytest.approx(Po, rel=1e-12) and abs(gap) <= 1e-8
    H.free()


@pytest.mark.parametrize("case", IGEN2_CASES[1:3])
@pytest.mark.parametrize("iters", [1, 10, 100])
def test_igen2_fista_and_pcdm_trajectories_match_oracle(case, iters):
    from oracle.sgt import pcdm
    m, n, s, kw = case
    H, O = make_igen2(m, n, s, kw)
    L_dev = H.describe().L
    x, rep, st = H.solve_fista(max_iter=iters, rel_gap_tol=0.0, check_every=7)
    xo = OF.fista(O.matvec, O.rmatvec, O.b, O.tau, L_dev, iters)
    assert np.abs(host(x) - xo).max() <= 1e-11 * max(1.0, np.abs(xo).max())
    for p in (1.0, 0.3):
        x, rep, st = H.solve_pcdm(max_iter=iters, rel_gap_tol=0.0, check_every=7, pcdm_p=p)
        xp = pcdm(O, O.tau, iters, p=p, omega=4)
        assert np.abs(host(x) - xp).max() <= 1e-11 * max(1.0, np.abs(xp).max())
    H.free()


@pytest.mark.parametrize("case", IGEN2_CASES[1:3])
def test_igen2_cg_newton_matches_oracle(case):
    # The first two Newton steps agree to 1e-6.  After that, N~'s column
    # scales (over six orders of magnitude) make the Newton systems so badly
    # conditioned that the two sides' PCGs, rounding in different orders, stop
    # at different iterations: the comparison is then the converged minimiser.
    m, n, s, kw = case
    H, O = make_igen2(m, n, s, kw)
    x, rep, st = H.solve_cg_newton(max_iter=2)
    xo, sto = ON.newton_cg(O.matvec, O.rmatvec, O.colnorm2(), O.b, O.tau, max_newton=2)
    assert rep["iterations"] == 2 and rep["inner"] == sto["pcg"]
    assert np.abs(host(x) - xo).max() <= 1e-6 * np.abs(xo).max()
    x, rep, st = H.solve_cg_newton(max_iter=200, rel_gap_tol=1e-8 / O.tau)
    xo, sto = ON.newton_cg(O.matvec, O.rmatvec, O.colnorm2(), O.b, O.tau, max_newton=200, grad_tol=1e-8)
    assert st == L.L1LS_OK and sto["grad_inf"] <= 1e-8
    x = host(x)
    assert np.abs(x - xo).max() <= 1e-6 * np.abs(xo).max()
    ro = np.linalg.norm(xo - O.xstar) / np.linalg.norm(O.xstar)
    assert rep["rel_err"] == pytest.approx(ro, rel=1e-3)
    H.free()
