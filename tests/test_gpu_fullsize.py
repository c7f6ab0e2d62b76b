"""GPU parity at the full size of the single-instance workload: n = 2^20,
m = 2^21, kappa = 1e4, two Givens stages, s = n/100, tau = 1, the seed the
benchmark uses, FP32 bulk over the stored CSR/CSC (and the blocked and
matrix-free operators), in the launch configuration the benchmark times
(check every 32 iterations).  The oracle generates the same instance and
runs its FP64 FISTA over its own sparse A.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1503_03520_amd as L  # noqa: E402
import seeded_inputs as SI  # noqa: E402
from fp32_bounds import fp32_trajectory_bound  # noqa: E402
from oracle import fista as F  # noqa: E402
from oracle import instance as OI  # noqa: E402

pytestmark = pytest.mark.gpu

N = 1 << 20
CFG = (2 * N, N, 1e4, N // 100, 1.0, 1503035201)
ITERS = 64
CHECK = 32

_state = {}


def full():
    if not _state:
        m, n, kappa, s, tau, seed = CFG
        print(f"\n[case] full size m={m} n={n} kappa={kappa} s={s} seed={seed}", flush=True)
        g = L.l1ls_generate(m, n, kappa, s, tau, seed, rounds=2,
                            storage=L.STORE_F32 | L.STORE_F64 | L.STORE_BLK32)
        o = OI.Instance(m, n, kappa, s, tau, seed, rounds=2)
        print("[case] oracle instance built", flush=True)
        A = o.sparse_A()
        _state.update(g=g, o=o, A=A)
    return _state["g"], _state["o"], _state["A"]


def _np(ptr, count, dtype):
    return L.device_to_numpy(ptr, count, dtype)


def _dev(v, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(v), dtype=dtype, device="cuda")


def test_full_size_generator():
    g, o, A = full()
    inf = g.info()
    assert _np(inf.perm_n_dev, o.n, np.int32).tolist() == o.perm_n.tolist()
    assert _np(inf.perm_m_dev, o.m, np.int32).tolist() == o.perm_m.tolist()
    assert _np(inf.support_dev, o.s, np.int32).tolist() == o.support.tolist()
    assert inf.nnz == A.nnz
    for dev, ref in ((inf.e_dev, o.e), (inf.b_dev, o.b)):
        got = _np(dev, o.m, np.float64)
        assert np.abs(got - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())
    assert math.isclose(inf.f_star, o.fstar, rel_tol=1e-12)


@pytest.mark.parametrize("op,prec", [(L.OP_STORED, L.F32), (L.OP_STORED, L.F64), (L.OP_BLOCKED, L.F32),
                                     (L.OP_MATRIX_FREE, L.F32)])
def test_full_size_products(op, prec):
    g, o, A = full()
    x = SI.normal_vector(o.n, 301)
    y = SI.normal_vector(o.m, 302)
    dt = torch.float32 if prec == L.F32 else torch.float64
    tol = 2e-6 if prec == L.F32 else 1e-13
    for trans, v, ref, size in ((0, x, o.matvec(x), o.m), (1, y, o.rmatvec(y), o.n)):
        out = torch.empty(size, dtype=dt, device="cuda")
        L.l1ls_apply(g, trans, op, prec, _dev(v, dt), out)
        torch.cuda.synchronize()
        err = np.abs(out.double().cpu().numpy() - ref).max()
        print(f"op {op} prec {prec} trans {trans}: max err {err:.3e}", flush=True)
        assert err <= tol * max(1.0, np.abs(ref).max())


_ref = {}


def oracle_trajectory():
    if not _ref:
        g, o, A = full()
        _ref["x"], _ref["bound"] = fp32_trajectory_bound(A, o.b, o.tau, 1.0, ITERS)
        print("[case] oracle FISTA done", flush=True)
    return _ref["x"], _ref["bound"]


@pytest.mark.parametrize("op", [L.OP_STORED, L.OP_BLOCKED])
def test_full_size_fista_fp32_trajectory_and_gap(op):
    # FP32 bulk against the FP64 oracle with the bound of the FP32 path
    # (tests/fp32_bounds.py); the device's FP64 primal value at its own
    # iterate against the oracle's objective there.
    g, o, A = full()
    ref, bound = oracle_trajectory()
    fs = L.Fista(g, precision=L.F32, rel_gap_tol=0.0, check_every=CHECK, max_iter=ITERS, op=op)
    fs.iterate(ITERS)
    rep = fs.report()
    x = fs.get_x().cpu().numpy()
    fs.destroy()
    err = np.abs(x - ref).max()
    print(f"op {op}: max |x - x_oracle| {err:.3e} (bound {bound:.3e})", flush=True)
    assert err <= bound
    r = A @ x - o.b
    P = o.tau * np.abs(x).sum() + 0.5 * r @ r
    assert abs(rep["primal"] - P) <= 1e-5 * abs(P)
    Pd, Dd, gap = L.l1ls_objective_gap(g, o.tau, _dev(x))
    assert math.isclose(Pd, P, rel_tol=1e-10)


@pytest.mark.parametrize("solver", ["fista_fp32", "cg_newton"])
def test_full_size_certified_solve_reaches_planted_minimiser(solver):
    # The bulk solve (FP32 FISTA, 300 iterations with the gap test every 32,
    # or 8 CG-Newton steps in FP64), then the FP64 polish of the reduced
    # problem (13).  Procedure IGen (section 3.1) makes x* the unique
    # minimiser; the oracle solves the reduced system on the planted support
    # and signs with a direct sparse solver, which reaches x* to the FP64
    # floor of this instance (kappa(A^T A) = 1e8), and the device's x must
    # equal that solution and x*.
    import scipy.sparse.linalg as spla

    g, o, A = full()
    if solver == "fista_fp32":
        x, rep, _ = L.l1ls_solve_fista(g, max_iter=300, rel_gap_tol=1e-8, check_every=CHECK, precision=L.F32,
                                       polish=1)
    else:
        x, rep, _ = L.l1ls_solve_cg_newton(g, max_iter=8, rel_gap_tol=1e-12, precision=L.F64, polish=1)
    xh = x.cpu().numpy()
    S = np.flatnonzero(o.xstar)
    AS = A.tocsc()[:, S]
    xo = np.zeros(o.n)
    xo[S] = spla.spsolve((AS.T @ AS).tocsc(), AS.T @ o.b - o.tau * np.sign(o.xstar[S]))
    nx = np.linalg.norm(o.xstar)
    e_oracle = np.linalg.norm(xo - o.xstar) / nx
    e_dev = np.linalg.norm(xh - xo) / nx
    print(f"{solver}: polish rounds {rep['polish_rounds']}, rel gap {rep['rel_gap']:.3e}, rel err {rep['rel_err']:.3e}; "
          f"oracle reduced solve vs x* {e_oracle:.3e}, device vs oracle {e_dev:.3e}", flush=True)
    assert rep["rel_gap"] <= 1e-8
    assert e_oracle <= 1e-9
    assert e_dev <= 2e-9 and rep["rel_err"] <= 1e-9
    assert np.array_equal(np.flatnonzero(xh), S)


def teardown_module(module):
    if _state:
        _state["g"].free()
        _state.clear()
    _ref.clear()
