"""GPU parity: the HIP library (through the C ABI) against the CPU oracle.

Both sides generate the instance from the same (m, n, kappa, s, tau, seed,
rounds); integer outputs must agree bit for bit, floating-point outputs
within the tolerances written in each test (derived in the design notes).
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

# (m, n, kappa, s, tau, seed, rounds): the FP64 workload (n = 1024, m = 2n,
# kappa 1e2, one stage, s = 10, tau = 1) and cases that are ragged with
# respect to the 256-thread tiles, two-stage, tiny and degenerate.
C1 = (2048, 1024, 1e2, 10, 1.0, 1503035200, 1)
CASES = [
    C1,
    (1010, 502, 1e3, 7, 0.5, 17, 2),     # ragged, two stages
    (4, 2, 3.0, 1, 1.0, 5, 1),           # minimum size
    (6, 6, 10.0, 2, 2.0, 6, 2),          # square A, N = 6 cycle-walks
    (600, 300, 1.0, 5, 1.0, 8, 2),       # kappa = 1 (orthonormal columns)
    (512, 256, 1e4, 0, 1.0, 9, 2),       # s = 0: x* = 0
]


def _np(ptr, count, dtype):
    return L.device_to_numpy(ptr, count, dtype)


_cache = {}


def pair(cfg, layout=L.LAYOUT_STAGE):
    key = (cfg, layout)
    if key not in _cache:
        m, n, kappa, s, tau, seed, r = cfg
        print(f"\n[case] generate m={m} n={n} kappa={kappa} s={s} tau={tau} seed={seed} rounds={r} "
              f"layout={layout}", flush=True)
        g = L.l1ls_generate(m, n, kappa, s, tau, seed, rounds=r, layout=layout)
        o = OI.Instance(m, n, kappa, s, tau, seed, rounds=r)
        _cache[key] = (g, o, o.sparse_A())
    return _cache[key]


def operator_order(o, A, layout):
    """The oracle's A with rows/columns in the library's storage order."""
    if layout == L.LAYOUT_NATURAL:
        B = A.tocsr()
    else:
        B = A.tocsr()[o.perm_m, :][:, o.perm_n].tocsr()
    B.sort_indices()
    return B


def ulp_close(a, b, ulps):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    tol = ulps * np.spacing(np.maximum(np.abs(a), np.abs(b)))
    return np.all(np.abs(a - b) <= tol)


@pytest.mark.parametrize("cfg", CASES)
@pytest.mark.parametrize("layout", [L.LAYOUT_NATURAL, L.LAYOUT_STAGE])
def test_generator_integers_bit_exact(cfg, layout):
    g, o, A = pair(cfg, layout)
    inf = g.info()
    m, n = o.m, o.n
    assert inf.layout == layout
    assert _np(inf.perm_n_dev, n, np.int32).tolist() == o.perm_n.tolist()
    assert _np(inf.perm_m_dev, m, np.int32).tolist() == o.perm_m.tolist()
    assert _np(inf.support_dev, o.s, np.int32).tolist() == o.support.tolist()
    assert inf.nnz == A.nnz
    B = operator_order(o, A, layout)
    Bc = B.tocsc()
    Bc.sort_indices()
    assert np.array_equal(_np(inf.csr_ptr_dev, m + 1, np.int32), B.indptr)
    assert np.array_equal(_np(inf.csr_col_dev, A.nnz, np.int32), B.indices)
    assert np.array_equal(_np(inf.csc_ptr_dev, n + 1, np.int32), Bc.indptr)
    assert np.array_equal(_np(inf.csc_row_dev, A.nnz, np.int32), Bc.indices)
    v64 = _np(inf.csr_val64_dev, A.nnz, np.float64)
    assert np.abs(v64 - B.data).max() <= 1e-14 * max(1.0, np.abs(B.data).max())
    assert np.abs(_np(inf.csc_val64_dev, A.nnz, np.float64) - Bc.data).max() <= 1e-14
    v32 = _np(inf.csr_val32_dev, A.nnz, np.float32)
    assert np.array_equal(v32, v64.astype(np.float32))


@pytest.mark.parametrize("cfg", CASES)
def test_generator_floats(cfg):
    g, o, A = pair(cfg)
    inf = g.info()
    m, n = o.m, o.n
    # rotation angles: same rejection decisions (so the same draws), then a
    # square root and two divisions of the device math library: <= 2 ulps
    for t in range(o.rounds):
        for dev, st, N in ((inf.cs_n_dev[t], o.G_stages[t], n), (inf.cs_m_dev[t], o.Q_stages[t], m)):
            cs = _np(dev, N, np.float64)
            d = np.abs(np.concatenate([cs[0::2] - st.c, cs[1::2] - st.s]))
            ref = np.concatenate([np.abs(st.c), np.abs(st.s)])
            ulps = d / np.spacing(np.maximum(ref, 1e-300))
            print(f"angle ulps: max {ulps.max():.1f}, nonzero {np.count_nonzero(d)}/{d.size}")
            assert ulps.max() <= 2.0
    # pow / log / cos of two math libraries: a few ulps
    assert ulp_close(_np(inf.sigma_dev, n, np.float64), o.sigma, 4)
    assert ulp_close(_np(inf.x_star_dev, n, np.float64), o.xstar, 8)
    gd = _np(inf.g_dev, n, np.float64)
    assert np.array_equal(gd, o.g)
    # e, b and A: products and sums of the above, compared to the vector scale
    for name, dev, ref in (("e", inf.e_dev, o.e), ("b", inf.b_dev, o.b)):
        got = _np(dev, m, np.float64)
        scale = max(1.0, np.abs(ref).max())
        assert np.abs(got - ref).max() <= 1e-13 * scale, name
    assert math.isclose(inf.f_star, o.fstar, rel_tol=1e-12)
    assert inf.L == 1.0


def _dev(v, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(v), dtype=dtype, device="cuda")


@pytest.mark.parametrize("cfg", CASES)
@pytest.mark.parametrize("op,layout", [(L.OP_STORED, L.LAYOUT_NATURAL), (L.OP_STORED, L.LAYOUT_STAGE),
                                       (L.OP_MATRIX_FREE, L.LAYOUT_STAGE)])
def test_operator_products(cfg, op, layout):
    g, o, A = pair(cfg, layout)
    x = SI.normal_vector(o.n, 101)
    y = SI.normal_vector(o.m, 102)
    ax = o.matvec(x)
    aty = o.rmatvec(y)
    for prec, dt, tol in ((L.F64, torch.float64, 1e-13), (L.F32, torch.float32, 2e-6)):
        out = torch.empty(o.m, dtype=dt, device="cuda")
        L.l1ls_apply(g, 0, op, prec, _dev(x, dt), out)
        torch.cuda.synchronize()
        assert np.abs(out.double().cpu().numpy() - ax).max() <= tol * max(1.0, np.abs(ax).max())
        out = torch.empty(o.n, dtype=dt, device="cuda")
        L.l1ls_apply(g, 1, op, prec, _dev(y, dt), out)
        torch.cuda.synchronize()
        assert np.abs(out.double().cpu().numpy() - aty).max() <= tol * max(1.0, np.abs(aty).max())


@pytest.mark.parametrize("cfg", CASES)
def test_objective_gap(cfg):
    g, o, A = pair(cfg)
    mv, rmv = (lambda v: A @ v), (lambda v: A.T @ v)
    P, D, gap = L.l1ls_objective_gap(g, o.tau, _dev(o.xstar))
    assert math.isclose(P, o.fstar, rel_tol=1e-12, abs_tol=1e-12)
    assert abs(gap) <= 1e-12
    x = o.xstar + 0.05 * SI.normal_vector(o.n, 103)
    P, D, gap = L.l1ls_objective_gap(g, o.tau, _dev(x))
    Pr, Dr, gr = F.duality_gap(mv, rmv, o.b, o.tau, x)
    assert math.isclose(P, Pr, rel_tol=1e-12) and math.isclose(D, Dr, rel_tol=1e-12, abs_tol=1e-9)
    tau2 = 0.37 * o.tau
    P, D, gap = L.l1ls_objective_gap(g, tau2, _dev(x))
    Pr, Dr, gr = F.duality_gap(mv, rmv, o.b, tau2, x)
    assert math.isclose(P, Pr, rel_tol=1e-12) and math.isclose(D, Dr, rel_tol=1e-12, abs_tol=1e-9)


@pytest.mark.parametrize("cfg", CASES)
@pytest.mark.parametrize("iters", [1, 2, 10, 100])
@pytest.mark.parametrize("layout", [L.LAYOUT_NATURAL, L.LAYOUT_STAGE])
def test_fista_trajectory_fp64(cfg, iters, layout):
    # FP64 x_k of the fused kernels against the oracle's x_k, same L.
    g, o, A = pair(cfg, layout)
    x, rep, _ = L.l1ls_solve_fista(g, max_iter=iters, rel_gap_tol=0.0, check_every=1, precision=L.F64)
    ref = F.fista(lambda v: A @ v, lambda v: A.T @ v, o.b, o.tau, 1.0, iters)
    scale = max(1.0, np.abs(ref).max())
    assert np.abs(x.cpu().numpy() - ref).max() <= 1e-11 * scale
    assert rep["iterations"] == iters


@pytest.mark.parametrize("cfg", CASES)
@pytest.mark.parametrize("iters", [1, 2, 10, 100])
def test_fista_trajectory_fp64_matrix_free(cfg, iters):
    # FISTA over the matrix-free operator (rotation triplets applied on the
    # fly, Algorithms MvPA/MvPAt) against the oracle's x_k.
    g, o, A = pair(cfg)
    x, rep, _ = L.l1ls_solve_fista(g, max_iter=iters, rel_gap_tol=0.0, check_every=1, precision=L.F64,
                                   op=L.OP_MATRIX_FREE)
    ref = F.fista(lambda v: A @ v, lambda v: A.T @ v, o.b, o.tau, 1.0, iters)
    scale = max(1.0, np.abs(ref).max())
    assert np.abs(x.cpu().numpy() - ref).max() <= 1e-11 * scale
    assert rep["iterations"] == iters


MF_MULTIBLOCK = [
    (4096, 2050, 1e3, 20, 1.0, 23, 2),  # several 256-pair workgroups per side, the n side's last one ragged
    # m >> n: ten m-side workgroups (the last ragged) with 300 active positions
    # among 5000, so the compact v's ranks carry across many workgroups
    (5000, 300, 1e2, 6, 1.0, 29, 2),
]


@pytest.mark.parametrize("cfg", MF_MULTIBLOCK)
@pytest.mark.parametrize("iters", [1, 2, 25])
def test_fista_trajectory_fp64_matrix_free_multiblock(cfg, iters):
    # The fused matrix-free passes recompute a neighbour workgroup's stage pair
    # at each workgroup edge; both sides here span several workgroups.
    g, o, A = pair(cfg)
    x, rep, _ = L.l1ls_solve_fista(g, max_iter=iters, rel_gap_tol=0.0, check_every=1, precision=L.F64,
                                   op=L.OP_MATRIX_FREE)
    ref = F.fista(lambda v: A @ v, lambda v: A.T @ v, o.b, o.tau, 1.0, iters)
    scale = max(1.0, np.abs(ref).max())
    assert np.abs(x.cpu().numpy() - ref).max() <= 1e-11 * scale


@pytest.mark.parametrize("cfg", MF_MULTIBLOCK)
def test_matrix_free_products_multiblock(cfg):
    # A x and A^T y of l1ls_apply (the stage-by-stage operator) against the
    # oracle's rotations, FP64 and FP32; the fused passes and their compact v
    # are covered by the FISTA trajectories above and the CG-Newton tests
    g, o, A = pair(cfg)
    x = SI.normal_vector(o.n, 111)
    y = SI.normal_vector(o.m, 112)
    ax, aty = o.matvec(x), o.rmatvec(y)
    for prec, dt, tol in ((L.F64, torch.float64, 1e-13), (L.F32, torch.float32, 2e-6)):
        for trans, v, ref, size in ((0, x, ax, o.m), (1, y, aty, o.n)):
            out = torch.empty(size, dtype=dt, device="cuda")
            L.l1ls_apply(g, trans, L.OP_MATRIX_FREE, prec, _dev(v, dt), out)
            torch.cuda.synchronize()
            assert np.abs(out.double().cpu().numpy() - ref).max() <= tol * max(1.0, np.abs(ref).max()), (prec, trans)


# n = 2^14: source chunks of 2^11 and 2^10 sources, 8 and 16 of them per side
MF_WIN_FULL_CHUNKS = (32768, 16384, 1e3, 160, 1.0, 31, 2)


@pytest.mark.parametrize("cfg", MF_MULTIBLOCK + [C1, MF_WIN_FULL_CHUNKS])
def test_matrix_free_windowed_gathers_are_bitwise_the_plain_ones(cfg):
    # The windowed gathers (L1LS_STORE_MF_WINDOWS; windows of 256 positions
    # at these sizes, so each side spans several) read the same elements as
    # the plain ones: FISTA over the fused passes in FP32 and FP64, CG-Newton
    # and the power method give bitwise the same results.
    m, n, kappa, s, tau, seed, r = cfg
    g, o, A = pair(cfg)
    gw = L.l1ls_generate(m, n, kappa, s, tau, seed, rounds=r, storage=L.STORE_F64 | L.STORE_MF_WINDOWS)
    try:
        for prec in (L.F32, L.F64):
            kw = dict(max_iter=40, rel_gap_tol=0.0, check_every=8, precision=prec, op=L.OP_MATRIX_FREE)
            a, ra, _ = L.l1ls_solve_fista(g, **kw)
            b, rb, _ = L.l1ls_solve_fista(gw, **kw)
            assert torch.equal(a, b) and ra["primal"] == rb["primal"], prec
        xs, rs, _ = L.l1ls_solve_cg_newton(g, max_iter=3, rel_gap_tol=1e-12, op=L.OP_MATRIX_FREE)
        xw, rw, _ = L.l1ls_solve_cg_newton(gw, max_iter=3, rel_gap_tol=1e-12, op=L.OP_MATRIX_FREE)
        assert torch.equal(xs, xw) and rs["inner"] == rw["inner"]
        assert (L.l1ls_power_iteration(g, 20, op=L.OP_MATRIX_FREE)
                == L.l1ls_power_iteration(gw, 20, op=L.OP_MATRIX_FREE))
    finally:
        gw.free()


@pytest.mark.parametrize("cfg", CASES[:2])
def test_fista_matrix_free_fp32_and_fp64_certificate(cfg):
    # FP32 bulk on both operators: the same tolerance to the FP64 oracle
    # (tests/fp32_bounds.py), and the FP64 certificate the solve returns
    # (P and D at its x) against the oracle's P and D at the oracle's iterate,
    # within what the distance between the two iterates allows:
    # |P(x) - P(x')| <= tau ||d||_1 + ||A^T r'||_2 ||d||_2 + ||d||_2^2 / 2
    # with d = x - x', ||A|| = 1 and ||d||_inf <= bound.
    g, o, A = pair(cfg)
    iters = 50
    mv, rmv = (lambda v: A @ v), (lambda v: A.T @ v)
    ref, bound = fp32_trajectory_bound(A, o.b, o.tau, 1.0, iters)
    Pr, Dr, _ = F.duality_gap(mv, rmv, o.b, o.tau, ref)
    rr = A @ ref - o.b
    for op in (L.OP_STORED, L.OP_MATRIX_FREE):
        x, rep, _ = L.l1ls_solve_fista(g, max_iter=iters, rel_gap_tol=0.0, check_every=5, precision=L.F32, op=op)
        d = x.cpu().numpy() - ref
        err = np.abs(d).max()
        print(f"op {op}: max |x - x_oracle| {err:.3e} (bound {bound:.3e})", flush=True)
        assert err <= bound
        d1, d2 = o.n * bound, math.sqrt(o.n) * bound
        tolP = o.tau * d1 + float(np.linalg.norm(rmv(rr))) * d2 + 0.5 * d2 * d2 + 1e-12 * abs(Pr)
        assert abs(rep["primal"] - Pr) <= tolP, (rep["primal"], Pr, tolP)
        # D = -theta^2 ||r||^2 / 2 - theta b^T r: with theta fixed it moves by at
        # most (||r|| + ||b||) ||A d||, and theta = min(1, tau / ||A^T r||_inf)
        # by at most theta ||d||_2 / ||A^T r||_inf <= ||d||_2 / tau, times
        # ||r|| (||r|| + ||b||); twice the first-order sum
        nr, nb = float(np.linalg.norm(rr)), float(np.linalg.norm(o.b))
        tolD = 2.0 * ((nr + nb) + nr * (nr + nb) / o.tau) * d2 + 1e-12 * abs(Dr)
        assert abs(rep["dual"] - Dr) <= tolD, (rep["dual"], Dr, tolD)


@pytest.mark.parametrize("cfg", CASES[:2])
def test_fista_trajectory_fp32(cfg):
    # FP32 bulk against the FP64 oracle, within the tolerance the oracle
    # derives from its own response to A and b rounded to FP32
    # (tests/fp32_bounds.py).
    g, o, A = pair(cfg)
    iters = 50
    x, rep, _ = L.l1ls_solve_fista(g, max_iter=iters, rel_gap_tol=0.0, check_every=5, precision=L.F32)
    ref, bound = fp32_trajectory_bound(A, o.b, o.tau, 1.0, iters)
    err = np.abs(x.cpu().numpy() - ref).max()
    print(f"max |x - x_oracle| {err:.3e} (bound {bound:.3e})", flush=True)
    assert err <= bound


@pytest.mark.parametrize("cfg", CASES)
def test_fista_internal_gap_matches_oracle(cfg):
    # The device gap at iteration k uses P(x_k) and the dual point from
    # r_y,k = A y_k - b (the residual the k-th gradient was taken at).
    g, o, A = pair(cfg)
    k = 20
    fs = L.Fista(g, rel_gap_tol=0.0, check_every=k, precision=L.F64)
    fs.iterate(k)
    rep = fs.report()
    fs.destroy()
    mv, rmv = (lambda v: A @ v), (lambda v: A.T @ v)
    xk, yk = F.fista(mv, rmv, o.b, o.tau, 1.0, k, return_y=True)
    Pr = F.primal(mv, o.b, o.tau, xk)
    Dr = F.dual_value(rmv, o.b, o.tau, A @ yk - o.b)
    assert math.isclose(rep["primal"], Pr, rel_tol=1e-11)
    assert math.isclose(rep["dual"], Dr, rel_tol=1e-11, abs_tol=1e-9 * abs(Pr))


def test_fista_converges_to_planted_solution_fp64():
    g, o, A = pair(C1)
    x, rep, st = L.l1ls_solve_fista(g, max_iter=20000, rel_gap_tol=1e-12, check_every=32, precision=L.F64)
    assert st == L.L1LS_OK and rep["converged"] == 1
    err = np.linalg.norm(x.cpu().numpy() - o.xstar) / np.linalg.norm(o.xstar)
    assert math.isclose(err, rep["rel_err"], rel_tol=1e-6)
    assert rep["rel_gap"] <= 1e-11 and err <= 1e-3
    # early exit: the iterate returned is the one at which the test passed
    assert rep["iterations"] % 32 == 0 and rep["iterations"] < 20000


def test_fista_tau_above_threshold_gives_zero():
    g, o, A = pair(CASES[1])
    tau = 1.001 * np.abs(A.T @ o.b).max()
    x, rep, _ = L.l1ls_solve_fista(g, tau=tau, max_iter=40, rel_gap_tol=0.0, check_every=8, precision=L.F64)
    assert np.array_equal(x.cpu().numpy(), np.zeros(o.n))


def test_fista_warm_start_at_solution_stays():
    g, o, A = pair(C1)
    x, rep, _ = L.l1ls_solve_fista(g, x0=_dev(o.xstar), max_iter=10, rel_gap_tol=0.0, check_every=1,
                                   precision=L.F64)
    assert np.abs(x.cpu().numpy() - o.xstar).max() <= 1e-12 * max(1.0, np.abs(o.xstar).max())


def test_stepping_equals_single_solve():
    g, o, A = pair(CASES[1])
    x1, _, _ = L.l1ls_solve_fista(g, max_iter=64, rel_gap_tol=0.0, check_every=16, precision=L.F32)
    fs = L.Fista(g, rel_gap_tol=0.0, check_every=16, precision=L.F32)
    for _ in range(4):
        fs.iterate(16)
    x2 = fs.get_x()
    fs.destroy()
    assert torch.equal(x1, x2)


def test_repeat_runs_are_bitwise_identical():
    g, o, A = pair(C1)
    a, _, _ = L.l1ls_solve_fista(g, max_iter=200, rel_gap_tol=0.0, check_every=50, precision=L.F32)
    b, _, _ = L.l1ls_solve_fista(g, max_iter=200, rel_gap_tol=0.0, check_every=50, precision=L.F32)
    assert torch.equal(a, b)


def test_nonfinite_warm_start_reported():
    g, o, A = pair(CASES[1])
    x0 = np.zeros(o.n)
    x0[3] = np.nan
    with pytest.raises(L.L1lsError) as ei:
        L.l1ls_solve_fista(g, x0=_dev(x0), max_iter=8, rel_gap_tol=0.0, check_every=4, precision=L.F64)
    assert ei.value.status == -4


@pytest.mark.parametrize("cfg", [CASES[0], CASES[1]])
def test_tile_schedule_variants_are_bitwise_equal(cfg):
    # every tile schedule the autotuner can pick for the stored FP32 passes
    # computes the same values in the same order
    g, o, A = pair(cfg)
    kr = "fista_f32_residual/%d" % int(np.ceil(np.log2(o.m)))
    kt = "fista_f32_transpose/%d" % int(np.ceil(np.log2(o.n)))
    old = (L.tune_get(kr), L.tune_get(kt))
    ref = None
    try:
        for vr, vt in ((0, 0), (1, 1), (2, 2), (3, 3), (1, 3), (3, 0)):
            L.tune_set(kr, vr)
            L.tune_set(kt, vt)
            x, rep, _ = L.l1ls_solve_fista(g, max_iter=40, rel_gap_tol=0.0, check_every=8, precision=L.F32)
            if ref is None:
                ref = (x, rep["primal"])
            assert torch.equal(x, ref[0]) and rep["primal"] == ref[1], (vr, vt)
    finally:
        L.tune_set(kr, old[0])
        L.tune_set(kt, old[1])
