"""Windowed gathers of the stored FP32 passes (L1LS_STORE_WINDOWS): the
same FISTA iteration as the plain stored passes, bit for bit, on instances
with several windows and source chunks per pass (and a ragged one with a
single partial chunk), and the same iterate as the oracle's FP64 FISTA
within the FP32 tolerance."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1503_03520_amd as L  # noqa: E402
from fp32_bounds import fp32_trajectory_bound  # noqa: E402
from oracle import instance as OI  # noqa: E402

pytestmark = pytest.mark.gpu

CASES = [
    (2 * (1 << 20), 1 << 20, 1e4, (1 << 20) // 100, 1.0, 1503035201, 2),   # 16 row windows, 64 x chunks
    (1 << 18, 1 << 17, 1e3, 1310, 0.7, 31, 2),
    (1010, 502, 1e3, 7, 0.5, 17, 2),                                       # one window, one partial chunk
    (600, 300, 1.0, 5, 1.0, 8, 1),
]


@pytest.mark.parametrize("cfg", CASES)
def test_windowed_passes_are_bitwise_the_plain_ones(cfg):
    m, n, kappa, s, tau, seed, r = cfg
    print(f"\n[case] windows m={m} n={n} kappa={kappa} rounds={r}", flush=True)
    plain = L.l1ls_generate(m, n, kappa, s, tau, seed, rounds=r, storage=L.STORE_F32 | L.STORE_F64)
    win = L.l1ls_generate(m, n, kappa, s, tau, seed, rounds=r, storage=L.STORE_F32 | L.STORE_F64 | L.STORE_WINDOWS)
    for iters, check in ((1, 1), (37, 8), (64, 32)):
        a, ra, _ = L.l1ls_solve_fista(plain, max_iter=iters, rel_gap_tol=0.0, check_every=check, precision=L.F32)
        b, rb, _ = L.l1ls_solve_fista(win, max_iter=iters, rel_gap_tol=0.0, check_every=check, precision=L.F32)
        assert torch.equal(a, b), iters
        assert ra["primal"] == rb["primal"] and ra["rel_gap"] == rb["rel_gap"], iters
    # the stepping interface reports the bucketing passes in slots 3 and 4
    fs = L.Fista(win, precision=L.F32, rel_gap_tol=0.0, check_every=8, time_kernels=1)
    fs.iterate(16)
    ms, cnt = fs.kernel_times(5)
    fs.destroy()
    assert cnt[0] == 17 and cnt[1] == 16 and cnt[3] == 17 and cnt[4] == 16
    if n <= 1 << 17:
        o = OI.Instance(m, n, kappa, s, tau, seed, rounds=r)
        A = o.sparse_A()
        ref, bound = fp32_trajectory_bound(A, o.b, tau, 1.0, 64)
        x, _, _ = L.l1ls_solve_fista(win, max_iter=64, rel_gap_tol=0.0, check_every=32, precision=L.F32)
        assert np.abs(x.cpu().numpy() - ref).max() <= bound
    plain.free()
    win.free()


def test_windowed_solve_to_tolerance_and_polish():
    cfg = CASES[1]
    m, n, kappa, s, tau, seed, r = cfg
    win = L.l1ls_generate(m, n, kappa, s, tau, seed, rounds=r, storage=L.STORE_F32 | L.STORE_F64 | L.STORE_WINDOWS)
    x, rep, st = L.l1ls_solve_fista(win, max_iter=2000, rel_gap_tol=1e-8, check_every=32, precision=L.F32, polish=1)
    assert rep["rel_gap"] <= 1e-8 and rep["rel_err"] <= 1e-9
    win.free()


def test_windowed_tile_schedules_are_bitwise_the_plain_passes():
    # every tile schedule the autotuner can pick for the windowed passes (its
    # own cache keys) gives the plain passes' iterates bit for bit
    m, n, kappa, s, tau, seed, r = CASES[1]
    plain = L.l1ls_generate(m, n, kappa, s, tau, seed, rounds=r, storage=L.STORE_F32)
    win = L.l1ls_generate(m, n, kappa, s, tau, seed, rounds=r, storage=L.STORE_F32 | L.STORE_WINDOWS)
    kr = "fista_f32_residual_win/%d" % int(np.ceil(np.log2(m)))
    kt = "fista_f32_transpose_win/%d" % int(np.ceil(np.log2(n)))
    old = (L.tune_get(kr), L.tune_get(kt))
    ref, rref, _ = L.l1ls_solve_fista(plain, max_iter=40, rel_gap_tol=0.0, check_every=8, precision=L.F32)
    try:
        for vr, vt in ((0, 0), (1, 1), (2, 2), (3, 3), (2, 1)):
            L.tune_set(kr, vr)
            L.tune_set(kt, vt)
            x, rep, _ = L.l1ls_solve_fista(win, max_iter=40, rel_gap_tol=0.0, check_every=8, precision=L.F32)
            assert torch.equal(x, ref) and rep["primal"] == rref["primal"], (vr, vt)
    finally:
        L.tune_set(kr, old[0])
        L.tune_set(kt, old[1])
    plain.free()
    win.free()
