"""The allocation-free FP64 gap (l1ls_objective_gap_noalloc) through the C ABI.

It runs the kernels of l1ls_objective_gap with their temporaries in the
library's fixed scratch array.  Two calls in a row, the second on a smaller
instance, must give what l1ls_objective_gap gives on the same x, and the
oracle's FP64 duality gap of problem (1) within rounding; instances above the
stated limit are refused before any device work.
"""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1503_03520_amd as L  # noqa: E402
import seeded_inputs as SI  # noqa: E402
from oracle import fista as F  # noqa: E402
from oracle import instance as OI  # noqa: E402

pytestmark = pytest.mark.gpu

# largest m the entry point accepts (its scratch array is sized for it)
MAX_M = 1 << 19


def _gap_pair(cfg, seed_x):
    m, n, kappa, s, tau, seed, rounds = cfg
    print(f"\n[case] noalloc gap m={m} n={n} kappa={kappa} s={s} seed={seed} rounds={rounds}", flush=True)
    g = L.l1ls_generate(m, n, kappa, s, tau, seed, rounds=rounds)
    x_np = SI.sparse_vector(n, max(1, n // 10), seed_x)
    x = torch.from_numpy(x_np).cuda()
    ref = L.l1ls_objective_gap(g, tau, x)
    got = L.l1ls_objective_gap_noalloc(g, tau, x)
    o = OI.Instance(m, n, kappa, s, tau, seed, rounds=rounds)
    A = o.sparse_A()
    orc = F.duality_gap(lambda v: A @ v, lambda v: A.T @ v, o.b, tau, x_np)
    g.free()
    return ref, got, orc


def _close(a, b, rel):
    return abs(a - b) <= rel * max(abs(a), abs(b), 1e-300)


def test_noalloc_gap_equals_allocating_gap_twice_second_smaller():
    big = (1 << 14, 1 << 13, 1e3, 80, 0.7, 1503035301, 2)   # many tiles, two stages
    small = (1010, 502, 1e2, 7, 1.3, 1503035302, 1)          # ragged tail, smaller
    for cfg, sx in ((big, 11), (small, 12)):
        ref, got, orc = _gap_pair(cfg, sx)
        # same kernels and the same order of the final sums: equal to rounding
        for a, b in zip(ref, got):
            assert _close(a, b, 1e-14), (cfg, ref, got)
        # the oracle's FP64 gap at the same x (P, D within a few ulps of sums
        # over m terms; the relative gap through (P - D) / |P|)
        assert _close(got[0], orc[0], 1e-12), (got, orc)
        assert _close(got[1], orc[1], 1e-12), (got, orc)
        assert abs(got[2] - orc[2]) <= 1e-12 * max(1.0, abs(orc[2])), (got, orc)


def test_noalloc_gap_at_planted_minimiser_is_zero():
    cfg = (4096, 2048, 1e2, 20, 1.0, 1503035303, 2)
    g = L.l1ls_generate(*cfg[:6], rounds=cfg[6])
    xs = torch.from_numpy(L.device_to_numpy(g.info().x_star_dev, cfg[1], np.float64)).cuda()
    P, D, gap = L.l1ls_objective_gap_noalloc(g, cfg[4], xs)
    assert abs(P - g.info().f_star) <= 1e-12 * abs(P)
    assert abs(gap) <= 1e-12
    g.free()


def test_noalloc_gap_refuses_instances_above_its_limit():
    m, n = 2 * MAX_M, MAX_M
    g = L.l1ls_generate(m, n, 10.0, 10, 1.0, 1503035304, rounds=1)
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    P, D, gap = ctypes.c_double(7.0), ctypes.c_double(7.0), ctypes.c_double(7.0)
    st = L.lib().l1ls_objective_gap_noalloc(g.handle, 1.0, ctypes.c_void_p(x.data_ptr()), ctypes.byref(P),
                                            ctypes.byref(D), ctypes.byref(gap), None)
    assert st == -1
    assert (P.value, D.value, gap.value) == (7.0, 7.0, 7.0)
    # the allocating entry point takes the same instance
    assert L.l1ls_objective_gap(g, 1.0, x)[0] > 0
    g.free()
