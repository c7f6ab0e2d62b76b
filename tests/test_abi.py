"""C-ABI library: loads, exports every declared symbol, rejects bad arguments.

Runs without a GPU: the argument checks of the entry points return before
any HIP call is made.
"""
import ctypes
import os
import re

import pytest

import paper_1503_03520_amd as L

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "l1ls.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(l1ls_[a-z0-9_]+)\s*\(", text)))


def test_header_and_binding_agree():
    declared = _declared_functions()
    assert declared, "no declarations parsed"
    assert sorted(L.EXPORTED) == declared


def test_library_exports_every_declared_symbol():
    lib = L.lib()
    for name in _declared_functions():
        assert hasattr(lib, name), name
    assert lib.l1ls_version() == 1


def test_status_strings():
    lib = L.lib()
    for code in (0, 1, -1, -2, -3, -4, -5, -6):
        assert lib.l1ls_status_string(code)


@pytest.mark.parametrize("m,n,kappa,s,tau,rounds", [
    (101, 50, 10.0, 1, 1.0, 1),     # m odd
    (100, 51, 10.0, 1, 1.0, 1),     # n odd
    (100, 50, 0.5, 1, 1.0, 1),      # kappa < 1
    (100, 50, 10.0, 51, 1.0, 1),    # s > n
    (100, 50, 10.0, -1, 1.0, 1),    # s < 0
    (100, 50, 10.0, 1, 0.0, 1),     # tau <= 0
    (100, 50, 10.0, 1, float("nan"), 1),
    (100, 50, float("inf"), 1, 1.0, 1),
    (100, 50, 10.0, 1, 1.0, 3),     # rounds > 2
    (100, 50, 10.0, 1, 1.0, 0),
    (2, 0, 10.0, 0, 1.0, 1),        # n < 2
])
def test_generate_rejects_invalid_arguments(m, n, kappa, s, tau, rounds):
    h = ctypes.c_void_p()
    o = L.GenOpts(rounds, 3, None, 1)
    st = L.lib().l1ls_generate_ex(m, n, kappa, s, tau, 1, ctypes.byref(o), ctypes.byref(h))
    assert st == -1 and not h.value


@pytest.mark.parametrize("m,n,kappa,s,rounds,storage,status", [
    (101, 200, 10.0, 1, 1, 3, -1),                        # IGen2 (m < n): m odd
    (0, 200, 10.0, 0, 1, 3, -1),                          # ... m < 2
    (100, 200, 10.0, 101, 1, 3, -1),                      # ... s > m
    (100, 200, 0.5, 1, 1, 3, -1),                         # ... kappa < 1
    (100, 200, 10.0, 1, 2, 3, -6),                        # ... one stage only
    (100, 200, 10.0, 1, 1, 0, -6),                        # ... a stored operator
    (100, 200, 10.0, 1, 1, 3 | 8, -6),                    # ... no matrix-free tables
])
def test_generate_igen2_argument_checks(m, n, kappa, s, rounds, storage, status):
    h = ctypes.c_void_p()
    o = L.GenOpts(rounds, storage, None, 1)
    st = L.lib().l1ls_generate_ex(m, n, kappa, s, 1.0, 1, ctypes.byref(o), ctypes.byref(h))
    assert st == status and not h.value


@pytest.mark.parametrize("rounds,storage,layout,n,status", [
    (2, 16, 1, 50, -1),                                   # unknown storage bit
    (1, L.STORE_BLK32, 1, 50, -6),                        # blocks need two stages
    (2, L.STORE_BLK32 | L.STORE_F32, 0, 50, -6),          # ... and the stage layout
    (2, L.STORE_BLK32, 1, 2, -6),                         # ... and n >= 4
])
def test_generate_rejects_unsupported_block_storage(rounds, storage, layout, n, status):
    h = ctypes.c_void_p()
    o = L.GenOpts(rounds, storage, None, layout)
    st = L.lib().l1ls_generate_ex(100, n, 10.0, 1, 1.0, 1, ctypes.byref(o), ctypes.byref(h))
    assert st == status and not h.value


def test_null_arguments_rejected():
    lib = L.lib()
    assert lib.l1ls_generate(100, 50, 10.0, 1, 1.0, 1, None) == -1
    assert lib.l1ls_instance_info(None, None) == -1
    assert lib.l1ls_apply(None, 0, 0, 1, None, None, None) == -1
    assert lib.l1ls_solve_fista(None, None, None, None) == -1
    assert lib.l1ls_solve_cg_newton(None, None, None, None) == -1
    assert lib.l1ls_fista_create(None, None, None) == -1
    assert lib.l1ls_fista_iterate(None, 1) == -1
    lib.l1ls_free(None)
    lib.l1ls_fista_destroy(None)


def test_solve_opts_defaults():
    o = L.SolveOpts()
    L.lib().l1ls_solve_opts_default(ctypes.byref(o))
    assert o.rel_gap_tol == 1e-8 and o.check_every == 32 and o.precision == L.F64
    assert o.mu == 1e-5 and o.pcg_rtol == 0.1 and o.max_backtrack == 50


def test_server_null_and_invalid_arguments():
    lib = L.lib()
    h = ctypes.c_void_p()
    assert lib.l1ls_server_create(0, 0, 16, 16, None, ctypes.byref(h)) == -1      # no slots
    assert lib.l1ls_server_create(4, 0, 0, 16, None, ctypes.byref(h)) == -1       # no iterations per tick
    assert lib.l1ls_server_create(4, 0, 16, 0, None, ctypes.byref(h)) == -1       # no check period
    r = L.Request(2048, 1024, 100.0, 10, 1.0, 1, 2, 0, 1e-5, 1000)
    rid = ctypes.c_int64(-1)
    assert lib.l1ls_server_submit(None, ctypes.byref(r), ctypes.byref(rid)) == -1
    assert lib.l1ls_server_tick(None, None, None) == -1
    assert lib.l1ls_server_take(None, 0, None, None) == -1
    assert lib.l1ls_server_completed(None, None, 0) == 0
    assert lib.l1ls_server_stats(None, None, None, None) == -1
    assert lib.l1ls_batch_add_ex(None, None, 1.0, 1e-5, 10, None) == -1
    lib.l1ls_server_destroy(None)


def test_request_footprint_estimate():
    f = L.request_footprint
    assert f(2048, 1024, rounds=2) > f(2048, 1024, rounds=1) > 0
    assert f(4096, 2048) > f(2048, 1024)
    assert f(2048, 1023) == 0 and f(1024, 2048) == 0 and f(2048, 1024, rounds=3) == 0
    assert f(2048, 1024, rel_gap_tol=0.0) == 0 and f(2048, 1024, max_iter=0) == 0
    assert L.lib().l1ls_request_footprint(None) == 0


def test_sgt_params_default_is_section_8_9():
    p = L.sgt_params(2 ** 30, 7)
    assert (p.n, p.m, p.s) == (2 ** 30, 2 ** 31, 2 ** 20)
    assert p.theta == 2.0 * 3.141592653589793 / 3.0
    assert (p.sigma_odd, p.sigma_even, p.x_neg, p.x_pos, p.tau, p.seed) == (0.1, 100.0, -1.0e4, 0.1, 1.0, 7)
    assert L.sgt_bytes(2 ** 30) >= 8 * 2 ** 30
    assert L.sgt_solve_bytes(2 ** 30) >= 40 * 2 ** 30
    assert L.sgt_bytes(1) == 0 and L.sgt_solve_bytes(0) == 0


@pytest.mark.parametrize("field,value", [
    ("n", 7), ("n", 0), ("n", 2 ** 33), ("m", 2), ("m", 9), ("s", 9), ("s", -1),
    ("sigma_odd", 0.0), ("sigma_even", -1.0), ("tau", 0.0), ("theta", float("nan")),
    ("x_neg", float("inf")), ("tau", float("nan")),
])
def test_sgt_generate_rejects_invalid_arguments(field, value):
    p = L.sgt_params(8, 1)
    setattr(p, field, value)
    h = ctypes.c_void_p()
    st = L.lib().l1ls_sgt_generate(ctypes.byref(p), None, ctypes.byref(h))
    assert st == -1 and not h.value


def test_sgt_null_arguments():
    lib = L.lib()
    h = ctypes.c_void_p()
    assert lib.l1ls_sgt_generate(None, None, ctypes.byref(h)) == -1
    assert lib.l1ls_sgt_describe(None, None) == -1
    assert lib.l1ls_sgt_planted(None, None, None, None) == -1
    assert lib.l1ls_sgt_apply(None, 0, None, None, None) == -1
    d = ctypes.c_double()
    assert lib.l1ls_sgt_objective_gap(None, 1.0, None, ctypes.byref(d), ctypes.byref(d), ctypes.byref(d),
                                       None) == -1
    assert lib.l1ls_sgt_solve_cg_newton(None, None, None, None) == -1
    h2 = ctypes.c_void_p()
    assert lib.l1ls_sgt_newton_create(None, None, None, ctypes.byref(h2)) == -1 and not h2.value
    assert lib.l1ls_sgt_newton_step(None, 1, None) == -1
    lib.l1ls_sgt_newton_destroy(None)
    lib.l1ls_sgt_free(None)


def test_law_validation():
    for kw in (dict(sigma_law=2), dict(xstar_law=3), dict(sigma_law=L.SIGMA_UNIFORM, sigma_shift=0.0),
               dict(xstar_law=L.XSTAR_OSGEN, gamma=0.0), dict(xstar_law=L.XSTAR_OSGEN3, s1=3, s2=3),
               dict(sigma_law=L.SIGMA_UNIFORM, sigma_scale=-1.0),
               dict(m=30),                                   # IGen2 needs n - m <= m
               dict(m=48, xstar_law=L.XSTAR_OSGEN3),         # OsGen3 is for m >= n
               dict(m=48, s=50), dict(m=47)):
        p = L.sgt_params(64, 1, s=kw.pop("s", 4), **kw)
        h = ctypes.c_void_p()
        assert L.lib().l1ls_sgt_generate(ctypes.byref(p), None, ctypes.byref(h)) == -1 and not h.value


def test_generate_rejects_stored_operator_beyond_32bit_gathers():
    # the stored passes gather m-vectors with 32-bit byte offsets
    h = ctypes.c_void_p()
    o = L.GenOpts(2, L.STORE_F32, None, 1)
    st = L.lib().l1ls_generate_ex(1 << 29, 1 << 20, 10.0, 1, 1.0, 1, ctypes.byref(o), ctypes.byref(h))
    assert st == -6 and not h.value


def test_power_iteration_rejects_null_and_bad_counts():
    lam = ctypes.c_double()
    assert L.lib().l1ls_power_iteration(None, 0, 10, None, ctypes.byref(lam), None) == -1
    assert L.lib().l1ls_power_iteration(None, 0, 0, None, ctypes.byref(lam), None) == -1


def test_set_allocator_rejects_missing_callbacks():
    lib = L.lib()
    spec = L.Allocator(L._ALLOC_FN(0), L._FREE_FN(0), None)
    assert lib.l1ls_set_allocator(ctypes.byref(spec)) == -1
    assert lib.l1ls_instance_bytes(None) == 0
