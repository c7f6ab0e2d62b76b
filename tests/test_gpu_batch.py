"""Batched FISTA on the GPU: parity with the single-instance path and the oracle.

A slot's iterates are computed by the same tile products, in the same order,
as the single-instance FP32 path, so after the same number of iterations they
agree bit for bit; and a slot's result does not depend on the other resident
slots (alone vs in a mix), including the iteration at which its gap test
passes.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1503_03520_amd as L  # noqa: E402
from fp32_bounds import fp32_trajectory_bound  # noqa: E402
from oracle import fista as F  # noqa: E402
from oracle import instance as OI  # noqa: E402

pytestmark = pytest.mark.gpu

# uneven sizes, both stage counts, several kappa (m = 2n, s = n/100)
CFGS = [
    (2048, 1024, 1e2, 10, 1.0, 101, 2),
    (2 * 1502, 1502, 1e3, 15, 1.0, 102, 2),
    (8192, 4096, 1e4, 40, 0.5, 103, 2),
    (1030, 514, 1e2, 5, 1.0, 104, 1),
    (16384, 8192, 1e5, 81, 1.0, 105, 2),
]
_gen = {}


def gen(cfg):
    if cfg not in _gen:
        m, n, kappa, s, tau, seed, r = cfg
        print(f"\n[case] batch instance m={m} n={n} kappa={kappa} seed={seed} rounds={r}", flush=True)
        _gen[cfg] = L.l1ls_generate(m, n, kappa, s, tau, seed, rounds=r)
    return _gen[cfg]


def test_batch_equals_single_path_bitwise():
    iters = 70
    insts = [gen(c) for c in CFGS]
    xs, reps, _ = L.l1ls_solve_fista_batched(insts, max_iter=iters, rel_gap_tol=0.0, check_every=10,
                                             precision=L.F32)
    for inst, x, rep in zip(insts, xs, reps):
        x1, r1, _ = L.l1ls_solve_fista(inst, max_iter=iters, rel_gap_tol=0.0, check_every=10, precision=L.F32)
        assert rep["iterations"] == iters
        assert torch.equal(x, x1)


def test_batch_matches_oracle_fp32_bound():
    iters = 40
    cfg = CFGS[2]
    inst = gen(cfg)
    xs, reps, _ = L.l1ls_solve_fista_batched([inst], max_iter=iters, rel_gap_tol=0.0, check_every=8,
                                             precision=L.F32)
    m, n, kappa, s, tau, seed, r = cfg
    o = OI.Instance(m, n, kappa, s, tau, seed, rounds=r)
    A = o.sparse_A()
    ref, bound = fp32_trajectory_bound(A, o.b, tau, 1.0, iters)
    assert np.abs(xs[0].cpu().numpy() - ref).max() <= bound


def _run_alone(cfg, tol, check, max_iter):
    B = L.Batch(1, rel_gap_tol=tol, check_every=check, precision=L.F32)
    s = B.add(gen(cfg))
    for _ in range(max_iter // check):
        B.iterate(check)
        reps, act = B.poll()
        if act == 0:
            break
    x = B.get_x(s)
    rep = B.poll()[0][s]
    B.destroy()
    return x, rep


def test_alone_equals_in_mix_with_late_admission():
    tol, check, max_iter = 1e-6, 16, 2000
    B = L.Batch(8, rel_gap_tol=tol, check_every=check, precision=L.F32)
    slots = {}
    slots[0] = B.add(gen(CFGS[0]))
    slots[2] = B.add(gen(CFGS[2]))
    B.iterate(37)                         # the others join mid-flight
    slots[1] = B.add(gen(CFGS[1]))
    slots[3] = B.add(gen(CFGS[3]))
    B.iterate(5)
    slots[4] = B.add(gen(CFGS[4]))
    for _ in range(max_iter // check + 4):
        B.iterate(check)
        reps, act = B.poll()
        if act == 0:
            break
    reps, act = B.poll()
    for q, cfg in enumerate(CFGS):
        xa, ra = _run_alone(cfg, tol, check, max_iter + 64)
        xm = B.get_x(slots[q])
        rm = reps[slots[q]]
        assert rm["converged"] == ra["converged"]
        assert rm["iterations"] == ra["iterations"], (q, rm["iterations"], ra["iterations"])
        assert torch.equal(xa, xm)
    B.destroy()


def test_remove_and_reuse_slot():
    B = L.Batch(2, rel_gap_tol=0.0, check_every=8, precision=L.F32)
    a = B.add(gen(CFGS[0]))
    b = B.add(gen(CFGS[1]))
    B.iterate(16)
    B.remove(a)
    c = B.add(gen(CFGS[3]))
    assert c == a
    B.iterate(24)
    reps, _ = B.poll()
    assert reps[b]["iterations"] == 40 and reps[c]["iterations"] == 24
    xc = B.get_x(c)
    x1, _, _ = L.l1ls_solve_fista(gen(CFGS[3]), max_iter=24, rel_gap_tol=0.0, check_every=8, precision=L.F32)
    assert torch.equal(xc, x1)
    B.destroy()


def test_admission_budget_and_capacity():
    fp = [L.instance_footprint(gen(c)) for c in CFGS[:3]]
    B = L.Batch(2, hbm_budget_bytes=fp[0] + fp[1] // 2, rel_gap_tol=0.0, check_every=8, precision=L.F32)
    assert B.try_add(gen(CFGS[0])) == 0
    assert B.try_add(gen(CFGS[1])) is None      # over the HBM budget
    B.destroy()
    B = L.Batch(1, rel_gap_tol=0.0, check_every=8, precision=L.F32)
    assert B.try_add(gen(CFGS[0])) == 0
    assert B.try_add(gen(CFGS[1])) is None      # no free slot
    B.destroy()


def test_batched_solve_converges_all():
    insts = [gen(c) for c in CFGS]
    xs, reps, st = L.l1ls_solve_fista_batched(insts, max_iter=20000, rel_gap_tol=1e-5, check_every=16,
                                              precision=L.F32)
    assert st == L.L1LS_OK
    for inst, x, rep in zip(insts, xs, reps):
        assert rep["converged"] == 1 and rep["rel_gap"] <= 1e-5
        P, D, gap = L.l1ls_objective_gap(inst, inst.params["tau"], x)
        assert gap <= 2e-5      # FP64 certificate of the FP32 iterate


def test_tile_schedule_does_not_change_results():
    # rounds of tiles per workgroup task (fixed, or chosen by the autotuner)
    # only regroup the same per-tile work
    iters = 40
    insts = [gen(c) for c in CFGS[:4]]
    ref = None
    for chunk in (0, 1, 3, 8):
        xs, reps, _ = L.l1ls_solve_fista_batched(insts, max_iter=iters, rel_gap_tol=0.0, check_every=8,
                                                 precision=L.F32, tile_chunk=chunk)
        if ref is None:
            ref = (xs, reps)
            continue
        for a, b, ra, rb in zip(ref[0], xs, ref[1], reps):
            assert torch.equal(a, b), chunk
            assert ra["rel_gap"] == rb["rel_gap"] and ra["primal"] == rb["primal"], chunk


def _drive(graph, tol, check):
    """The same admission sequence with and without graph replay; eager
    polls, copies and another solve run between the replays."""
    B = L.Batch(6, rel_gap_tol=tol, check_every=check, precision=L.F32, graph=graph)
    slots = [B.add(gen(CFGS[0])), B.add(gen(CFGS[2]))]
    seen = []
    B.iterate(3 * check + 5)                 # three whole periods, then five launched one by one
    seen.append(B.poll())
    slots.append(B.add(gen(CFGS[1])))        # the resident set changes: a new period is captured
    B.iterate(2 * check)
    x0 = B.get_x(slots[0])
    L.l1ls_solve_fista(gen(CFGS[3]), max_iter=8, rel_gap_tol=0.0, check_every=8, precision=L.F32)
    seen.append(B.poll())
    B.remove(slots[1])
    slots.append(B.add(gen(CFGS[4])))
    for _ in range(6):
        B.iterate(check)
        seen.append(B.poll())
    xs = [B.get_x(s) for s in (slots[0], slots[2], slots[3])]
    B.destroy()
    return x0, xs, seen


@pytest.mark.parametrize("tol", [0.0, 1e-5])
def test_graph_replay_equals_launched_iterations(tol):
    # the kernels of a captured check period read the iteration count and
    # the momentum table from device memory, so replaying the graph computes
    # what launching each kernel computes, bit for bit, replay after replay
    check = 8
    xa0, xa, seen_a = _drive(0, tol, check)
    xb0, xb, seen_b = _drive(1, tol, check)
    assert torch.equal(xa0, xb0)
    for a, b in zip(xa, xb):
        assert torch.equal(a, b)
    for (ra, aa), (rb, ab) in zip(seen_a, seen_b):
        assert aa == ab
        for p, q in zip(ra, rb):
            assert (p["iterations"], p["converged"], p["primal"], p["dual"], p["rel_gap"]) == \
                   (q["iterations"], q["converged"], q["primal"], q["dual"], q["rel_gap"])


@pytest.mark.parametrize("graph", [0, 1])
def test_persistent_small_slots_equal_shared_passes(graph):
    # Slots with few rows run every iteration of an iterate call in one
    # workgroup (kb_persist); with persist_rows = -1 they take the shared
    # passes, with 4096 the slots of at most 4096 rows and with 1 << 20 every
    # slot here runs in one workgroup.  All three
    # give the same iterates and stop at the same iteration, bit for bit,
    # with late admission and a removal between calls.
    def drive(persist_rows):
        B = L.Batch(6, rel_gap_tol=1e-5, check_every=8, precision=L.F32, graph=graph,
                    persist_rows=persist_rows)
        s = [B.add(gen(CFGS[0])), B.add(gen(CFGS[4]))]
        B.iterate(13)
        s.append(B.add(gen(CFGS[3])))
        s.append(B.add(gen(CFGS[1])))
        B.iterate(40)
        B.remove(s[1])
        for _ in range(40):
            B.iterate(16)
            if B.poll()[1] == 0:
                break
        reps = B.poll()[0]
        out = [(B.get_x(q), reps[q]["iterations"], reps[q]["converged"], reps[q]["rel_gap"]) for q in (s[0], s[2], s[3])]
        B.destroy()
        return out

    ref = drive(-1)
    for rows in (4096, 1 << 20):
        got = drive(rows)
        for (xa, ia, ca, ga), (xb, ib, cb, gb) in zip(ref, got):
            assert (ia, ca, ga) == (ib, cb, gb), rows
            assert torch.equal(xa, xb), rows
    # and the single path at the same tolerance and check period
    for (x, it, conv, _), cfg in zip(ref, (CFGS[0], CFGS[3], CFGS[1])):
        x1, r1, _ = L.l1ls_solve_fista(gen(cfg), max_iter=it, rel_gap_tol=1e-5, check_every=8, precision=L.F32)
        assert torch.equal(x, x1)
