"""GPU parity of the batched and regularisation-path workloads at their full
sizes, in the launch configuration the benchmark times (FP32 bulk, gap
checks every 16 iterations), over a fixed number of iterations so that
every result can be set beside the oracle's FP64 FISTA at the same count.

- Batched: the 256 instances the benchmark draws (n log-uniform in
  [2^10, 2^16], m = 2n, kappa in {1e2, ..., 1e6}, s = n/100, two stages) in
  one batch; a sample of them (the smallest, the largest and every 32nd)
  against the oracle, all of them against the single-solve path bitwise.
- Path: n = 2^16, m = 2^17, kappa = 1e4, 64 tau values log-spaced over
  [1e-3, 1] ||A^T b||_inf as one sparse-times-dense iteration; every column
  against the oracle.
The FP32 bound is that of the single path (tests/fp32_bounds.py).
"""
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1503_03520_amd as L  # noqa: E402
from fp32_bounds import fp32_trajectory_bound  # noqa: E402
from oracle import fista as F  # noqa: E402
from oracle import instance as OI  # noqa: E402

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402

pytestmark = pytest.mark.gpu

ITERS = 48
CHECK = 16


def test_batched_workload_full_size():
    cfgs = bench.batched_configs(256)
    print(f"\n[case] batched workload: {len(cfgs)} instances, n {min(c[1] for c in cfgs)}.."
          f"{max(c[1] for c in cfgs)}", flush=True)
    insts = [L.l1ls_generate(*c[:6], rounds=c[6], storage=L.STORE_F32) for c in cfgs]
    kw = dict(max_iter=ITERS, rel_gap_tol=0.0, check_every=CHECK, precision=L.F32)
    xs, reps, _ = L.l1ls_solve_fista_batched(insts, **kw)
    assert all(r["iterations"] == ITERS for r in reps)
    order = sorted(range(len(cfgs)), key=lambda j: cfgs[j][1])
    sample = sorted({order[0], order[-1], *range(0, len(cfgs), 32)})
    for j in sample:
        m, n, kappa, s, tau, seed, r = cfgs[j]
        o = OI.Instance(m, n, kappa, s, tau, seed, rounds=r)
        A = o.sparse_A()
        ref, bound = fp32_trajectory_bound(A, o.b, o.tau, 1.0, ITERS)
        err = np.abs(xs[j].cpu().numpy() - ref).max()
        print(f"instance {j}: n={n} kappa={kappa:g} max err {err:.3e} (bound {bound:.3e})", flush=True)
        assert err <= bound, j
    # every slot computes what the single path computes
    for j, inst in enumerate(insts):
        x1, _, _ = L.l1ls_solve_fista(inst, polish=0, **kw)
        assert torch.equal(x1, xs[j]), j


def test_path_workload_full_size():
    n = 1 << 16
    m, kappa, s, tau, seed = 2 * n, 1e4, n // 100, 1.0, 1503035203
    print(f"\n[case] path workload m={m} n={n} kappa={kappa} seed={seed}", flush=True)
    g = L.l1ls_generate(m, n, kappa, s, tau, seed, rounds=2)
    o = OI.Instance(m, n, kappa, s, tau, seed, rounds=2)
    A = o.sparse_A()
    tmax = float(np.abs(A.T @ o.b).max())
    taus = np.geomspace(1e-3, 1.0, 64) * tmax
    X, reps, _ = L.l1ls_solve_fista_path(g, taus, max_iter=ITERS, rel_gap_tol=0.0, check_every=CHECK,
                                         precision=L.F32)
    Xh = X.cpu().numpy()
    worst = 0.0
    for c, t in enumerate(taus):
        ref, bound = fp32_trajectory_bound(A, o.b, float(t), 1.0, ITERS)
        err = np.abs(Xh[c] - ref).max()
        worst = max(worst, err)
        assert err <= bound, c
        assert reps[c]["iterations"] == ITERS
    print(f"path: worst column error {worst:.3e} (bound {bound:.3e})", flush=True)


def test_serving_workload_full_size_requests_equal_single_path():
    # Requests as the serving benchmark draws them (n log-uniform in
    # [2^10, 2^22], kappa log-uniform in [1e2, 1e6], tau log-uniform in
    # [1e-2, 1], two stages), its scheduler settings (256 slots, 160 GiB
    # budget, 16 iterations per tick, gap checks every 16, tolerance 1e-6,
    # cap 5000): the three largest and three smallest of the first 40 and
    # four others, served together.  Each result equals the single-instance
    # FP32 path on the same instance bit for bit (the single path is held to
    # the oracle at full size in test_gpu_fullsize.py).
    reqs = bench.serve_requests(40, 1503035204)
    order = sorted(range(len(reqs)), key=lambda i: reqs[i]["n"])
    pick = sorted(set(order[:3] + order[-3:] + [0, 10, 20, 30]))
    tol, check, cap = 1e-6, 16, 5000
    print(f"\n[case] serving: requests {pick}, n = {[reqs[i]['n'] for i in pick]}", flush=True)
    S = L.Server(256, hbm_budget_bytes=160 << 30, iters_per_tick=16, check_every=check)
    ids = {}
    for i in pick:
        r = reqs[i]
        ids[S.submit(r["m"], r["n"], r["kappa"], r["s"], r["tau"], r["seed"], rounds=r["rounds"],
                     rel_gap_tol=tol, max_iter=cap)] = i
    out, ticks = {}, 0
    while len(out) < len(pick):
        S.tick()
        ticks += 1
        for rid in S.completed():
            out[ids[rid]] = S.take(rid)
        assert ticks < 100000
    S.destroy()
    for i in pick:
        r = reqs[i]
        inst = L.l1ls_generate(r["m"], r["n"], r["kappa"], r["s"], r["tau"], r["seed"], rounds=r["rounds"],
                               storage=L.STORE_F32)
        x1, r1, _ = L.l1ls_solve_fista(inst, max_iter=cap, rel_gap_tol=tol, check_every=check, precision=L.F32,
                                       polish=0)
        xs, rs = out[i]
        print(f"request {i}: n={r['n']} iterations {rs['iterations']} converged {rs['converged']}", flush=True)
        assert rs["iterations"] == r1["iterations"] and rs["converged"] == r1["converged"], i
        assert torch.equal(xs, x1), i
        inst.free()
