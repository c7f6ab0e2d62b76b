"""Benchmark: FISTA iterations per second on the memory-scale instance.

Workload (default): n = 2^26, m = 2^27, kappa = 1e6, two Givens stages per
side, s = n/1000, x* ~ N(0,1), tau = 1; FP32 bulk iteration on stored CSR +
CSC (FP32 values, int32 indices), FP64 gap partials.  One step = one FISTA
iteration of the whole hot path: the CSR residual pass (A x - b with the
momentum residual), the CSC transpose pass (A^T r, gradient step,
soft-threshold prox, momentum) and, once per check period, the FP64 gap
statistics and the device-side duality-gap test.  The check period divides
both --warmup and --steps, so the timed window holds whole periods.  All
inputs are generated on the device before the timed region.  The matrix-free
and blocked operators, a certified solve (CG-Newton, then the FP64 polish),
the single large instance (n = 2^20) and the small FP64 instance are
reported under "extra".  Other workloads: --workload.

Prints one JSON line.  `--gpus N` with N > 1 exits: the solver runs on one
GPU.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILE_SUMMARY = os.path.join(ROOT, "profiles", "fista_stored_f32_n2p26.txt")


def profile_summary_path(n):
    """The committed counter summary of the FISTA passes at size n."""
    return os.path.join(ROOT, "profiles", "fista_stored_f32_n2p%d.txt" % (n.bit_length() - 1))
KERNEL_SOURCES = ["kernels.hpp", "fista.hip", "common.hpp", "blocks.hip", "window.hip"]


def kernel_source_hash():
    """Hash of the sources the timed kernels are built from."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1503_03520_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_profile_summary(path=PROFILE_SUMMARY):
    """key: value lines of a committed rocprofv3 summary (or None)."""
    if not os.path.exists(path):
        return None
    out = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                out[k.strip()] = v.strip()
    return out


# key: (kernel name pattern, rank of the grid among the pattern's grids,
# largest first).  The plain stored passes run without XCD placement,
# the windowed ones with it; the windowed gathers' bucketing pass runs
# once per side, r_y's (m sources) with the larger grid.
PASS_KERNELS = {"residual": (r"k_residual<float, \d+, (true|false), false>", 0),
                "transpose_prox": (r"k_transpose_prox<float, \d+, (true|false), false>", 0),
                "residual_win": (r"k_residual<float, \d+, (true|false), true>", 0),
                "transpose_prox_win": (r"k_transpose_prox<float, \d+, (true|false), true>", 0),
                "bucket_r_y": (r"k_sw_scatter", 0), "bucket_x": (r"k_sw_scatter", 1),
                "blk_residual": (r"k_blk_residual<false>", 0), "blk_transpose_prox": (r"k_blk_transpose_prox<false>", 0),
                "mf_res_qt": (r"k_mf_res_qt<float, 2, 0, float>", 0), "mf_prox_gt": (r"k_mf_prox_gt<float, 2>", 0),
                "mf_win_scatter": (r"k_win_scatter<float>", 0)}


def write_profile_summary(args):
    """Summarise rocprofv3 CSV output (kernel trace + FETCH_SIZE / WRITE_SIZE runs
    of this script, and the same counters for a plain 1 GiB copy) into a text file."""
    import csv
    import statistics

    def kernel_rows(d, kind):
        for root, _, files in os.walk(d):
            for f in files:
                if f.endswith(kind):
                    return list(csv.DictReader(open(os.path.join(root, f))))
        raise SystemExit(f"no *{kind} under {d}")

    import re

    names = PASS_KERNELS
    # The bench launches these kernels at the headline size and (in the
    # n = 2^20 leg) at a smaller one: each figure is taken over the dispatches
    # with the kernel's largest grid (the headline instance's), or the grid
    # of the given rank.
    trace = kernel_rows(args.kt, "kernel_trace.csv")

    def grid_of(r):
        return int(r.get("Grid_Size_X") or r.get("Grid_Size") or 0)

    dur = {}
    big = {}
    for key, (pat, rank) in names.items():
        rows = [r for r in trace if re.search(pat, r["Kernel_Name"])]
        grids = sorted({grid_of(r) for r in rows}, reverse=True)
        if len(grids) <= rank:
            continue
        g = grids[rank]
        rows = [r for r in rows if grid_of(r) == g]
        ns = [int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in rows]
        dur[key] = (sum(ns) / len(ns), len(ns))
        big[key] = g

    def counter(d, cname, pat, grid=None):
        vals = [float(r["Counter_Value"]) for r in kernel_rows(d, "counter_collection.csv")
                if re.search(pat, r["Kernel_Name"]) and r["Counter_Name"] == cname
                and (grid is None or int(r.get("Grid_Size") or 0) == grid)]
        return statistics.median(vals), len(vals)

    copy_f, _ = counter(args.copyf, "FETCH_SIZE", "copyBuffer")
    copy_w, _ = counter(args.copyw, "WRITE_SIZE", "copyBuffer")
    gib_kib = float(1 << 20)            # the copy moves 1 GiB = 2^20 KiB each way
    f_scale, w_scale = gib_kib / copy_f, gib_kib / copy_w
    kt_cmd = args.kt_command or "python3 bench.py --steps 20 --warmup 5"
    pmc_cmd = args.pmc_command or "python3 bench.py --steps 20 --warmup 5"
    lines = ["# rocprofv3 summary: FISTA hot passes, stored CSR/CSC (*_win: with the windowed gathers, bucket_*: "
             "their bucketing passes; blk_*: the blocked stored operator; mf_*: the matrix-free operator, "
             "mf_win_scatter its windowed gathers' bucketing pass), FP32 bulk, " + (args.stats_title or "n=2^26, m=2^27, 2 stages"),
             "# each figure over the kernel's dispatches with its largest grid (the headline instance's launches)",
             f"# kernel trace: rocprofv3 --kernel-trace --stats --output-format csv -d <dir> -o bench -- {kt_cmd}",
             f"# counters:     rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE) --output-format csv -d <dir> -o bench -- "
             f"{pmc_cmd}",
             f"# copy scale:   rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE) ... -- python3 bench.py --copy-calibration",
             f"# summary:      python3 bench.py --profile-summary --kt ... --fetch ... --write ... --copyf ... --copyw ...",
             f"kernel_source_hash: {kernel_source_hash()}",
             f"copy_fetch_kib_per_gib: {copy_f:.1f}",
             f"copy_write_kib_per_gib: {copy_w:.1f}",
             f"fetch_scale: {f_scale:.4f}",
             f"write_scale: {w_scale:.4f}"]
    for key, (pat, _) in names.items():
        if key not in dur:
            continue  # not launched in this run (the windowed gathers' pass below n = 2^22)
        lines.append(f"{key}_avg_ns: {dur[key][0]:.0f}")
        lines.append(f"{key}_calls: {dur[key][1]}")
        lines.append(f"{key}_grid: {big[key]}")
        fk, nf = counter(args.fetch, "FETCH_SIZE", pat, big[key])
        wk, nw = counter(args.write, "WRITE_SIZE", pat, big[key])
        lines.append(f"{key}_fetch_kib_median: {fk:.1f}")
        lines.append(f"{key}_write_kib_median: {wk:.1f}")
        lines.append(f"{key}_traffic_bytes: {(fk * f_scale + wk * w_scale) * 1024:.0f}")
    with open(args.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


# Counters of the vector memory path read for the stored passes (two
# rocprofv3 --pmc runs, each within one run's counter limits), and what the
# summary derives from them.  GRBM_GUI_ACTIVE is summed over the 8 XCDs and
# the TCP_ (vector L1) counters over the 256 CUs.
PMC_PASSES = [
    "TCP_UTCL1_TRANSLATION_MISS_sum TCP_UTCL1_REQUEST_sum TCP_TCC_READ_REQ_sum TCP_TOTAL_CACHE_ACCESSES_sum "
    "TCC_REQ_sum TCC_HIT_sum GRBM_GUI_ACTIVE SQ_WAVE_CYCLES SQ_WAIT_INST_ANY SQ_BUSY_CYCLES",
    "TA_BUSY_avr TA_ADDR_STALLED_BY_TC_CYCLES_sum TCP_PENDING_STALL_CYCLES_sum TCP_TCR_TCP_STALL_CYCLES_sum "
    "TCP_UTCL1_TRANSLATION_HIT_sum TCP_TCC_READ_REQ_LATENCY_sum TCC_TAG_STALL_sum TCC_BUSY_avr TCC_EA0_RDREQ_sum "
    "GRBM_GUI_ACTIVE"]


def write_counter_summary(args):
    """Per-kernel medians of the PMC_PASSES counters (rocprofv3 CSV directories
    in --pmc-dirs) for the stored passes, with the latency figures they give."""
    import csv
    import re
    import statistics

    per = {}
    for d in args.pmc_dirs:
        rows = []
        for root, _, files in os.walk(d):
            for f in files:
                if f.endswith("counter_collection.csv"):
                    rows += list(csv.DictReader(open(os.path.join(root, f))))
        if not rows:
            raise SystemExit(f"no *counter_collection.csv under {d}")
        for key, (pat, rank) in PASS_KERNELS.items():
            rs = [r for r in rows if re.search(pat, r["Kernel_Name"])]
            grids = sorted({int(r.get("Grid_Size") or 0) for r in rs}, reverse=True)
            if len(grids) <= rank:
                continue
            by = {}
            for r in rs:
                if int(r.get("Grid_Size") or 0) == grids[rank]:
                    by.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
            per.setdefault(key, {}).update({c: statistics.median(v) for c, v in by.items()})
    cus, xcds = 256, 8
    lines = ["# rocprofv3 counters of the vector memory path, stored FISTA passes (*_win: windowed gathers, "
             "bucket_*: their bucketing passes), " + (args.stats_title or "n=2^26, m=2^27, 2 stages"),
             "# medians over each kernel's dispatches with its largest grid; GRBM_GUI_ACTIVE summed over 8 XCDs,",
             "# TCP_* (vector L1) over 256 CUs, TCC_* (L2) over all channels",
             *[f"# counters:     rocprofv3 --pmc {c} --output-format csv -d <dir> -o bench -- {args.pmc_command}"
               for c in PMC_PASSES],
             "# summary:      python3 bench.py --counter-summary --pmc-dirs <dir> <dir> --out <file>",
             "# derived: cycles = GRBM_GUI_ACTIVE / 8 (per XCD, i.e. per CU); l2_read_latency = "
             "TCP_TCC_READ_REQ_LATENCY_sum / TCP_TCC_READ_REQ_sum;",
             "#   reads_in_flight_per_cu = TCP_TCC_READ_REQ_LATENCY_sum / 256 / cycles; vl1d_waiting_on_l2 = "
             "TCP_PENDING_STALL_CYCLES_sum / 256 / cycles;",
             "#   vl1d_stalled_issuing_to_l2 = TCP_TCR_TCP_STALL_CYCLES_sum / 256 / cycles; ta_stalled_by_vl1d = "
             "TA_ADDR_STALLED_BY_TC_CYCLES_sum / 256 / cycles;",
             "#   l2_hit = TCC_HIT_sum / TCC_REQ_sum; utcl1_miss = TCP_UTCL1_TRANSLATION_MISS_sum / TCP_UTCL1_REQUEST_sum",
             f"kernel_source_hash: {kernel_source_hash()}"]
    for key, c in per.items():
        for name in sorted(c):
            lines.append(f"{key}.{name}: {c[name]:.6g}")
        cyc = c.get("GRBM_GUI_ACTIVE", 0.0) / xcds
        req = c.get("TCP_TCC_READ_REQ_sum", 0.0)
        lat = c.get("TCP_TCC_READ_REQ_LATENCY_sum")
        derived = {}
        if lat is not None and req > 0:
            derived["l2_read_latency_cycles"] = lat / req
        if lat is not None and cyc > 0:
            derived["reads_in_flight_per_cu"] = lat / cus / cyc
        for dname, cname in (("vl1d_waiting_on_l2", "TCP_PENDING_STALL_CYCLES_sum"),
                             ("vl1d_stalled_issuing_to_l2", "TCP_TCR_TCP_STALL_CYCLES_sum"),
                             ("ta_stalled_by_vl1d", "TA_ADDR_STALLED_BY_TC_CYCLES_sum")):
            if cname in c and cyc > 0:
                derived[dname] = c[cname] / cus / cyc
        if c.get("TCC_REQ_sum"):
            derived["l2_hit"] = c.get("TCC_HIT_sum", 0.0) / c["TCC_REQ_sum"]
        if c.get("TCP_UTCL1_REQUEST_sum"):
            derived["utcl1_miss"] = c.get("TCP_UTCL1_TRANSLATION_MISS_sum", 0.0) / c["TCP_UTCL1_REQUEST_sum"]
        for dname, v in derived.items():
            lines.append(f"{key}.{dname}: {v:.4g}")
    with open(args.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def write_stats_summary(args):
    """Top kernels of a rocprofv3 --kernel-trace --stats run as a short text table."""
    import csv
    rows = None
    for root, _, files in os.walk(args.kt):
        for f in files:
            if f.endswith("kernel_stats.csv"):
                rows = list(csv.DictReader(open(os.path.join(root, f))))
    if rows is None:
        raise SystemExit(f"no *kernel_stats.csv under {args.kt}")
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = [f"# rocprofv3 --kernel-trace --stats, kernel statistics (top entries)",
             f"# command: {args.stats_command}",
             f"# workload: {args.stats_title}",
             f"{'kernel':<62}{'calls':>7}{'avg_us':>10}{'min_us':>10}{'max_us':>10}{'pct':>7}"]
    for r in rows[:args.stats_top]:
        lines.append(f"{r['Name'][:60]:<62}{int(r['Calls']):>7}{float(r['AverageNs']) / 1e3:>10.2f}"
                     f"{float(r['MinNs']) / 1e3:>10.2f}{float(r['MaxNs']) / 1e3:>10.2f}{float(r['Percentage']):>7.2f}")
    with open(args.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def algorithmic_bytes(m, n, nnz, es=4, ie=4):
    """Bytes one launch of each pass must move at minimum (FP32 values, int32 indices).

    residual pass:  row_ptr (m+1), col + val (nnz), x gathered once (n),
                    b, r_x read, r_x write, r_y write (4 m-vectors)
    transpose pass: col_ptr (n+1), row + val (nnz), r_y gathered once (m),
                    x_{k-1}, x_{k-2} read, x_k write (3 n-vectors)
    """
    k1 = ie * (m + 1) + (ie + es) * nnz + es * n + 4 * es * m
    k2 = ie * (n + 1) + (ie + es) * nnz + es * m + 3 * es * n
    return k1, k2


def blocked_bytes(m, n, nruns):
    """Bytes one launch of each pass over the blocked operator must move (FP32).

    residual pass:  run pointer (m+1), start + 4 values per row run (nruns),
                    x gathered once (n + 2 with the wrap copies),
                    b, r_x read, r_x write, r_y write (4 m-vectors)
    transpose pass: start + 4 values per column run (4 per column),
                    r_y gathered once (m + 2), x_{k-1}, x_{k-2} read, x_k write
    """
    k1 = 4 * (m + 1) + 20 * nruns + 4 * (n + 2) + 16 * m
    k2 = 20 * 4 * n + 4 * (m + 2) + 12 * n
    return k1, k2


def mf_bytes(m, n, es=4, windows=False):
    """Algorithmic bytes of one matrix-free FISTA iteration (FP32, two stages).

    transpose pass fused with G^T (n side): inv (int32, n), v gathered once (n),
    the n-side (c, s) of both stages (n/2 pairs each), x_{k-1} and x_{k-2}
    read, x_k written, sigma (n), w written (n).
    residual pass fused with Q^T (m side): emb (int32, m), w gathered once (n),
    the m-side (c, s) of both stages, b and r_x,prev read, r_x written, sigma
    (m), v written at the n active positions only (n).  r_y stays on chip; the
    per-workgroup rank bases (m / 512 int32) are left out.
    windows (the windowed gathers the library uses from n = 2^22 on): each of
    the two gathers adds a bucketing pass (source read, two int32 tables, the
    bucketed copy written: 12 + es bytes per element); the gather tables
    replace emb and inv byte for byte.
    """
    tr = 4 * n + es * n + es * 2 * n + es * 3 * n + es * n + es * n
    res = 4 * m + es * n + es * 2 * m + es * 2 * m + es * m + es * m + es * n
    win = 2 * (12 + es) * n if windows else 0
    return tr + res + win


def cpu_baseline(m, n, kappa, s, tau, seed, rounds, budget_s):
    """The oracle's FISTA (plain FP64 numpy/scipy) on the same workload."""
    import numpy as np
    from oracle import fista as F
    from oracle import instance as OI

    t0 = time.perf_counter()
    inst = OI.Instance(m, n, kappa, s, tau, seed, rounds=rounds)
    A = inst.sparse_A()
    At = A.T.tocsr()
    gen_s = time.perf_counter() - t0
    mv, rmv = (lambda v: A @ v), (lambda v: At @ v)
    # calibrate with 2 iterations, then run a bounded sample
    t0 = time.perf_counter()
    F.fista(mv, rmv, inst.b, tau, inst.L, 2)
    per = (time.perf_counter() - t0) / 2
    iters = max(3, int(budget_s / max(per, 1e-6)))
    t0 = time.perf_counter()
    F.fista(mv, rmv, inst.b, tau, inst.L, iters)
    dt = time.perf_counter() - t0
    return {"value": iters / dt, "unit": "iters/s", "cores": 1, "kind": "oracle",
            "sample": f"{iters} FP64 FISTA iterations of the CPU oracle (numpy + scipy.sparse, one thread) "
                      f"on the same n=2^20 instance generated by the oracle ({gen_s:.1f} s, not timed)"}


def _even(v):
    return max(2, int(round(v / 2.0)) * 2)


def serve_requests(count, seed, log2n_lo=10, log2n_hi=22):
    """Solve requests of the serving workload: n log-uniform in [2^lo, 2^hi]
    (even), m = 2n, kappa log-uniform in [1e2, 1e6], s = n/100, tau
    log-uniform in [1e-2, 1], two Givens stages, relative-gap tolerance 1e-6."""
    import numpy as np
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = _even(2.0 ** rng.uniform(log2n_lo, log2n_hi))
        out.append(dict(m=2 * n, n=n, kappa=float(10 ** rng.uniform(2, 6)), s=max(1, n // 100),
                        tau=float(10 ** rng.uniform(-2, 0)), seed=1503035204 * 1000 + i, rounds=2))
    return out


def _pct(v, q):
    import numpy as np
    return float(np.percentile(np.asarray(v), q)) if len(v) else None


def bench_serve(args):
    """Continuous-batching server vs the one-at-a-time single-solve path.

    Both serve the same request list with the same tolerance, check period
    and iteration cap.  1) Calibration: the plain path solves every request
    alone, back to back (generation + FISTA), giving its capacity mu.
    2) Arrival times: a Poisson process at rate lambda = rate_mult * mu
    (separate random stream).  3) The plain path serves the arrivals in real
    time, first come first served, one at a time.  4) The server serves the
    same arrivals in real time.  Latency = arrival -> result available on the
    host; solves/s = requests / (last result - first arrival)."""
    import numpy as np
    import torch

    import paper_1503_03520_amd as L

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    tol, check, cap = args.serve_tol, args.check_every, args.serve_max_iter
    reqs = serve_requests(args.requests + args.serve_warmup, 1503035204, args.serve_log2n_lo, args.serve_log2n_hi)
    warm, reqs = reqs[:args.serve_warmup], reqs[args.serve_warmup:]

    finish = not args.serve_fp32_only
    storage = (L.STORE_F32 | L.STORE_F64) if finish else L.STORE_F32

    def plain_one(r):
        inst = L.l1ls_generate(r["m"], r["n"], r["kappa"], r["s"], r["tau"], r["seed"], rounds=r["rounds"],
                               storage=storage, stream=stream)
        x, rep, _ = L.l1ls_solve_fista(inst, max_iter=cap, rel_gap_tol=tol, check_every=check, precision=L.F32,
                                       polish=2 if finish else 0, stream=stream)
        torch.cuda.synchronize()
        inst.free()
        return rep

    last = [time.perf_counter()]

    def progress(**kv):  # a line every 10 s, so a long run is seen to be alive
        if time.perf_counter() - last[0] > 10.0:
            last[0] = time.perf_counter()
            print(json.dumps({"progress": "serve", **kv}), file=sys.stderr, flush=True)

    for r in warm:
        plain_one(r)
    service, conv_plain, iters_plain = [], 0, []
    for i, r in enumerate(reqs):
        progress(phase="calibration", done=i)
        t0 = time.perf_counter()
        rep = plain_one(r)
        service.append(time.perf_counter() - t0)
        conv_plain += rep["converged"] == 1
        iters_plain.append(rep["iterations"])
    mu = len(reqs) / sum(service)

    def arrivals(rate_mult):
        rng = np.random.default_rng(1503035205)
        gaps = rng.exponential(1.0 / (rate_mult * mu), size=len(reqs))
        return np.cumsum(gaps) - gaps[0]

    def run_plain(arr):
        lat = []
        t0 = time.perf_counter()
        for i, (r, a) in enumerate(zip(reqs, arr)):
            progress(phase="plain", done=i)
            now = time.perf_counter() - t0
            if now < a:
                time.sleep(a - now)
            plain_one(r)
            lat.append(time.perf_counter() - t0 - a)
        span = time.perf_counter() - t0
        return lat, span

    def run_server(arr):
        S = L.Server(args.serve_slots, hbm_budget_bytes=int(args.serve_budget_gib * (1 << 30)),
                     iters_per_tick=args.serve_iters_per_tick, check_every=check, stream=stream)
        lat, conv, iters, peak, nxt = {}, 0, [], 0, 0
        ids = {}
        t0 = time.perf_counter()
        while len(lat) < len(reqs):
            progress(phase="server", done=len(lat))
            now = time.perf_counter() - t0
            while nxt < len(reqs) and arr[nxt] <= now:
                r = reqs[nxt]
                rid = S.submit(r["m"], r["n"], r["kappa"], r["s"], r["tau"], r["seed"], rounds=r["rounds"],
                               rel_gap_tol=tol, max_iter=cap, fp64_finish=finish)
                ids[rid] = nxt
                nxt += 1
            q, res, _ = S.stats()
            if q or res:
                S.tick()
                peak = max(peak, S.stats()[1])
            elif nxt < len(reqs):
                time.sleep(max(0.0, arr[nxt] - (time.perf_counter() - t0)))
            # results of the finishing workers can land between two ticks (or
            # after the last one): collect them on every pass
            done_t = time.perf_counter() - t0
            for rid in S.completed():
                _, rep = S.take(rid, want_x=False)
                i = ids[rid]
                lat[i] = done_t - arr[i]
                conv += rep["converged"] == 1
                iters.append(rep["iterations"])
        span = time.perf_counter() - t0
        S.destroy()
        return [lat[i] for i in range(len(reqs))], span, conv, iters, peak

    # the server's size classes (n < 2^14, n < 2^18, larger)
    classes = [("n<2^14", 0, 1 << 14), ("2^14<=n<2^18", 1 << 14, 1 << 18), ("n>=2^18", 1 << 18, 1 << 62)]

    def by_class(lat):
        out = {}
        for name, lo, hi in classes:
            v = [lat[i] for i, r in enumerate(reqs) if lo <= r["n"] < hi]
            out[name] = {"requests": len(v), "p50_s": _pct(v, 50), "p99_s": _pct(v, 99)}
        return out

    results = []
    for mult in args.rate_mults:
        arr = arrivals(mult)
        lp, sp = run_plain(arr) if mult <= args.plain_max_mult else (None, None)
        ls, ss, conv_s, iters_s, peak = run_server(arr)
        row = {"rate_mult": mult, "rate_per_s": mult * mu,
               "server": {"solves_per_s": len(reqs) / ss, "p50_s": _pct(ls, 50), "p99_s": _pct(ls, 99),
                          "converged": conv_s, "peak_resident": peak, "by_size_class": by_class(ls)},
               }
        if lp is not None:
            row["plain_fifo"] = {"solves_per_s": len(reqs) / sp, "p50_s": _pct(lp, 50), "p99_s": _pct(lp, 99),
                                 "by_size_class": by_class(lp)}
        results.append(row)
        print(json.dumps({"progress": "serve", **row}), file=sys.stderr, flush=True)
        if args.serve_dump:
            with open(args.serve_dump, "a") as fh:
                for i, r in enumerate(reqs):
                    fh.write(json.dumps({"mult": mult, "i": i, "n": r["n"], "kappa": r["kappa"], "tau": r["tau"],
                                         "arrival": float(arr[i]), "service": service[i],
                                         "iters": iters_plain[i], "lat_plain": lp[i] if lp else None,
                                         "lat_server": ls[i]}) + "\n")
    head = results[0]
    line = {
        "metric": "served solves/sec at a Poisson rate of %.2g x plain-path capacity (p50/p99 latency beside)"
                  % args.rate_mults[0],
        "value": head["server"]["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1, "steps": len(reqs), "warmup": len(warm),
        "ms_per_step": 1e3 / head["server"]["solves_per_s"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (instances generated on the device at admission, seeds 1503035204000+i)",
        "config": {"workload": "serving: Poisson arrivals, n log-uniform [2^%d, 2^%d], m = 2n, kappa log-uniform "
                               "[1e2, 1e6], s = n/100, tau log-uniform [1e-2, 1], 2 Givens stages"
                               % (args.serve_log2n_lo, args.serve_log2n_hi),
                   "requests": len(reqs), "rel_gap_tol": tol, "check_every": check, "max_iter": cap,
                   "slots": args.serve_slots, "iters_per_tick": args.serve_iters_per_tick,
                   "hbm_budget_gib": args.serve_budget_gib,
                   "accuracy": ("FP64 gap <= tol (FP32 FISTA, then FP64 polish of the reduced problem when the "
                                "FP64 gap misses tol)") if finish else "FP32 device gap <= tol (FISTA in FP32)"},
        "p50_s": head["server"]["p50_s"], "p99_s": head["server"]["p99_s"],
        "extra": {"plain_capacity_solves_per_s": mu, "plain_converged": conv_plain,
                  "plain_iters_median": _pct(iters_plain, 50), "plain_service_s_mean": float(np.mean(service)),
                  "plain_service_s_p99": _pct(service, 99), "rates": results},
    }
    print(json.dumps(line), flush=True)


def batched_configs(count):
    """(m, n, kappa, s, tau, seed, rounds) of the batched workload's instances:
    n log-uniform in [2^10, 2^16] (even), m = 2n, kappa from {1e2, ..., 1e6},
    s = n/100, tau = 1, two stages; sizes drawn by numpy PCG64 seed 1503035203."""
    import numpy as np
    rng = np.random.default_rng(1503035203)
    cfgs = []
    for j in range(count):
        n = _even(2.0 ** rng.uniform(10, 16))
        cfgs.append((2 * n, n, float(10 ** rng.integers(2, 7)), max(1, n // 100), 1.0, 1503035203000 + j, 2))
    return cfgs


def bench_batched(args):
    """Many uneven instances in shared launches vs the single-solve path.

    256 instances, n log-uniform in [2^10, 2^16] (even), m = 2n, kappa drawn
    from {1e2, 1e3, 1e4, 1e5, 1e6}, s = n/100, tau = 1, two Givens stages,
    FP32.  Both paths stop at the same device gap test (relative gap <= tol,
    every check_every iterations) with the same cap; instances are generated
    before timing.  value = solves/s of the batched path."""
    import numpy as np
    import torch

    import paper_1503_03520_amd as L

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    cfgs = batched_configs(args.instances)
    insts = [L.l1ls_generate(*c[:6], rounds=c[6], storage=L.STORE_F32, stream=stream) for c in cfgs]
    torch.cuda.synchronize()
    kw = dict(max_iter=args.batch_max_iter, rel_gap_tol=args.batch_tol, check_every=args.check_every,
              precision=L.F32, stream=stream)
    # warm-up over every instance: it also runs the tile-schedule autotuner
    # once per size class (a per-process cost, kept out of the timed region)
    L.l1ls_solve_fista_batched(insts, **dict(kw, max_iter=16))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xs, reps, _ = L.l1ls_solve_fista_batched(insts, **kw)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    # the same batch with every check period enqueued as one replayed HIP graph
    L.l1ls_solve_fista_batched(insts, **dict(kw, max_iter=16, graph=1))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xg, repg, _ = L.l1ls_solve_fista_batched(insts, **dict(kw, graph=1))
    torch.cuda.synchronize()
    tg = time.perf_counter() - t0
    graph_same = sum(int(torch.equal(a, b)) for a, b in zip(xs, xg))
    # the slots of at most 4096 rows (n <= 2048) running each call's
    # iterations in one workgroup, beside the shared passes of the others
    L.l1ls_solve_fista_batched(insts, **dict(kw, max_iter=16, persist_rows=4096))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xn, _, _ = L.l1ls_solve_fista_batched(insts, **dict(kw, persist_rows=4096))
    torch.cuda.synchronize()
    tn = time.perf_counter() - t0
    shared_same = sum(int(torch.equal(a, b)) for a, b in zip(xs, xn))
    t0 = time.perf_counter()
    same, conv_p, iters_p = 0, 0, 0
    xp = []
    for inst in insts:
        x1, r1, _ = L.l1ls_solve_fista(inst, polish=0, **kw)
        xp.append(x1)
        conv_p += r1["converged"] == 1
        iters_p += r1["iterations"]
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    same = sum(int(torch.equal(a, b)) for a, b in zip(xs, xp))
    iters_b = sum(r["iterations"] for r in reps)
    nnz = sum(i.info().nnz for i in insts)
    line = {
        "metric": "batched solves/sec (uneven instances in shared launches) vs the single-solve path",
        "value": len(insts) / tb, "unit": "solves/s", "n_gpus": 1, "steps": len(insts), "warmup": 1,
        "ms_per_step": tb * 1e3 / len(insts), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic (instances from the device generator, seeds 1503035203000+j)",
        "config": {"workload": "batched: %d instances, n log-uniform [2^10, 2^16], m = 2n, kappa in "
                               "{1e2..1e6}, s = n/100, tau = 1, 2 Givens stages" % len(insts),
                   "rel_gap_tol": args.batch_tol, "check_every": args.check_every,
                   "max_iter": args.batch_max_iter, "total_nnz": nnz},
        "extra": {"batched_s": tb, "plain_s": tp, "plain_solves_per_s": len(insts) / tp, "speedup": tp / tb,
                  "graph": {"batched_s": tg, "solves_per_s": len(insts) / tg, "speedup_vs_launched": tb / tg,
                            "bitwise_equal_to_launched": graph_same},
                  "persistent_small_slots": {"persist_rows": 4096, "batched_s": tn, "solves_per_s": len(insts) / tn,
                                             "bitwise_equal_to_default": shared_same},
                  "converged_batched": sum(r["converged"] == 1 for r in reps), "converged_plain": conv_p,
                  "iterations_batched": iters_b, "iterations_plain": iters_p,
                  "instance_iterations_per_s": {"batched": iters_b / tb, "plain": iters_p / tp},
                  "bitwise_equal_results": same},
    }
    print(json.dumps(line), flush=True)


def bench_path(args):
    """64 tau values on one shared instance as one sparse-times-dense FISTA vs
    64 single solves.  n = 2^16, m = 2^17, kappa = 1e4, two Givens stages,
    s = n/100; tau log-spaced over [1e-3, 1] * ||A^T b||_inf.  Both stop at
    the same per-column device gap test with the same cap."""
    import numpy as np
    import torch

    import paper_1503_03520_amd as L

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    n = 1 << args.path_log2n
    m = 2 * n
    inst = L.l1ls_generate(m, n, 1e4, max(1, n // 100), 1.0, 1503035203, rounds=2, stream=stream)
    b = torch.from_numpy(L.device_to_numpy(inst.info().b_dev, m, np.float64)).cuda()
    atb = torch.empty(n, dtype=torch.float64, device="cuda")
    L.l1ls_apply(inst, 1, L.OP_STORED, L.F64, b, atb, stream=stream)
    torch.cuda.synchronize()
    tmax = float(atb.abs().max())
    taus = list(np.geomspace(1e-3, 1.0, args.path_k) * tmax)
    kw = dict(max_iter=args.path_max_iter, rel_gap_tol=args.batch_tol, check_every=args.check_every,
              precision=L.F32, stream=stream)
    L.l1ls_solve_fista_path(inst, taus[:4], **dict(kw, max_iter=64))   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    X, reps, _ = L.l1ls_solve_fista_path(inst, taus, **kw)
    torch.cuda.synchronize()
    tpath = time.perf_counter() - t0
    t0 = time.perf_counter()
    conv_p, iters_p = 0, 0
    for t in taus:
        x1, r1, _ = L.l1ls_solve_fista(inst, tau=t, polish=0, **kw)
        conv_p += r1["converged"] == 1
        iters_p += r1["iterations"]
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    gaps = []
    for c in range(len(taus)):
        gaps.append(L.l1ls_objective_gap(inst, taus[c], X[c].contiguous())[2])
    # equal accuracy: every column finished in FP64 (the FP64 gap of the FP32
    # result, the polish where it misses the tolerance), against single solves
    # finished the same way
    t0 = time.perf_counter()
    Xf, repf, _ = L.l1ls_solve_fista_path(inst, taus, **dict(kw, polish=2))
    torch.cuda.synchronize()
    tpf = time.perf_counter() - t0
    t0 = time.perf_counter()
    conv_pf = 0
    for t in taus:
        x1, r1, _ = L.l1ls_solve_fista(inst, tau=t, polish=2, **kw)
        conv_pf += r1["converged"] == 1
    torch.cuda.synchronize()
    tpf_plain = time.perf_counter() - t0
    fp64_finish = {"path_s": tpf, "plain_s": tpf_plain, "speedup": tpf_plain / tpf,
                   "columns_per_s": len(taus) / tpf,
                   "converged_path_fp64": sum(r["converged"] == 1 for r in repf), "converged_plain_fp64": conv_pf,
                   "polished_columns": sum(r["polish_rounds"] > 0 for r in repf),
                   "fp64_gap_max": max(r["rel_gap"] for r in repf)}
    line = {
        "metric": "regularisation-path columns/sec (%d taus as one SpMM FISTA) vs single solves" % len(taus),
        "value": len(taus) / tpath, "unit": "solves/s", "n_gpus": 1, "steps": len(taus), "warmup": 1,
        "ms_per_step": tpath * 1e3 / len(taus), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic (device generator, seed 1503035203)",
        "config": {"workload": "path: n = 2^%d, m = 2n, kappa = 1e4, 2 Givens stages, s = n/100, %d taus "
                               "log-spaced over [1e-3, 1] * ||A^T b||_inf" % (args.path_log2n, len(taus)),
                   "rel_gap_tol": args.batch_tol, "check_every": args.check_every, "max_iter": args.path_max_iter},
        "extra": {"path_s": tpath, "plain_s": tp, "speedup": tp / tpath,
                  "converged_path": sum(r["converged"] == 1 for r in reps), "converged_plain": conv_p,
                  "iterations_path_max": max(r["iterations"] for r in reps),
                  "iterations_path_sum": sum(r["iterations"] for r in reps), "iterations_plain_sum": iters_p,
                  "fp64_gap_max_converged": max([g for g, r in zip(gaps, reps) if r["converged"] == 1] or [0.0]),
                  "fp64_gap_max": max(gaps), "fp64_finish": fp64_finish},
    }
    print(json.dumps(line), flush=True)


def bench_large(args):
    """Memory-scale instance on one GPU: n = 2^26, m = 2^27, kappa = 1e6, two
    Givens stages, s = n/1000, tau = 1.  FISTA iterations/s on the stored
    FP32 CSR + CSC and on the matrix-free operator (rotations and sigma
    applied on the fly), and CG-Newton Newton steps and PCG iterations per
    second, with the Hessian-vector products on the FP32 values of A (FP64
    vectors and sums) and all-FP64."""
    import torch

    import paper_1503_03520_amd as L

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    n = 1 << args.large_log2n
    m = 2 * n
    kappa, s, tau, seed = 1e6, max(1, n // 1000), 1.0, 1503035202
    t0 = time.perf_counter()
    inst = L.l1ls_generate(m, n, kappa, s, tau, seed, rounds=2, stream=stream,
                           storage=L.STORE_F32 | L.STORE_F64 | L.STORE_BLK32)
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    nnz = inst.info().nnz
    print(json.dumps({"progress": "generated", "seconds": gen_s, "nnz": nnz}), file=sys.stderr, flush=True)

    def fista_rate(op, steps, warmup):
        fs = L.Fista(inst, precision=L.F32, rel_gap_tol=0.0, check_every=32, max_iter=warmup + steps,
                     stream=stream, op=op)
        fs.iterate(warmup)
        torch.cuda.synchronize()
        t = time.perf_counter()
        fs.iterate(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        x = fs.get_x()
        fs.destroy()
        return steps / dt, x

    stored, x_s = fista_rate(L.OP_STORED, args.steps, args.warmup)
    print(json.dumps({"progress": "stored", "iters_per_s": stored}), file=sys.stderr, flush=True)
    mfree, x_m = fista_rate(L.OP_MATRIX_FREE, args.steps, args.warmup)
    print(json.dumps({"progress": "matrix_free", "iters_per_s": mfree}), file=sys.stderr, flush=True)
    blocked, x_b = fista_rate(L.OP_BLOCKED, args.steps, args.warmup)
    print(json.dumps({"progress": "blocked", "iters_per_s": blocked}), file=sys.stderr, flush=True)
    same = float((x_s - x_m).abs().max())
    newton = {}
    for prec, op, name in ((L.F32, L.OP_STORED, "f32_hessian_products"), (L.F64, L.OP_STORED, "f64"),
                           (L.F64, L.OP_MATRIX_FREE, "matrix_free_f64"),
                           (L.F32, L.OP_MATRIX_FREE, "matrix_free_f32_hessian_products")):
        t = time.perf_counter()
        xn, rn, _ = L.l1ls_solve_cg_newton(inst, max_iter=args.newton_steps, rel_gap_tol=1e-12, stream=stream,
                                           precision=prec, op=op)
        torch.cuda.synchronize()
        tn = time.perf_counter() - t
        P, D, gap = L.l1ls_objective_gap(inst, tau, xn)
        newton[name] = {"newton_steps": rn["iterations"], "pcg_iterations": rn["inner"], "seconds": tn,
                        "newton_steps_per_s": rn["iterations"] / tn, "ms_per_pcg_iteration": tn / max(rn["inner"], 1) * 1e3,
                        "fp64_rel_gap": gap}
        print(json.dumps({"progress": "cg_newton", name: newton[name]}), file=sys.stderr, flush=True)
    k1, k2 = algorithmic_bytes(m, n, nnz)
    line = {
        "metric": "FISTA iters/sec on the memory-scale instance, stored vs matrix-free; CG-Newton steps/sec",
        "value": stored, "unit": "iters/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 / stored, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic (device generator, seed %d)" % seed,
        "config": {"workload": "memory-scale instance: n = 2^%d, m = 2n, kappa = 1e6, 2 Givens stages, "
                               "s = n/1000, tau = 1" % args.large_log2n, "nnz": nnz},
        "extra": {"generate_s": gen_s, "stored_iters_per_s": stored,
                  "stored_gbs_algorithmic": (k1 + k2) * stored / 1e9,
                  "matrix_free_iters_per_s": mfree, "matrix_free_gbs_algorithmic": mf_bytes(m, n, windows=n >= 1 << 22) * mfree / 1e9,
                  "matrix_free_speedup": mfree / stored,
                  "matrix_free_gathers": "windowed" if n >= 1 << 22 else "plain",
                  "blocked_iters_per_s": blocked,
                  "blocked_gbs_algorithmic": sum(blocked_bytes(m, n, 4 * n)) * blocked / 1e9,
                  "stored_vs_blocked_max_abs_diff": float((x_s - x_b).abs().max()),
                  "stored_vs_matrix_free_max_abs_diff": same,
                  "cg_newton": newton},
    }
    print(json.dumps(line), flush=True)


def bench_table1(args):
    """Section 8.9 (Table 1) instance: A = Sigma G^T, one stage of adjacent
    Givens rotations with theta = 2 pi / 3, sigma 0.1 / 100, s = n / 2^10,
    x* entries -1e4 and 0.1, tau = 1, at n = 2^30 (m = 2^31).  A step is one
    whole CG-Newton solve of `--newton-steps` Newton steps (section 8.9
    reports 8) from x = 0, generation excluded; value = seconds per solve."""
    import torch

    import paper_1503_03520_amd as L

    torch.cuda.set_device(0)
    n = 1 << args.table1_log2n
    seed = 1503035206
    stream = torch.cuda.current_stream()
    free, _ = torch.cuda.mem_get_info()
    need = L.sgt_bytes(n) + L.sgt_solve_bytes(n) + 8 * n
    if need > free:
        print(json.dumps({"error": f"n = 2^{args.table1_log2n} needs {need / 2**30:.1f} GiB, {free / 2**30:.1f} free"}))
        sys.exit(3)
    prm = L.sgt_params(n, seed)
    t = time.perf_counter()
    H = L.SgtInstance(prm, stream=stream)
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t
    print(json.dumps({"progress": "generated", "seconds": gen_s}), file=sys.stderr, flush=True)
    x = torch.empty(n, dtype=torch.float64, device="cuda")
    for _ in range(args.warmup):
        H.solve_cg_newton(x_out=x, max_iter=1, stream=stream)
    torch.cuda.synchronize()
    times, rep = [], None
    for _ in range(args.steps):
        # one Newton step per call, so that a long solve reports as it goes (the
        # report's gap and error passes add two streaming passes per step)
        torch.cuda.synchronize()
        t = time.perf_counter()
        N = H.newton(x_out=x, stream=stream)
        for _k in range(args.newton_steps):
            rep, st = N.step(1)
            print(json.dumps({"progress": "newton_step", "step": rep["iterations"], "pcg": rep["inner"],
                              "seconds": time.perf_counter() - t, "rel_err": rep["rel_err"]}),
                  file=sys.stderr, flush=True)
            if st == L.L1LS_OK:
                break
        N.destroy()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
        print(json.dumps({"progress": "solve", "seconds": times[-1], "newton": rep["iterations"],
                          "pcg": rep["inner"], "rel_err": rep["rel_err"]}), file=sys.stderr, flush=True)
    # HIP events around the passes of the first Newton steps (at most 4, so the
    # run stays short at 2^32; hundreds of PCG passes)
    _, rep_t, _ = H.solve_cg_newton(x_out=x, max_iter=min(args.newton_steps, 4), stream=stream, time_kernels=1)
    kt = H.kernel_times()
    avg_ms = {k: v[0] / max(v[1], 1) for k, v in kt.items()}
    # algorithmic bytes per launch: PCG pass reads r, d, p, dx and writes p,
    # dx, r; line search reads x, dx, b; setup reads x, gd, b, writes d, r
    it_bytes, ls_bytes, setup_bytes = 56 * n, 24 * n, 40 * n
    achieved = it_bytes / (avg_ms["pcg_iteration"] * 1e-3) / 1e9
    sec = sum(times) / len(times)
    pcg = rep["inner"]
    line = {
        "metric": "CG-Newton seconds per solve of the section 8.9 (Table 1) instance",
        "value": sec,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": {30: sec / 1923.0, 32: sec / 1968.0}.get(args.table1_log2n),
        "dtype": "f64",
        "data": "synthetic (section 8.9 instance generated on the device, seed %d)" % seed,
        "config": {"workload": "section 8.9 instance: A = Sigma G^T (m = 2n), adjacent Givens pairs at theta = "
                               "2 pi / 3, sigma 0.1 / 100, s = n / 2^10 with x* entries -1e4 / 0.1, tau = 1; "
                               "CG-Newton mu = 1e-5, PCG rtol 0.1, diagonal preconditioner, from x = 0",
                   "n": n, "m": 2 * n, "s": prm.s, "newton_steps": args.newton_steps},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "kh_cg_iter (PCG iteration: p, dx, r and the r.u, w.u, r.r partials)",
                     "algorithmic_bytes_per_launch": it_bytes},
        "extra": {
            "newton_steps": rep["iterations"], "pcg_iterations": pcg, "rel_err": rep["rel_err"],
            "fp64_rel_gap": rep["rel_gap"], "generate_s": gen_s, "solve_seconds": times,
            "ms_per_pcg_iteration": sec * 1e3 / max(pcg, 1),
            "pass_avg_ms": avg_ms,
            "pass_gbs": {"pcg_iteration": it_bytes / (avg_ms["pcg_iteration"] * 1e-3) / 1e9,
                         "line_search": ls_bytes / (avg_ms["line_search"] * 1e-3) / 1e9,
                         "newton_setup": setup_bytes / (avg_ms["newton_setup"] * 1e-3) / 1e9},
            "bytes_per_pcg_iteration": it_bytes,
            "device_bytes": need,
            "paper": {"table_1": {"2^30": {"seconds": 1923, "cores": 64}, "2^32": {"seconds": 1968, "cores": 256}},
                      "machine": "ARCHER Cray XC30 (section 8.2)",
                      "newton_steps": 8, "pcg_per_newton": "about 100", "rel_err": "order 1e-4"},
        },
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_table1(n, args.newton_steps)
    print(json.dumps(line), flush=True)


def cpu_baseline_table1(n, newton_steps, log2_sample=18):
    """The oracle's CG-Newton (numpy, FP64) on the same class at n = 2^18,
    scaled linearly to n (section 8.9 reports the same Newton and PCG counts
    at every size, and every pass is linear in n)."""
    from oracle import newton as ON
    from oracle.sgt import SgtInstance

    ns = 1 << log2_sample
    I = SgtInstance(ns, ns // 1024, 1503035206)
    cn = I.colnorm2()
    t = time.perf_counter()
    _, st = ON.newton_cg(I.matvec, I.rmatvec, cn, I.b, I.tau, max_newton=newton_steps)
    sec = time.perf_counter() - t
    return {"value": sec * n / ns, "unit": "s", "cores": 1, "kind": "oracle",
            "sample": f"oracle CG-Newton, {newton_steps} Newton steps ({st['pcg']} PCG iterations) at n = 2^"
                      f"{log2_sample} took {sec:.2f} s on one core, scaled by n / 2^{log2_sample}"}


def grid_instances(log2n):
    """The instances of sections 8.4, 8.5 and 8.6 (A = Sigma G^T, m = 2n,
    s = n / 2^7): (section, n, label, parameter overrides)."""
    import math
    n = 1 << log2n
    out = []
    for q in range(6):
        for g in (10.0, 1e3):
            out.append(("8.4", n, f"q={q} OsGen gamma={g:g} theta=2pi/3",
                        dict(sigma_law=1, sigma_scale=10.0 ** q, xstar_law=1, gamma=g)))
    for th, tn in ((2 * math.pi / 10, "2pi/10"), (2 * math.pi / 1e3, "2pi/10^3")):
        for q in range(4):
            out.append(("8.5", n, f"q={q} OsGen3 gamma=100 theta={tn}",
                        dict(theta=th, sigma_law=1, sigma_scale=10.0 ** q, xstar_law=2, gamma=100.0)))
    for ln in (20, 22, 24, 26):
        out.append(("8.6", 1 << ln, f"n=2^{ln} OsGen3 gamma=100 theta=2pi/10",
                    dict(theta=2 * math.pi / 10, sigma_law=1, sigma_scale=10.0, xstar_law=2, gamma=100.0)))
    # Procedure IGen2 (section 3.2): m = n rows of B plus n/2 columns of N~
    for q in range(3):
        out.append(("3.2", n + n // 2, f"IGen2 m={n} n=1.5m q={q} OsGen gamma=10 theta=2pi/3",
                    dict(m=n, sigma_law=1, sigma_scale=10.0 ** q, xstar_law=1, gamma=10.0)))
    return out


def bench_grid(args):
    """Sections 8.4 to 8.6 on one GPU with the paper's protocol (section 8.3):
    CG-Newton (the paper's pdNCG reading) runs first, then FISTA and PCDM
    (every coordinate in every step) run until f_tau falls to CG-Newton's
    objective or an iteration cap.  Every instance is generated on the
    device; value = seconds for the whole grid."""
    import torch

    import paper_1503_03520_amd as L

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    rows, t_all = [], time.perf_counter()
    fista_pass = None
    for sec, n, label, kw in grid_instances(args.grid_log2n):
        if args.grid_sections and sec not in args.grid_sections:
            continue
        p = L.sgt_params(n, 1503035207, s=min(n, kw.get("m", n)) // 128, **kw)
        t = time.perf_counter()
        H = L.SgtInstance(p, stream=stream)
        torch.cuda.synchronize()
        gen_s = time.perf_counter() - t
        d = H.describe()
        k_rho = H.kappa_rho(0.1) if sec != "3.2" else None  # not defined for m < n (section 5)
        x = torch.empty(n, dtype=torch.float64, device="cuda")
        _, rn, _ = H.solve_cg_newton(x_out=x, max_iter=args.grid_newton, rel_gap_tol=1e-9, stream=stream)
        f_cgn = rn["primal"]
        _, rf, st = H.solve_fista(x_out=x, max_iter=args.grid_fista_max, rel_gap_tol=0.0, f_target=f_cgn,
                                  check_every=args.check_every, stream=stream, time_kernels=1 if fista_pass is None else 0)
        if fista_pass is None:
            kt = H.fista_kernel_times()
            fista_pass = (n, kt["iteration"][0] / max(kt["iteration"][1], 1))
        _, rp, stp = H.solve_pcdm(x_out=x, max_iter=args.grid_fista_max, rel_gap_tol=0.0, f_target=f_cgn,
                                  check_every=args.check_every, stream=stream, pcdm_p=1.0)
        row = {"section": sec, "instance": label, "n": n, "m": p.m, "L": d.L,
               "kappa_AtA": (d.sigma_max / d.sigma_min) ** 2 if sec != "3.2" else None,
               "kappa_0.1_xstar": k_rho, "generate_s": gen_s,
               "cg_newton": {"newton_steps": rn["iterations"], "pcg_iterations": rn["inner"], "seconds": rn["seconds"],
                             "f": f_cgn, "rel_err": rn["rel_err"], "converged": rn["converged"]},
               "fista": {"iterations": rf["iterations"], "seconds": rf["seconds"], "f": rf["primal"],
                         "reached_cg_newton_f": st == L.L1LS_OK, "rel_err": rf["rel_err"]},
               "pcdm": {"steps": rp["iterations"], "seconds": rp["seconds"], "f": rp["primal"],
                        "reached_cg_newton_f": stp == L.L1LS_OK, "rel_err": rp["rel_err"]}}
        rows.append(row)
        print(json.dumps({"progress": "grid", **row}), file=sys.stderr, flush=True)
        H.free()
        del x
    total = time.perf_counter() - t_all
    n0, ms = fista_pass
    ach = 32.0 * n0 / (ms * 1e-3) / 1e9
    line = {
        "metric": "seconds for the sections 8.4-8.6 instance grid (CG-Newton, then FISTA and PCDM to CG-Newton's objective)",
        "value": total, "unit": "s", "n_gpus": 1, "steps": len(rows), "warmup": 0, "ms_per_step": total * 1e3 / max(len(rows), 1),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (sections 8.4-8.6 and IGen2 instances generated on the device, seed 1503035207)",
        "config": {"workload": "sections 8.4-8.6: A = Sigma G^T, m = 2n, s = n/2^7, sigma uniform on [0, 10^q] + 0.1; "
                               "8.4: OsGen gamma 10 / 1e3, q = 0..5, theta = 2 pi/3; 8.5: OsGen3 gamma = 100, q = 0..3, "
                               "theta = 2 pi/10 and 2 pi/10^3; 8.6: OsGen3, q = 1, n = 2^20..2^26; "
                               "3.2: IGen2 with m = 2^22, n = 1.5 m, q = 0..2",
                   "n": 1 << args.grid_log2n, "newton_cap": args.grid_newton, "fista_cap": args.grid_fista_max},
        "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                     "traffic": None, "kernel": "kh_fista (FISTA iteration on the pairs)",
                     "algorithmic_bytes_per_launch": 32 * n0},
        "extra": {"instances": rows,
                  "paper": {"8.4": "pdNCG at most 30 iterations; FISTA thousands to tens of thousands; kappa_0.1 ~ 1",
                            "8.5": "kappa_0.1 ~ 40 on average", "8.6": "kappa_0.1 ~ 3 on average; linear-like scaling in n"}},
    }
    print(json.dumps(line), flush=True)


# The two single-instance workloads of the FISTA bench: the memory-scale
# instance (the headline) and the single large instance (reported beside it).
FISTA_CONFIGS = {
    "c3": dict(log2n=26, kappa=1e6, sdiv=1000, seed=1503035202,
               name="memory-scale instance: n = 2^26, m = 2n, kappa = 1e6, 2 Givens stages, s = n/1000, tau = 1; "
                    "FP32 bulk on stored CSR + CSC"),
    "c2": dict(log2n=20, kappa=1e4, sdiv=100, seed=1503035201,
               name="single large instance: n = 2^20, m = 2n, kappa = 1e4, 2 Givens stages, s = n/100, tau = 1; "
                    "FP32 bulk on stored CSR + CSC"),
}


def check_period(steps, warmup, cap=32):
    """Largest gap-check period <= cap that divides both the warm-up and the
    timed iteration counts, so that the timed window is a whole number of
    check periods (each ends with its gap evaluation)."""
    import math
    g = math.gcd(int(steps), int(warmup)) if warmup > 0 else int(steps)
    for d in range(min(cap, max(g, 1)), 0, -1):
        if g % d == 0:
            return d
    return 1


def host_description():
    """CPU model and the cores this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "usable_cores": usable, "os_cpu_count": os.cpu_count()}


def fista_legs(L, torch, inst, stream, steps, warmup, check, ops):
    """FISTA on `inst` (FP32 bulk, gap test every `check` iterations, no
    tolerance): per operator a plain run (HIP events around the whole window)
    and a run with per-kernel HIP events, each after `warmup` untimed
    iterations."""
    def run(op, time_kernels):
        fs = L.Fista(inst, precision=L.F32, rel_gap_tol=0.0, check_every=check, max_iter=warmup + steps,
                     time_kernels=time_kernels, stream=stream, op=op)
        fs.iterate(warmup)
        torch.cuda.synchronize()
        ms0, c0 = fs.kernel_times(5) if time_kernels else (None, None)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fs.iterate(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        out = {"ms": e0.elapsed_time(e1)}
        if time_kernels:
            ms1, c1 = fs.kernel_times(5)
            kms = [a - b for a, b in zip(ms1, ms0)]
            kl = [a - b for a, b in zip(c1, c0)]
            out["avg_ms"] = [kms[i] / max(kl[i], 1) for i in range(5)]
            out["launches"] = kl
        out["report"] = fs.report()
        out["x"] = fs.get_x()
        fs.destroy()
        return out

    res = {}
    for op in ops:
        plain = run(op, 0)
        timed = run(op, 1)
        res[op] = {"iters_per_s": steps / (plain["ms"] * 1e-3), "ms_per_step": plain["ms"] / steps,
                   "avg_ms": timed["avg_ms"], "launches": timed["launches"], "x": plain["x"],
                   "timed_window_ms_with_events": timed["ms"]}
    return res


def bench_fista(args):
    """FISTA iterations per second on one instance; the headline is the
    memory-scale instance (n = 2^26) on the stored FP32 CSR + CSC.  A step is
    one FISTA iteration of the whole hot path: the CSR residual pass, the CSC
    transpose pass with the prox step, and (every check period) the FP64 gap
    statistics and the device-side gap test."""
    import numpy as np
    import torch

    import paper_1503_03520_amd as L

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    cfg = FISTA_CONFIGS[args.config]
    n = 1 << (args.log2n if args.log2n else cfg["log2n"])
    m = 2 * n
    kappa, s, tau, seed, rounds = cfg["kappa"], max(1, n // cfg["sdiv"]), 1.0, cfg["seed"], 2
    check = args.check_every if args.check_every else check_period(args.steps, args.warmup)

    def progress(**kv):
        print(json.dumps({"progress": kv}), file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    # from n = 2^22 on the stored passes gather through the window tables
    # (L1LS_STORE_WINDOWS); the plain gathers are a side leg
    windows = n >= 1 << 22 and not args.no_windows
    inst = L.l1ls_generate(m, n, kappa, s, tau, seed, rounds=rounds, stream=stream,
                           storage=L.STORE_F32 | L.STORE_F64 | L.STORE_BLK32 | (L.STORE_WINDOWS if windows else 0))
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    nnz = inst.info().nnz
    progress(step="generated", n=n, nnz=nnz, seconds=gen_s, windowed_gathers=windows)

    legs = fista_legs(L, torch, inst, stream, args.steps, args.warmup, check,
                      (L.OP_STORED, L.OP_MATRIX_FREE, L.OP_BLOCKED))
    st, mf, bl = legs[L.OP_STORED], legs[L.OP_MATRIX_FREE], legs[L.OP_BLOCKED]
    progress(step="fista legs", stored=st["iters_per_s"], matrix_free=mf["iters_per_s"], blocked=bl["iters_per_s"])

    k1_bytes, k2_bytes = algorithmic_bytes(m, n, nnz)
    avg = st["avg_ms"]
    dominant = 0 if avg[0] >= avg[1] else 1
    dom_bytes = (k1_bytes, k2_bytes)[dominant]
    achieved = dom_bytes / (avg[dominant] * 1e-3) / 1e9
    pair_gbs = (k1_bytes + k2_bytes) / ((avg[0] + avg[1]) * 1e-3) / 1e9
    key = ("residual", "transpose_prox")[dominant] + ("_win" if windows else "")
    traffic = None
    summ = read_profile_summary(profile_summary_path(n))
    if summ and summ.get("kernel_source_hash") == kernel_source_hash() and f"{key}_traffic_bytes" in summ:
        traffic = float(summ[f"{key}_traffic_bytes"])

    xstar = torch.from_numpy(L.device_to_numpy(inst.info().x_star_dev, n, np.float64)).cuda()

    def rel_err(x):
        return float((x - xstar).norm() / xstar.norm())

    P, D, gap = L.l1ls_objective_gap(inst, tau, st["x"])
    b1, b2 = blocked_bytes(m, n, 4 * n)
    bavg = bl["avg_ms"]
    lam30 = L.l1ls_power_iteration(inst, 30, stream=stream)

    # Certified solve (outside the timed window): CG-Newton on the
    # matrix-free FP64 operator, then the FP64 polish of the reduced problem
    # on the stored FP64 A; the result is compared with the planted x*.
    t0 = time.perf_counter()
    xc, rc, _ = L.l1ls_solve_cg_newton(inst, max_iter=args.newton_steps, rel_gap_tol=1e-12, precision=L.F64,
                                       op=L.OP_MATRIX_FREE, polish=1, stream=stream)
    torch.cuda.synchronize()
    cert_s = time.perf_counter() - t0
    certified = {"method": "CG-Newton (matrix-free FP64, %d Newton steps) + FP64 polish" % args.newton_steps,
                 "seconds": cert_s, "newton_steps": rc["iterations"], "pcg_iterations": rc["inner"],
                 "polish_rounds": rc["polish_rounds"], "rel_gap_fp64": rc["rel_gap"],
                 "rel_err_planted": rc["rel_err"]}
    progress(step="certified", **certified)
    del xc
    extra = {
        "kernel_avg_us": {"residual": avg[0] * 1e3, "transpose_prox": avg[1] * 1e3, "gap": avg[2] * 1e3},
        "kernel_launches_in_window": {"residual": st["launches"][0], "transpose_prox": st["launches"][1],
                                      "gap": st["launches"][2]},
        "spmv_pair_gbs": pair_gbs, "spmv_pair_frac": pair_gbs / HBM_PEAK_GBS,
        "bytes_per_iter": k1_bytes + k2_bytes,
        "algorithmic_bytes_per_launch": {"residual": k1_bytes, "transpose_prox": k2_bytes},
        "generate_s": gen_s,
        "fista_fp32_after_window": {"iterations": args.warmup + args.steps, "rel_gap_fp64": gap,
                                    "rel_err_planted": rel_err(st["x"])},
        "certified_solve": certified,
        "lipschitz": {"closed_form": inst.info().L, "power_iteration_30_steps": lam30},
        "matrix_free": {"iters_per_s": mf["iters_per_s"], "ms_per_step": mf["ms_per_step"],
                        "kernel_avg_us": {k: mf["avg_ms"][i] * 1e3
                                          for i, k in enumerate(("residual_pair", "transpose_pair", "gap"))},
                        "bytes_per_iter": mf_bytes(m, n, windows=n >= 1 << 22),
                        "bytes_per_iter_two_stage_model": 152 * n,
                        "max_abs_diff_vs_stored": float((mf["x"] - st["x"]).abs().max())},
        "blocked": {"iters_per_s": bl["iters_per_s"], "ms_per_step": bl["ms_per_step"],
                    "kernel_avg_us": {"residual": bavg[0] * 1e3, "transpose_prox": bavg[1] * 1e3,
                                      "gap": bavg[2] * 1e3},
                    "algorithmic_gbs": {"residual": b1 / (bavg[0] * 1e-3) / 1e9,
                                        "transpose_prox": b2 / (bavg[1] * 1e-3) / 1e9},
                    "bytes_per_iter": b1 + b2,
                    "max_abs_diff_vs_stored": float((bl["x"] - st["x"]).abs().max())},
    }
    if windows:
        # the bucketing passes of the windowed gathers, and the stored passes
        # with their plain gathers on the same instance built without the
        # window tables (the iterates are the same bit for bit)
        extra["kernel_avg_us"].update({"bucket_x": avg[3] * 1e3, "bucket_r_y": avg[4] * 1e3})
        extra["kernel_launches_in_window"].update({"bucket_x": st["launches"][3], "bucket_r_y": st["launches"][4]})
        extra["iteration_algorithmic_gbs"] = (k1_bytes + k2_bytes) / (st["ms_per_step"] * 1e-3) / 1e9
        extra["instance_bytes"] = inst.nbytes()
        inst.free()
        inst = None
        torch.cuda.empty_cache()
        p_inst = L.l1ls_generate(m, n, kappa, s, tau, seed, rounds=rounds, stream=stream, storage=L.STORE_F32)
        pl = fista_legs(L, torch, p_inst, stream, args.steps, args.warmup, check, (L.OP_STORED,))[L.OP_STORED]
        pk = (k1_bytes, k2_bytes)
        extra["stored_plain_gathers"] = {
            "iters_per_s": pl["iters_per_s"], "ms_per_step": pl["ms_per_step"],
            "kernel_avg_us": {"residual": pl["avg_ms"][0] * 1e3, "transpose_prox": pl["avg_ms"][1] * 1e3,
                              "gap": pl["avg_ms"][2] * 1e3},
            "algorithmic_gbs": {k: pk[i] / (pl["avg_ms"][i] * 1e-3) / 1e9
                                for i, k in enumerate(("residual", "transpose_prox"))},
            "bitwise_equal_to_windowed": bool(torch.equal(pl["x"], st["x"]))}
        p_inst.free()
        progress(step="plain gathers", iters_per_s=pl["iters_per_s"])
    for leg in legs.values():
        leg.pop("x", None)
    if inst is not None:
        inst.free()
    del xstar
    torch.cuda.empty_cache()

    if args.config == "c3" and not args.no_c2:
        extra["c2"] = bench_c2_leg(L, torch, stream, args.steps, args.warmup, check)
        progress(step="c2", iters_per_s=extra["c2"]["iters_per_s"])

    # the small FP64 workload (n = 1024, m = 2048, kappa = 1e2, one stage,
    # s = 10, tau = 1): latency-bound, solved to rel gap 1e-8, then polished
    small = L.l1ls_generate(2048, 1024, 1e2, 10, 1.0, 1503035200, rounds=1, stream=stream)
    L.l1ls_solve_fista(small, max_iter=64, rel_gap_tol=0.0, precision=L.F64, stream=stream)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, srep, _ = L.l1ls_solve_fista(small, max_iter=20000, rel_gap_tol=1e-8, check_every=32, precision=L.F64,
                                    stream=stream)
    torch.cuda.synchronize()
    small_s = time.perf_counter() - t0
    _, prep, _ = L.l1ls_solve_fista(small, max_iter=20000, rel_gap_tol=1e-8, check_every=32, precision=L.F64,
                                    polish=1, stream=stream)
    small.free()
    extra["small_fp64"] = {"workload": "n=1024, m=2048, kappa=1e2, 1 stage, s=10, tau=1, FP64",
                           "iterations_to_gap_1e-8": srep["iterations"], "seconds": small_s,
                           "iters_per_s": srep["iterations"] / small_s, "rel_gap": srep["rel_gap"],
                           "rel_err_planted": srep["rel_err"],
                           "with_polish": {"seconds": prep["seconds"], "rel_gap": prep["rel_gap"],
                                           "rel_err_planted": prep["rel_err"]}}
    extra["host"] = host_description()
    extra["autotuned_tile_schedule"] = {
        "residual": L.tune_get("fista_f32_residual/%d" % (m - 1).bit_length()),
        "transpose": L.tune_get("fista_f32_transpose/%d" % (n - 1).bit_length()),
        "residual_windowed": L.tune_get("fista_f32_residual_win/%d" % (m - 1).bit_length()),
        "transpose_windowed": L.tune_get("fista_f32_transpose_win/%d" % (n - 1).bit_length())}

    value = st["iters_per_s"]
    line = {
        "metric": "FISTA iters/sec (SpMV pair A*y, A^T*r fused with prox, momentum, gap)",
        "value": value,
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": st["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (instance generated on the device from the paper's generator, seed %d)" % seed,
        "config": {"workload": cfg["name"] if n == 1 << cfg["log2n"] else cfg["name"] + " (n = 2^%d)" % n.bit_length(),
                   "n": n, "m": m, "kappa": kappa, "givens_stages": rounds, "s": s, "tau": tau,
                   "nnz": nnz, "check_every": check,
                   "gap_checks_in_timed_window": st["launches"][2]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": ("k_residual (CSR A x - b + momentum residual)",
                                "k_transpose_prox (CSC A^T r + prox)")[dominant]
                     + (", windowed gathers (XCD-placed)" if windows else ""),
                     "algorithmic_bytes_per_launch": dom_bytes},
        "extra": extra,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_scaled(args, cfg, n, nnz)
    print(json.dumps(line), flush=True)


def bench_c2_leg(L, torch, stream, steps, warmup, check):
    """The single large instance (n = 2^20) beside the headline: the stored
    FP32 passes, and FP32 FISTA followed by the FP64 polish to a certified
    gap."""
    cfg = FISTA_CONFIGS["c2"]
    n = 1 << cfg["log2n"]
    m = 2 * n
    inst = L.l1ls_generate(m, n, cfg["kappa"], n // cfg["sdiv"], 1.0, cfg["seed"], rounds=2, stream=stream,
                           storage=L.STORE_F32 | L.STORE_F64)
    nnz = inst.info().nnz
    leg = fista_legs(L, torch, inst, stream, steps, warmup, check, (L.OP_STORED,))[L.OP_STORED]
    k1, k2 = algorithmic_bytes(m, n, nnz)
    avg = leg["avg_ms"]
    pair = (k1 + k2) / ((avg[0] + avg[1]) * 1e-3) / 1e9
    t0 = time.perf_counter()
    _, rp, _ = L.l1ls_solve_fista(inst, max_iter=1000, rel_gap_tol=1e-8, check_every=32, precision=L.F32,
                                  polish=1, stream=stream)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    inst.free()
    return {"workload": cfg["name"], "nnz": nnz, "iters_per_s": leg["iters_per_s"], "ms_per_step": leg["ms_per_step"],
            "kernel_avg_us": {"residual": avg[0] * 1e3, "transpose_prox": avg[1] * 1e3, "gap": avg[2] * 1e3},
            "spmv_pair_gbs": pair, "spmv_pair_frac": pair / HBM_PEAK_GBS,
            "certified_solve": {"method": "FP32 FISTA (at most 1000 iterations, gap test every 32) + FP64 polish",
                                "seconds": ts, "fista_iterations": rp["iterations"], "polish_rounds": rp["polish_rounds"],
                                "polish_pcg_iterations": rp["inner"], "rel_gap_fp64": rp["rel_gap"],
                                "rel_err_planted": rp["rel_err"]}}


def cpu_baseline_scaled(args, cfg, n, nnz):
    """The oracle's FP64 FISTA on the host, on a bounded sample of the
    workload: the same recipe (kappa, stages, s = n / sdiv) at n = 2^sample
    (the instance built by the oracle, not timed), a fixed number of timed
    iterations, and the rate scaled to the full instance by the ratio of the
    stored nonzeros (both products are linear in nnz).  The value is the
    oracle's C form with OpenMP on every usable host core (its iterates are
    the numpy oracle's bit for bit); the numpy oracle on one thread and the
    C form on one thread are reported beside it."""
    from oracle import cfista as CF
    from oracle import fista as F
    from oracle import instance as OI

    ns = 1 << min(args.cpu_sample_log2n, n.bit_length() - 1)
    ms_ = 2 * ns
    t0 = time.perf_counter()
    o = OI.Instance(ms_, ns, cfg["kappa"], max(1, ns // cfg["sdiv"]), 1.0, cfg["seed"], rounds=2)
    A = o.sparse_A()
    At = A.T.tocsr()
    pair = CF.CsrPair(A)
    gen_s = time.perf_counter() - t0
    scale = A.nnz / float(nnz)
    host = host_description()
    cores = host["usable_cores"]

    def rate_of(run, budget):
        t0 = time.perf_counter()
        run(2)
        per = (time.perf_counter() - t0) / 2
        iters = max(3, min(args.cpu_iters * 10, int(budget / max(per, 1e-9))))
        t0 = time.perf_counter()
        run(iters)
        return iters, iters / (time.perf_counter() - t0)

    it_c, rate_c = rate_of(lambda k: CF.fista(pair, o.b, 1.0, o.L, k, threads=cores), args.cpu_budget / 3)
    it_c1, rate_c1 = rate_of(lambda k: CF.fista(pair, o.b, 1.0, o.L, k, threads=1), args.cpu_budget / 3)
    mv, rmv = (lambda v: A @ v), (lambda v: At @ v)
    it_np, rate_np = rate_of(lambda k: F.fista(mv, rmv, o.b, 1.0, o.L, k), args.cpu_budget / 3)
    return {"value": rate_c * scale, "unit": "iters/s", "cores": cores, "kind": "oracle",
            "sample": f"{it_c} FP64 FISTA iterations of the CPU oracle in C with OpenMP on {cores} threads "
                      f"(bitwise the numpy oracle's iterates) on the same recipe at n = 2^{ns.bit_length() - 1} "
                      f"(nnz {A.nnz}; instance built by the oracle in {gen_s:.1f} s, not timed): {rate_c:.3f} "
                      f"iters/s there, scaled by nnz {A.nnz}/{nnz} to the full instance",
            "rate_at_sample": rate_c, "sample_n": ns,
            "one_thread": {"c_iters_per_s": rate_c1 * scale, "numpy_iters_per_s": rate_np * scale,
                           "c_rate_at_sample": rate_c1, "numpy_rate_at_sample": rate_np,
                           "iterations": {"c": it_c1, "numpy": it_np}},
            "host": host}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=64)
    ap.add_argument("--warmup", type=int, default=32)
    ap.add_argument("--check-every", type=int, default=0,
                    help="gap test period; 0: the largest period <= 32 dividing --steps and --warmup")
    ap.add_argument("--config", default="c3", choices=sorted(FISTA_CONFIGS),
                    help="fista workload: c3 the memory-scale instance (default), c2 the single large instance")
    ap.add_argument("--log2n", type=int, default=0, help="fista workload: override log2(n) of --config")
    ap.add_argument("--no-c2", action="store_true", help="fista workload: skip the n = 2^20 leg in extra")
    ap.add_argument("--no-windows", action="store_true",
                    help="fista workload: skip the side leg over the window tables (L1LS_STORE_WINDOWS)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--cpu-iters", type=int, default=10)
    ap.add_argument("--cpu-sample-log2n", type=int, default=22)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 1 GiB device copy (torch copy_) five times, to scale HBM counters")
    ap.add_argument("--profile-summary", action="store_true",
                    help="summarise rocprofv3 CSV directories (--kt, --fetch, --write, --copyf, --copyw) into --out")
    for d in ("kt", "fetch", "write", "copyf", "copyw"):
        ap.add_argument(f"--{d}")
    ap.add_argument("--stats-summary", action="store_true",
                    help="write the top kernels of the rocprofv3 --stats run in --kt to --out")
    ap.add_argument("--counter-summary", action="store_true",
                    help="summarise the PMC_PASSES counter runs in --pmc-dirs into --out")
    ap.add_argument("--pmc-dirs", nargs="*", default=[])
    ap.add_argument("--stats-title", default="")
    ap.add_argument("--kt-command", default="", help="profile summary: the kernel-trace command it came from")
    ap.add_argument("--pmc-command", default="", help="profile summary: the counter command it came from")
    ap.add_argument("--stats-command", default="")
    ap.add_argument("--stats-top", type=int, default=14)
    ap.add_argument("--out", default=PROFILE_SUMMARY)
    ap.add_argument("--workload", default="fista", choices=["fista", "serve", "batched", "path", "large", "table1", "grid"],
                    help="fista: the single large instance (default); serve: the request stream; "
                         "batched: 256 uneven instances; path: 64 taus on one instance; "
                         "large: the n = 2^26 instance, stored vs matrix-free, CG-Newton; "
                         "table1: the section 8.9 (Table 1) instance at n = 2^30, CG-Newton; "
                         "grid: the sections 8.4-8.6 instances, CG-Newton then FISTA")
    ap.add_argument("--large-log2n", type=int, default=26)
    ap.add_argument("--table1-log2n", type=int, default=30)
    ap.add_argument("--grid-log2n", type=int, default=22)
    ap.add_argument("--grid-newton", type=int, default=30)
    ap.add_argument("--grid-fista-max", type=int, default=20000)
    ap.add_argument("--grid-sections", nargs="*", default=None, help="subset of 8.4 8.5 8.6 3.2")
    ap.add_argument("--newton-steps", type=int, default=8)
    ap.add_argument("--instances", type=int, default=256)
    ap.add_argument("--batch-tol", type=float, default=1e-5)
    ap.add_argument("--batch-max-iter", type=int, default=20000)
    ap.add_argument("--path-log2n", type=int, default=16)
    ap.add_argument("--path-k", type=int, default=64)
    ap.add_argument("--path-max-iter", type=int, default=4000)
    ap.add_argument("--requests", type=int, default=200)
    ap.add_argument("--serve-warmup", type=int, default=10)
    ap.add_argument("--serve-tol", type=float, default=1e-6)
    ap.add_argument("--serve-max-iter", type=int, default=5000)
    ap.add_argument("--serve-slots", type=int, default=256)
    ap.add_argument("--serve-iters-per-tick", type=int, default=16)
    ap.add_argument("--serve-budget-gib", type=float, default=160.0)
    ap.add_argument("--serve-log2n-lo", type=int, default=10)
    ap.add_argument("--serve-log2n-hi", type=int, default=22)
    ap.add_argument("--rate-mults", type=float, nargs="+", default=[0.7])
    ap.add_argument("--serve-dump", default=None, help="append per-request rows (JSON lines) to this file")
    ap.add_argument("--serve-fp32-only", action="store_true",
                    help="serve FP32 results (no FP64 certificate or polish); the default finishes every "
                         "result in FP64, as the plain path does")
    ap.add_argument("--plain-max-mult", type=float, default=1.0,
                    help="skip the real-time plain run above this rate multiple (its queue grows without bound)")
    args = ap.parse_args()
    if args.profile_summary:
        write_profile_summary(args)
        return
    if args.stats_summary:
        write_stats_summary(args)
        return
    if args.counter_summary:
        write_counter_summary(args)
        return
    if args.copy_calibration:
        import torch
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 4, "copy_bytes_written": b.numel() * 4, "launches": 5}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    if args.workload != "fista":
        if "--check-every" not in sys.argv:
            args.check_every = 16
        if args.workload == "large" and "--steps" not in sys.argv:
            args.steps, args.warmup = 50, 5
        if args.workload == "table1" and "--steps" not in sys.argv:
            args.steps, args.warmup = 1, 1
        {"serve": bench_serve, "batched": bench_batched, "path": bench_path,
         "large": bench_large, "table1": bench_table1, "grid": bench_grid}[args.workload](args)
        return

    bench_fista(args)


if __name__ == "__main__":
    main()
