"""The byte models behind the benchmark's algorithmic rates, pinned to the
per-iteration figures derived by hand in the design notes: the stored pair
at the single-instance workload's sizes, the matrix-free iteration at
m = 2n (100 n bytes in FP32, plus 2 (12 + 4) n for the bucketing passes of
the windowed gathers) and the blocked pair (runs of four entries); and the
derived figures of the memory-path counter summary."""
import bench

N = 1 << 20


def test_stored_pair_bytes_at_the_single_instance_sizes():
    # residual: row_ptr, (col, val) per entry, x once, 4 m-vectors;
    # transpose: col_ptr, (row, val) per entry, r_y once, 3 n-vectors
    m, n, nnz = 2 * N, N, 16777188
    k1, k2 = bench.algorithmic_bytes(m, n, nnz)
    assert k1 == 180354852
    assert k2 == 4 * (n + 1) + 8 * nnz + 4 * m + 12 * n


def test_matrix_free_bytes():
    for n in (N, 1 << 26):
        assert bench.mf_bytes(2 * n, n) == 100 * n
        assert bench.mf_bytes(2 * n, n, windows=True) == 132 * n
        # FP64: every floating-point term doubles; the int32 maps (inv: n,
        # emb: m = 2n) do not
        assert bench.mf_bytes(2 * n, n, es=8) == 2 * 100 * n - 4 * n - 4 * 2 * n


def test_blocked_bytes_are_below_the_stored_ones():
    # four runs per column, 20 bytes per run of four entries against 32 for
    # four CSR/CSC entries
    m, n = 2 * N, N
    b1, b2 = bench.blocked_bytes(m, n, 4 * n)
    s1, s2 = bench.algorithmic_bytes(m, n, 16 * n)
    assert b2 == 80 * n + 4 * (m + 2) + 12 * n
    assert s1 - b1 == 8 * 16 * n - 20 * 4 * n - 8
    assert b1 < s1 and b2 < s2


def test_counter_summary_derives_latency_and_reads_in_flight(tmp_path):
    # bench.py --counter-summary on a synthetic counter file: per-kernel
    # medians over the largest grid, and the derived figures (Little's law:
    # reads in flight per CU = summed read latency / 256 / cycles per CU)
    import argparse
    import csv

    rows = []
    name = "void l1ls::k_residual<float, 10, false, true>(int const*)"
    vals = {"GRBM_GUI_ACTIVE": 8 * 1000.0, "TCP_TCC_READ_REQ_sum": 2000.0,
            "TCP_TCC_READ_REQ_LATENCY_sum": 256 * 1000.0 * 50, "TCP_PENDING_STALL_CYCLES_sum": 256 * 700.0,
            "TCC_REQ_sum": 400.0, "TCC_HIT_sum": 100.0, "TCP_UTCL1_REQUEST_sum": 1e6,
            "TCP_UTCL1_TRANSLATION_MISS_sum": 5.0}
    for disp, grid in ((1, 4096), (2, 4096), (3, 64)):
        for c, v in vals.items():
            rows.append({"Dispatch_Id": disp, "Grid_Size": grid, "Kernel_Name": name, "Counter_Name": c,
                         "Counter_Value": v * (1 if grid == 4096 else 1000)})
    d = tmp_path / "pmc"
    d.mkdir()
    with open(d / "x_counter_collection.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=list(rows[0].keys()))
        w.writeheader()
        w.writerows(rows)
    out = tmp_path / "summary.txt"
    args = argparse.Namespace(pmc_dirs=[str(d)], out=str(out), stats_title="", pmc_command="cmd")
    bench.write_counter_summary(args)
    got = {k.strip(): float(v) for k, v in (ln.split(":", 1) for ln in out.read_text().splitlines()
                                             if ln.startswith("residual_win."))}
    assert got["residual_win.l2_read_latency_cycles"] == 256 * 1000.0 * 50 / 2000.0
    assert got["residual_win.reads_in_flight_per_cu"] == 50.0
    assert got["residual_win.vl1d_waiting_on_l2"] == 0.7
    assert got["residual_win.l2_hit"] == 0.25
    assert got["residual_win.utcl1_miss"] == 5e-6
