"""The byte models behind the benchmark's algorithmic rates, pinned to the
per-iteration figures derived by hand in the design notes: the stored pair
at the single-instance workload's sizes, the matrix-free iteration at
m = 2n (100 n bytes in FP32, plus 2 (12 + 4) n for the bucketing passes of
the windowed gathers) and the blocked pair (runs of four entries)."""
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
