// Blocked stored operator for two Givens stages per side.
//
// With G = S_2 S_1 and Q = S~_2 S~_1 (eq. (16), section 4), A = Q Sigma G^T
// is the sum over the n middle indices i of the rank-one terms
// sigma_i (Q e_i)(G e_i)^T.  In stage order (position p holds index pi(p)),
// G e_i touches the four consecutive positions 2k-1 .. 2k+2 (mod n) around
// the stage-1 pair k of i (stage 1 pairs (2k, 2k+1), stage 2 pairs
// (2k+1, 2k+2), section 4.2), and Q e_i the same four around its m-side
// pair.  So every row and every column of A is a short list of runs of four
// consecutive entries, each run the contribution of one middle index:
//   row p:    runs (i, G-run start, (sigma_i u_i[r]) w_i[0..3]),  0..4 per row
//   column a: runs (i, Q-run start, (sigma_i u_i[0..3]) w_i[c]),  exactly 4
// (u_i = Q e_i, w_i = G e_i, r and c the offsets of p and a in their runs).
// A run stores one int32 start and four FP32 values: 20 bytes for four
// entries against 32 in CSR/CSC, and its gather is one contiguous 16-byte
// span.  Row and column runs hold bit-identical values (the same product
// in the same order), so the two passes apply exactly A and A^T.
//
// Vectors that are gathered (x on the n side, r_y on the m side) live in an
// extended layout of N + 2 elements: e[q + 1] = v[q], e[0] = v[N - 1] and
// e[N + 1] = v[0], so the runs that wrap around (2k - 1 = -1 and
// 2k + 2 = N) read consecutive memory.  A run starting at position 2k - 1
// starts at element 2k of e (8-byte aligned).  The writers of v[0] and
// v[N - 1] also write the two copies.
#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"

using namespace l1ls;

namespace {

typedef float f2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));

// S_2 S_1 e_a on one side, as four values on the positions ext-1 .. ext+2
// (mod N) where ext = 2k and k = a >> 1 is the stage-1 pair of position a.
// The rotation on pair (f, g) sends e_f to c e_f + s e_g and e_g to
// -s e_f + c e_g (section 4, G(i, j, theta)).
struct StageRun {
    int32_t ext;
    double v[4];
};

__device__ __forceinline__ StageRun stage_run(const SideTables& T, int64_t a) {
    const int64_t half = T.N / 2;
    const int64_t k = a >> 1;
    const double c1 = T.cs[0][2 * k], s1 = T.cs[0][2 * k + 1];
    const double v0 = (a & 1) ? -s1 : c1;  // coefficient at position 2k
    const double v1 = (a & 1) ? c1 : s1;   // coefficient at position 2k + 1
    // position 2k is the second element of stage-2 pair k - 1 (2k - 1, 2k),
    // position 2k + 1 the first element of stage-2 pair k (2k + 1, 2k + 2)
    const int64_t ka = (k == 0) ? half - 1 : k - 1;
    const double c2a = T.cs[1][2 * ka], s2a = T.cs[1][2 * ka + 1];
    const double c2b = T.cs[1][2 * k], s2b = T.cs[1][2 * k + 1];
    StageRun R;
    R.ext = (int32_t)(2 * k);
    R.v[0] = -(v0 * s2a);
    R.v[1] = v0 * c2a;
    R.v[2] = v1 * c2b;
    R.v[3] = v1 * s2b;
    return R;
}

// The two stage-1 pairs whose runs cover position p, with p's offset in
// each run: p = 2j lies at offset 1 of run j and offset 3 of run j - 1;
// p = 2j + 1 at offset 0 of run j + 1 and offset 2 of run j (mod N/2).
__device__ __forceinline__ void covering_runs(int64_t p, int64_t half, int64_t (&k)[2], int (&off)[2]) {
    const int64_t j = p >> 1;
    if ((p & 1) == 0) {
        k[0] = j;
        off[0] = 1;
        k[1] = (j == 0) ? half - 1 : j - 1;
        off[1] = 3;
    } else {
        k[0] = (j + 1 == half) ? 0 : j + 1;
        off[0] = 0;
        k[1] = j;
        off[1] = 2;
    }
}

// Row runs of row position p: count (vals == nullptr) or fill at ptr[p].
__global__ void k_blk_rows(SideTables Tn, SideTables Tm, const double* __restrict__ sigma, int64_t n, int64_t m,
                           const int32_t* __restrict__ ptr, int32_t* __restrict__ cnt, int32_t* __restrict__ start,
                           f4* __restrict__ vals) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= m) return;
    int64_t k[2];
    int off[2];
    covering_runs(p, m / 2, k, off);
    int32_t e = vals ? ptr[p] : 0;
    int c = 0;
    for (int h = 0; h < 2; ++h)
        for (int64_t q = 2 * k[h]; q <= 2 * k[h] + 1; ++q) {
            const int32_t i = Tm.perm[q];
            if (i >= n) continue;
            ++c;
            if (!vals) continue;
            const StageRun u = stage_run(Tm, q);
            const StageRun w = stage_run(Tn, Tn.pinv[i]);
            const double su = sigma[i] * u.v[off[h]];
            f4 v;
            v.x = (float)(su * w.v[0]);
            v.y = (float)(su * w.v[1]);
            v.z = (float)(su * w.v[2]);
            v.w = (float)(su * w.v[3]);
            start[e] = w.ext;
            vals[e] = v;
            ++e;
        }
    if (!vals) cnt[p] = c;
}

// Column runs of column position a: slot h of column a at [h * n + a].
__global__ void k_blk_cols(SideTables Tn, SideTables Tm, const double* __restrict__ sigma, int64_t n,
                           int32_t* __restrict__ start, f4* __restrict__ vals) {
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n) return;
    int64_t k[2];
    int off[2];
    covering_runs(a, n / 2, k, off);
    int slot = 0;
    for (int h = 0; h < 2; ++h)
        for (int64_t q = 2 * k[h]; q <= 2 * k[h] + 1; ++q, ++slot) {
            const int32_t i = Tn.perm[q];
            const StageRun w = stage_run(Tn, q);
            const StageRun u = stage_run(Tm, Tm.pinv[i]);
            const double wc = w.v[off[h]];
            const double s = sigma[i];
            f4 v;
            v.x = (float)((s * u.v[0]) * wc);
            v.y = (float)((s * u.v[1]) * wc);
            v.z = (float)((s * u.v[2]) * wc);
            v.w = (float)((s * u.v[3]) * wc);
            start[(int64_t)slot * n + a] = u.ext;
            vals[(int64_t)slot * n + a] = v;
        }
}

// e[0] = e[N], e[N + 1] = e[1] (the wrap copies of the extended layout).
__global__ void k_blk_wrap(float* __restrict__ e, int64_t N) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        e[0] = e[N];
        e[N + 1] = e[1];
    }
}

__device__ __forceinline__ float run_dot(f4 v, f2 a, f2 b) {
    return v.x * a.x + v.y * a.y + v.z * b.x + v.w * b.y;
}

constexpr int kRowRuns = 4;  // runs per row at most (four Q-neighbours)
constexpr int kRowQ = 3;     // branch-free rounds of 64 runs per row tile
constexpr int kColRuns = 4;  // runs per column (four G-neighbours)

// Residual pass over the row runs, one tile of 64 rows per wave:
//   r_x = A x - b,  r_y = (1 + beta) r_x - beta r_x,prev   (init: r_y = r_x)
// with the FP64 partials of k_residual.  xe: x in the extended layout;
// rx: m; rye: r_y in the extended layout.  PLAIN: rx = A x only.
template <bool PLAIN>
__global__ __launch_bounds__(L1LS_BLOCK) void k_blk_residual(
    const int32_t* __restrict__ ptr, const int32_t* __restrict__ start, const f4* __restrict__ val,
    const float* __restrict__ xe, const float* __restrict__ b, float* __restrict__ rx, float* __restrict__ rye,
    float beta, int64_t m, int init, double* __restrict__ part, const GapState* __restrict__ gs, int stats) {
    const int32_t done = gs ? __builtin_nontemporal_load(&gs->done) : 0;  // guards the stores only
    __shared__ float lds[L1LS_BLOCK / L1LS_WAVE][kTile * kRowRuns];
    const int lane = threadIdx.x % L1LS_WAVE;
    const int wid = threadIdx.x / L1LS_WAVE;
    const int64_t row0 = ((int64_t)blockIdx.x * (L1LS_BLOCK / L1LS_WAVE) + wid) * kTile;
    const int64_t i = row0 + lane;
    const bool live = i < m;
    int32_t pb = 0, pe = 0;
    float bi = 0.f, rprev = 0.f;
    if (live) {
        pb = ptr[i];
        pe = ptr[i + 1];
        if (!PLAIN) {
            bi = __builtin_nontemporal_load(b + i);
            if (!init) rprev = __builtin_nontemporal_load(rx + i);
        }
    }
    const int lastlane = (row0 + kTile <= m) ? kTile - 1 : (m > row0 ? (int)(m - row0 - 1) : 0);
    const int32_t beg = __builtin_amdgcn_readfirstlane(__shfl(pb, 0, L1LS_WAVE));
    const int32_t end = __builtin_amdgcn_readfirstlane(__shfl(pe, lastlane, L1LS_WAVE));
    const int32_t cnt = (row0 < m) ? end - beg : 0;  // wave-uniform, <= 64 * kRowRuns
    if (cnt > 0) {  // wave-uniform
        const int32_t* __restrict__ sb = start + beg;
        const f4* __restrict__ vb = val + beg;
        const int32_t last = cnt - 1;
        // The first kRowQ * 64 runs without branches, so that all loads of a
        // lane are in flight together: lanes past the end reload the last run
        // (in bounds) and store nothing.  A tile of 64 rows has 4 * 64 * n / m
        // runs on average; the rest goes through the tail loop.
        int32_t s[kRowQ];
        f4 v[kRowQ];
        f2 ga[kRowQ], gb[kRowQ];
#pragma unroll
        for (int q = 0; q < kRowQ; ++q) s[q] = __builtin_nontemporal_load(sb + min(q * kTile + lane, last));
#pragma unroll
        for (int q = 0; q < kRowQ; ++q) v[q] = __builtin_nontemporal_load(vb + min(q * kTile + lane, last));
#pragma unroll
        for (int q = 0; q < kRowQ; ++q) {
            ga[q] = *reinterpret_cast<const f2*>(xe + s[q]);
            gb[q] = *reinterpret_cast<const f2*>(xe + s[q] + 2);
        }
#pragma unroll
        for (int q = 0; q < kRowQ; ++q)
            if (q * kTile + lane <= last) lds[wid][q * kTile + lane] = run_dot(v[q], ga[q], gb[q]);
        for (int32_t e = kRowQ * kTile + lane; e <= last; e += kTile) {
            const int32_t se = sb[e];
            lds[wid][e] = run_dot(vb[e], *reinterpret_cast<const f2*>(xe + se),
                                  *reinterpret_cast<const f2*>(xe + se + 2));
        }
    }
    __syncthreads();
    double st[3] = {0.0, 0.0, 0.0};
    if (live && !done) {
        float acc = 0.f;
        for (int32_t k = pb - beg; k < pe - beg; ++k) acc += lds[wid][k];
        if (PLAIN) {
            rx[i] = acc;
            return;
        }
        const float r = acc - bi;
        const float yv = init ? r : (1.f + beta) * r - beta * rprev;
        st_stream(rx + i, r);
        st_stream(rye + 1 + i, yv);
        if (i == 0) rye[m + 1] = yv;
        if (i == m - 1) rye[0] = yv;
        st[0] = (double)r * (double)r;
        st[1] = (double)yv * (double)yv;
        st[2] = (double)bi * (double)yv;
    }
    if (PLAIN || !stats) return;  // launch-uniform
    block_reduce_stats<3, 3>(st);
    if (threadIdx.x == 0 && !done) {
        part[3 * blockIdx.x + 0] = st[0];
        part[3 * blockIdx.x + 1] = st[1];
        part[3 * blockIdx.x + 2] = st[2];
    }
}

// Transpose pass with the prox step over the column runs, one column per
// lane: g = A^T r_y, y = x_{k-1} + beta (x_{k-1} - x_{k-2}),
// x_k = soft(y - g / L, tau / L), with the FP64 partials of
// k_transpose_prox.  xc: x_{k-1} (n); xpe: the slot of x_{k-2}, extended
// layout, receives x_k.  PLAIN: xpe[1 + a] = g only.
template <bool PLAIN>
__global__ __launch_bounds__(L1LS_BLOCK) void k_blk_transpose_prox(
    const int32_t* __restrict__ start, const f4* __restrict__ val, const float* __restrict__ rye,
    const float* __restrict__ xc, float* __restrict__ xpe, float beta, float L, float thr, int64_t n,
    double* __restrict__ part, const GapState* __restrict__ gs, int stats) {
    const int32_t done = gs ? __builtin_nontemporal_load(&gs->done) : 0;
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = a < n;
    const int64_t ac = live ? a : n - 1;  // dead lanes load column n - 1 and store nothing
    int32_t s[kColRuns];
    f4 v[kColRuns];
#pragma unroll
    for (int h = 0; h < kColRuns; ++h) s[h] = __builtin_nontemporal_load(start + h * n + ac);
#pragma unroll
    for (int h = 0; h < kColRuns; ++h) v[h] = __builtin_nontemporal_load(val + h * n + ac);
    float xcur = 0.f, xprev = 0.f;
    if (!PLAIN) {
        xcur = __builtin_nontemporal_load(xc + ac);
        xprev = __builtin_nontemporal_load(xpe + 1 + ac);
    }
    f2 ga[kColRuns], gb[kColRuns];
#pragma unroll
    for (int h = 0; h < kColRuns; ++h) {
        ga[h] = *reinterpret_cast<const f2*>(rye + s[h]);
        gb[h] = *reinterpret_cast<const f2*>(rye + s[h] + 2);
    }
    float acc = 0.f;
#pragma unroll
    for (int h = 0; h < kColRuns; ++h) acc += run_dot(v[h], ga[h], gb[h]);
    double st[2] = {0.0, 0.0};  // sum |x_k|, max |g|
    if (live && !done) {
        if (PLAIN) {
            xpe[1 + a] = acc;
            return;
        }
        const float y = xcur + beta * (xcur - xprev);
        const float xn = soft_threshold<float>(y - acc / L, thr);
        st_stream(xpe + 1 + a, xn);
        if (a == 0) xpe[n + 1] = xn;
        if (a == n - 1) xpe[0] = xn;
        st[0] = fabs((double)xn);
        st[1] = fabs((double)acc);
    }
    if (PLAIN || !stats) return;
    block_reduce_stats<2, 1>(st);
    if (threadIdx.x == 0 && !done) {
        part[2 * blockIdx.x + 0] = st[1];
        part[2 * blockIdx.x + 1] = st[0];
    }
}

inline unsigned blk_row_grid(int64_t m) {
    const int64_t tiles = (m + kTile - 1) / kTile;
    return (unsigned)std::max<int64_t>(1, (tiles + 3) / 4);
}
inline unsigned blk_col_grid(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + L1LS_BLOCK - 1) / L1LS_BLOCK); }

__global__ void k_blk_gather_in(const float* __restrict__ in, float* __restrict__ e, const int32_t* __restrict__ of,
                                int64_t N) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const float v = in[of[p]];
    e[p + 1] = v;
    if (p == 0) e[N + 1] = v;
    if (p == N - 1) e[0] = v;
}

__global__ void k_blk_scatter_out(const float* __restrict__ o, float* __restrict__ out, const int32_t* __restrict__ of,
                                  int64_t N) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    out[of[p]] = o[p];
}

}  // namespace

// Build the row and column runs (requires two stages and the stage layout).
l1ls_status build_blocks(l1ls_instance* I, hipStream_t s, DevArena& tmp) {
    if (I->rounds != 2 || I->layout != L1LS_LAYOUT_STAGE || I->n < 4) return L1LS_E_UNSUPPORTED;
    const int64_t n = I->n, m = I->m;
    if (kColRuns * n >= ((int64_t)1 << 31)) return L1LS_E_UNSUPPORTED;
    int32_t* cnt = nullptr;
    L1LS_TRY(tmp.alloc(&cnt, m));
    L1LS_TRY(I->arena.alloc(&I->blk_rptr, m + 1));
    hipLaunchKernelGGL(k_blk_rows, grid_1d(m), dim3(L1LS_BLOCK), 0, s, I->side[0], I->side[1], I->sigma, n, m,
                       (const int32_t*)nullptr, cnt, (int32_t*)nullptr, (f4*)nullptr);
    L1LS_TRY(exclusive_scan_i32(cnt, I->blk_rptr, m, s, tmp));
    int32_t nr = 0;
    HIP_TRY(hipMemcpyAsync(&nr, I->blk_rptr + m, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    // every middle index contributes one run to each of four rows
    if (nr != kRowRuns * n) return L1LS_E_STATE;
    I->blk_nruns = nr;
    f4* rv = nullptr;
    f4* cv = nullptr;
    L1LS_TRY(I->arena.alloc(&I->blk_rstart, nr));
    L1LS_TRY(I->arena.alloc(&rv, nr));
    L1LS_TRY(I->arena.alloc(&I->blk_cstart, kColRuns * n));
    L1LS_TRY(I->arena.alloc(&cv, kColRuns * n));
    I->blk_rval = reinterpret_cast<float*>(rv);
    I->blk_cval = reinterpret_cast<float*>(cv);
    hipLaunchKernelGGL(k_blk_rows, grid_1d(m), dim3(L1LS_BLOCK), 0, s, I->side[0], I->side[1], I->sigma, n, m,
                       (const int32_t*)I->blk_rptr, cnt, I->blk_rstart, rv);
    hipLaunchKernelGGL(k_blk_cols, grid_1d(n), dim3(L1LS_BLOCK), 0, s, I->side[0], I->side[1], I->sigma, n,
                       I->blk_cstart, cv);
    HIP_TRY(hipGetLastError());
    return L1LS_OK;
}

// One residual pass of the FISTA driver over the blocked operator.
void blk_residual_launch(const l1ls_instance* I, const float* xe, const float* b, float* rx, float* rye, float beta,
                         int init, double* part, const GapState* gs, int stats, hipStream_t s) {
    hipLaunchKernelGGL((k_blk_residual<false>), dim3(blk_row_grid(I->m)), dim3(L1LS_BLOCK), 0, s, I->blk_rptr,
                       I->blk_rstart, reinterpret_cast<const f4*>(I->blk_rval), xe, b, rx, rye, beta, I->m, init,
                       part, gs, stats);
}

// One transpose pass (with the prox step) over the blocked operator.
void blk_transpose_launch(const l1ls_instance* I, const float* rye, const float* xc, float* xpe, float beta, float L,
                          float thr, double* part, const GapState* gs, int stats, hipStream_t s) {
    hipLaunchKernelGGL((k_blk_transpose_prox<false>), dim3(blk_col_grid(I->n)), dim3(L1LS_BLOCK), 0, s,
                       I->blk_cstart, reinterpret_cast<const f4*>(I->blk_cval), rye, xc, xpe, beta, L, thr, I->n,
                       part, gs, stats);
}

int blk_row_blocks(int64_t m) { return (int)blk_row_grid(m); }
int blk_col_blocks(int64_t n) { return (int)blk_col_grid(n); }

void blk_wrap_launch(float* e, int64_t N, hipStream_t s) {
    hipLaunchKernelGGL(k_blk_wrap, dim3(1), dim3(64), 0, s, e, N);
}

// out = A in (trans 0) or A^T in (trans 1), FP32, vectors in the original
// order, through the same product code as the FISTA passes.
l1ls_status apply_blocked(const l1ls_instance* I, int trans, const float* in, float* out, hipStream_t s) {
    if (!I->blk_rptr) return L1LS_E_UNSUPPORTED;
    DevArena tmp;
    const int64_t nin = trans ? I->m : I->n, nout = trans ? I->n : I->m;
    float *e = nullptr, *o = nullptr;
    auto done = [&](l1ls_status st) {
        (void)hipStreamSynchronize(s);
        tmp.release();
        return st;
    };
    l1ls_status st;
    if ((st = tmp.alloc(&e, nin + 2)) != L1LS_OK) return done(st);
    if ((st = tmp.alloc(&o, nout + 2)) != L1LS_OK) return done(st);
    hipLaunchKernelGGL(k_blk_gather_in, grid_1d(nin), dim3(L1LS_BLOCK), 0, s, in, e,
                       trans ? I->op_row_of : I->op_col_of, nin);
    if (trans == 0) {
        hipLaunchKernelGGL((k_blk_residual<true>), dim3(blk_row_grid(I->m)), dim3(L1LS_BLOCK), 0, s, I->blk_rptr,
                           I->blk_rstart, reinterpret_cast<const f4*>(I->blk_rval), e, (const float*)nullptr, o,
                           (float*)nullptr, 0.f, I->m, 1, (double*)nullptr, (const GapState*)nullptr, 0);
        hipLaunchKernelGGL(k_blk_scatter_out, grid_1d(nout), dim3(L1LS_BLOCK), 0, s, o, out, I->op_row_of, nout);
    } else {
        hipLaunchKernelGGL((k_blk_transpose_prox<true>), dim3(blk_col_grid(I->n)), dim3(L1LS_BLOCK), 0, s,
                           I->blk_cstart, reinterpret_cast<const f4*>(I->blk_cval), e, (const float*)nullptr, o,
                           0.f, 1.f, 0.f, I->n, (double*)nullptr, (const GapState*)nullptr, 0);
        hipLaunchKernelGGL(k_blk_scatter_out, grid_1d(nout), dim3(L1LS_BLOCK), 0, s, o + 1, out, I->op_col_of, nout);
    }
    if (hipGetLastError() != hipSuccess) return done(L1LS_E_HIP);
    return done(L1LS_OK);
}
