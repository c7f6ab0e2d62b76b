// Regularisation path: FISTA (section 8.1) for up to 64 values of tau on one
// instance at once, as sparse-times-dense products (section 8.6 varies tau).
//
// X (n x 64) and the residuals R_x, R_y (m x 64) are row-major in operator
// order; lane c of a wave owns column c (one tau).  All columns start at
// x_0 = 0 and advance in lockstep, so t_k and beta_k are shared; a column
// whose gap test passed is frozen (its lane stops storing).  Each nonzero
// of A is read once per iteration and drives a 256-byte coalesced gather of
// a row of X (or R_y).  Per-column FP64 statistics feed a per-column
// duality gap with that column's tau.
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"

l1ls_status gap_fp64(const l1ls_instance* I, double tau, const double* x, double* P, double* D, double* gap,
                     hipStream_t s, DevAlloc* al = nullptr);
l1ls_status polish_fp64(const l1ls_instance* I, double tau, double* x_dev, hipStream_t stream, int* rounds_out,
                        int64_t* pcg_iters_out, double support_tol, DevAlloc* al = nullptr);

using namespace l1ls;

namespace {

constexpr int kCols = 64;          // tau values per launch (one per lane)
constexpr int kPathWaves = 16;     // waves per workgroup
constexpr int kRowsPerWave = 2;    // rows (columns) per wave
constexpr int kRowsPerBlock = kPathWaves * kRowsPerWave;

struct PathCol {  // per tau column, device
    double tau, thr;   // tau and tau / L
    double P, D, gap;
    int64_t conv_iter;
    int32_t done, nonfinite;
};

// sum_k val[k] * V[idx[k], lane] over entries [pb, pe) (at most kMaxNnz):
// lanes 0..15 fetch the entries, every lane gathers its column of the rows
// of V they name (the second 8 only when the row has more than 8 entries).
__device__ __forceinline__ float row_dot(const int32_t* __restrict__ idx, const float* __restrict__ val,
                                         const float* __restrict__ V, int32_t pb, int32_t pe, int lane) {
    const int32_t cnt = pe - pb;
    if (cnt <= 0) return 0.f;
    const int32_t q = min(lane, cnt - 1);
    const int32_t my_c = (lane < kMaxNnz) ? idx[pb + q] : 0;
    const float my_v = (lane < kMaxNnz && lane < cnt) ? val[pb + q] : 0.f;
    float g[kMaxNnz];
    float w[kMaxNnz];
#pragma unroll
    for (int e = 0; e < kMaxNnz; ++e) {
        w[e] = 0.f;
        g[e] = 0.f;
    }
#pragma unroll
    for (int e = 0; e < kMaxNnz / 2; ++e) {
        const int32_t c = __builtin_amdgcn_readlane(my_c, e);
        w[e] = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int32_t, my_v), e));
        g[e] = V[(size_t)c * kCols + lane];
    }
    if (cnt > kMaxNnz / 2) {  // wave-uniform
#pragma unroll
        for (int e = kMaxNnz / 2; e < kMaxNnz; ++e) {
            const int32_t c = __builtin_amdgcn_readlane(my_c, e);
            w[e] = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int32_t, my_v), e));
            g[e] = V[(size_t)c * kCols + lane];
        }
    }
    float acc = 0.f;
#pragma unroll
    for (int e = 0; e < kMaxNnz; ++e) acc += w[e] * g[e];
    return acc;
}

// Two rows of A with the same column list (a stage-2 pair of rows, or of
// columns in the CSC: both members reach the same positions through the
// stages, so they share their pattern): one gather of V per entry serves
// both dot products.  Falls back to two row_dot calls when the lists differ.
__device__ __forceinline__ void row_dot_pair(const int32_t* __restrict__ idx, const float* __restrict__ val,
                                             const float* __restrict__ V, int32_t pb0, int32_t pe0, int32_t pb1,
                                             int32_t pe1, int lane, float& acc0, float& acc1) {
    const int32_t cnt = pe0 - pb0;
    bool same = (cnt == pe1 - pb1) && cnt > 0;
    int32_t c0 = 0;
    if (same) {  // wave-uniform
        const int32_t q = min(lane, cnt - 1);
        c0 = (lane < kMaxNnz) ? idx[pb0 + q] : 0;
        const int32_t c1 = (lane < kMaxNnz) ? idx[pb1 + q] : 0;
        same = __ballot(c0 != c1) == 0;
    }
    if (!same) {
        acc0 = row_dot(idx, val, V, pb0, pe0, lane);
        acc1 = row_dot(idx, val, V, pb1, pe1, lane);
        return;
    }
    const int32_t q = min(lane, cnt - 1);
    const float v0 = (lane < kMaxNnz && lane < cnt) ? val[pb0 + q] : 0.f;
    const float v1 = (lane < kMaxNnz && lane < cnt) ? val[pb1 + q] : 0.f;
    float g[kMaxNnz], w0[kMaxNnz], w1[kMaxNnz];
#pragma unroll
    for (int e = 0; e < kMaxNnz; ++e) {
        g[e] = 0.f;
        w0[e] = 0.f;
        w1[e] = 0.f;
    }
#pragma unroll
    for (int e = 0; e < kMaxNnz / 2; ++e) {
        const int32_t c = __builtin_amdgcn_readlane(c0, e);
        w0[e] = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int32_t, v0), e));
        w1[e] = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int32_t, v1), e));
        g[e] = V[(size_t)c * kCols + lane];
    }
    if (cnt > kMaxNnz / 2) {  // wave-uniform
#pragma unroll
        for (int e = kMaxNnz / 2; e < kMaxNnz; ++e) {
            const int32_t c = __builtin_amdgcn_readlane(c0, e);
            w0[e] = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int32_t, v0), e));
            w1[e] = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int32_t, v1), e));
            g[e] = V[(size_t)c * kCols + lane];
        }
    }
    float a0 = 0.f, a1 = 0.f;
#pragma unroll
    for (int e = 0; e < kMaxNnz; ++e) {
        a0 += w0[e] * g[e];
        a1 += w1[e] * g[e];
    }
    acc0 = a0;
    acc1 = a1;
}

template <int NS, int NSUM>
__device__ __forceinline__ void block_reduce_cols(double (&v)[NS], double* __restrict__ out) {
    // across the waves of the block, per lane (column); out[stat * 64 + lane]
    __shared__ double red[kPathWaves][NS][kCols];
    const int lane = threadIdx.x % L1LS_WAVE, wid = threadIdx.x / L1LS_WAVE;
#pragma unroll
    for (int s = 0; s < NS; ++s) red[wid][s][lane] = v[s];
    __syncthreads();
    if (wid == 0) {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            double a = red[0][s][lane];
            for (int w = 1; w < kPathWaves; ++w) a = (s < NSUM) ? a + red[w][s][lane] : fmax(a, red[w][s][lane]);
            out[s * kCols + lane] = a;
        }
    }
}

// residual pass: R_x = A X - b 1^T, R_y = (1+beta) R_x - beta R_x,prev
__global__ __launch_bounds__(kPathWaves * L1LS_WAVE) void kp_residual(
    const int32_t* __restrict__ ptr, const int32_t* __restrict__ col, const float* __restrict__ val,
    const float* __restrict__ X, const float* __restrict__ b, float* __restrict__ Rx, float* __restrict__ Ry,
    float beta, int init, int64_t m, const PathCol* __restrict__ pc, int32_t ncols, double* __restrict__ part,
    int stats) {
    const int lane = threadIdx.x % L1LS_WAVE, wid = threadIdx.x / L1LS_WAVE;
    const bool on = lane < ncols && !pc[lane].done;
    double v[3] = {0.0, 0.0, 0.0};
    // wave w owns the stage-2 pair of rows (2w+1, 2w+2 mod m)
    const int64_t row0 = (int64_t)blockIdx.x * kRowsPerBlock + wid * kRowsPerWave;
    if (row0 < m) {
        const int64_t rows[2] = {row0 + 1, (row0 + 2 == m) ? 0 : row0 + 2};
        float acc[2];
        row_dot_pair(col, val, X, ptr[rows[0]], ptr[rows[0] + 1], ptr[rows[1]], ptr[rows[1] + 1], lane, acc[0],
                     acc[1]);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int64_t i = rows[q];
            const float bi = b[i];
            const size_t o = (size_t)i * kCols + lane;
            const float r = acc[q] - bi;
            const float yv = init ? r : (1.f + beta) * r - beta * Rx[o];
            if (on) {
                Rx[o] = r;
                Ry[o] = yv;
                v[0] += (double)r * (double)r;
                v[1] += (double)yv * (double)yv;
                v[2] += (double)bi * (double)yv;
            }
        }
    }
    if (!stats) return;
    block_reduce_cols<3, 3>(v, part + (size_t)blockIdx.x * 3 * kCols);
}

// transpose pass with the prox step per column: X_k = soft(Y - (A^T R_y)/L, tau_c/L)
__global__ __launch_bounds__(kPathWaves * L1LS_WAVE) void kp_transpose(
    const int32_t* __restrict__ ptr, const int32_t* __restrict__ row, const float* __restrict__ val,
    const float* __restrict__ Ry, const float* __restrict__ Xc, float* __restrict__ Xp, float beta, float L,
    int64_t n, const PathCol* __restrict__ pc, int32_t ncols, double* __restrict__ part, int stats) {
    const int lane = threadIdx.x % L1LS_WAVE, wid = threadIdx.x / L1LS_WAVE;
    const bool on = lane < ncols && !pc[lane].done;
    const float thr = on ? (float)pc[lane].thr : 0.f;
    double v[2] = {0.0, 0.0};  // sum |x| | max |g|
    // wave w owns the stage-2 pair of columns (2w+1, 2w+2 mod n)
    const int64_t col0 = (int64_t)blockIdx.x * kRowsPerBlock + wid * kRowsPerWave;
    if (col0 < n) {
        const int64_t cols[2] = {col0 + 1, (col0 + 2 == n) ? 0 : col0 + 2};
        float gq[2];
        row_dot_pair(row, val, Ry, ptr[cols[0]], ptr[cols[0] + 1], ptr[cols[1]], ptr[cols[1] + 1], lane, gq[0],
                     gq[1]);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int64_t j = cols[q];
            const float g = gq[q];
            const size_t o = (size_t)j * kCols + lane;
            const float xcur = Xc[o];
            const float y = xcur + beta * (xcur - Xp[o]);
            const float xn = soft_threshold<float>(y - g / L, thr);
            if (on) {
                Xp[o] = xn;
                v[0] += fabs((double)xn);
                v[1] = fmax(v[1], fabs((double)g));
            }
        }
    }
    if (!stats) return;
    block_reduce_cols<2, 1>(v, part + (size_t)blockIdx.x * 2 * kCols);
}

// Per-column gap from the partials, in two fixed-order stages: kp_gap_sum
// (kGapBlocks workgroups) folds contiguous slices of the workgroup partials
// into [kGapBlocks][5][64]; kp_gap (one workgroup) folds those and applies
// the gap test per column.
constexpr int kGapBlocks = 64;

__global__ __launch_bounds__(1024) void kp_gap_sum(const double* __restrict__ p1cur,
                                                   const double* __restrict__ p1prev, int g1,
                                                   const double* __restrict__ p2, int g2, double* __restrict__ out) {
    __shared__ double red[16][5][kCols];
    const int c = threadIdx.x % kCols, grp = threadIdx.x / kCols;
    const int s1 = (g1 + kGapBlocks - 1) / kGapBlocks, s2 = (g2 + kGapBlocks - 1) / kGapBlocks;
    const int b1 = blockIdx.x * s1, e1 = min(g1, b1 + s1), b2 = blockIdx.x * s2, e2 = min(g2, b2 + s2);
    double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int bk = b1 + grp; bk < e1; bk += 16) {
        v[0] += p1cur[((size_t)bk * 3 + 0) * kCols + c];
        v[1] += p1prev[((size_t)bk * 3 + 1) * kCols + c];
        v[2] += p1prev[((size_t)bk * 3 + 2) * kCols + c];
    }
    for (int bk = b2 + grp; bk < e2; bk += 16) {
        v[3] += p2[((size_t)bk * 2 + 0) * kCols + c];
        v[4] = fmax(v[4], p2[((size_t)bk * 2 + 1) * kCols + c]);
    }
    for (int q = 0; q < 5; ++q) red[grp][q][c] = v[q];
    __syncthreads();
    if (grp != 0) return;
    for (int q = 0; q < 5; ++q) {
        double a = red[0][q][c];
        for (int r = 1; r < 16; ++r) a = (q < 4) ? a + red[r][q][c] : fmax(a, red[r][q][c]);
        out[((size_t)blockIdx.x * 5 + q) * kCols + c] = a;
    }
}

__global__ __launch_bounds__(kCols) void kp_gap(const double* __restrict__ sums, PathCol* __restrict__ pc,
                                                int32_t ncols, double tol, int64_t iter) {
    const int c = threadIdx.x;
    if (c >= ncols) return;
    double v[5];
    for (int q = 0; q < 5; ++q) {
        double a = sums[(size_t)q * kCols + c];
        for (int b = 1; b < kGapBlocks; ++b) {
            const double x = sums[((size_t)b * 5 + q) * kCols + c];
            a = (q < 4) ? a + x : fmax(a, x);
        }
        v[q] = a;
    }
    PathCol& P = pc[c];
    if (P.done) return;
    const double tau = P.tau;
    const double Pv = tau * v[3] + 0.5 * v[0];
    const double theta = (v[4] <= tau) ? 1.0 : tau / v[4];
    const double Dv = -0.5 * theta * theta * v[1] - theta * v[2];
    const double gap = (Pv - Dv) / fabs(Pv);
    P.P = Pv;
    P.D = Dv;
    P.gap = gap;
    const bool finite = (Pv == Pv) && (Dv == Dv) && (Pv - Pv == 0.0) && (Dv - Dv == 0.0);
    if (!finite) {
        P.nonfinite = 1;
        P.done = 1;
        P.conv_iter = iter;
    } else if (tol > 0.0 && gap <= tol) {
        P.done = 1;
        P.conv_iter = iter;
    }
}

__global__ void kp_fill(float* __restrict__ a, int64_t N) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) a[i] = 0.f;
}

// X_out column c (original order, FP64, column-major n x ncols) from X (operator order, row-major n x 64)
__global__ void kp_extract(const float* __restrict__ X0, const float* __restrict__ X1,
                           const PathCol* __restrict__ pc, int64_t kfinal, const int32_t* __restrict__ pos,
                           int64_t n, int32_t ncols, double* __restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * ncols) return;
    const int64_t j = t % n;
    const int c = (int)(t / n);
    const int64_t kc = pc[c].conv_iter >= 0 ? pc[c].conv_iter : kfinal;
    const float* X = (kc & 1) ? X1 : X0;
    const int64_t p = pos ? pos[j] : j;
    out[t] = (double)X[(size_t)p * kCols + c];
}

inline dim3 g1d(int64_t N) { return dim3((unsigned)std::max<int64_t>(1, (N + L1LS_BLOCK - 1) / L1LS_BLOCK)); }

inline double next_t_host(double t) {
#pragma clang fp contract(off)
    return (1.0 + std::sqrt(1.0 + 4.0 * t * t)) / 2.0;
}

}  // namespace

extern "C" l1ls_status l1ls_solve_fista_path(const l1ls_instance* I, const double* taus, int32_t k,
                                             const l1ls_solve_opts* o, double* X_out, l1ls_report* reports) {
    if (!I || !taus || !o || !X_out || !reports || k < 1 || k > kCols) return L1LS_E_ARG;
    if (!I->csr_v32 || !I->csc_v32) return L1LS_E_UNSUPPORTED;
    if (o->check_every < 1 || o->max_iter < 0 || !(o->rel_gap_tol >= 0.0)) return L1LS_E_ARG;
    if (o->polish < 0 || o->polish > 2) return L1LS_E_ARG;
    if (o->polish && (!I->csr_v64 || !I->csc_v64)) return L1LS_E_UNSUPPORTED;
    for (int c = 0; c < k; ++c)
        if (!(taus[c] > 0.0) || !is_finite(taus[c])) return L1LS_E_ARG;
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = (hipStream_t)o->stream;
    const int64_t n = I->n, m = I->m;
    const double L = o->L > 0 ? o->L : I->L;
    const int g1 = (int)((m + kRowsPerBlock - 1) / kRowsPerBlock);
    const int g2 = (int)((n + kRowsPerBlock - 1) / kRowsPerBlock);
    DevArena A;
    float *X0 = nullptr, *X1 = nullptr, *Rx = nullptr, *Ry = nullptr;
    double *p1 = nullptr, *p2 = nullptr;
    PathCol* pc = nullptr;
    L1LS_TRY(A.alloc(&X0, (size_t)n * kCols));
    L1LS_TRY(A.alloc(&X1, (size_t)n * kCols));
    L1LS_TRY(A.alloc(&Rx, (size_t)m * kCols));
    L1LS_TRY(A.alloc(&Ry, (size_t)m * kCols));
    L1LS_TRY(A.alloc(&p1, (size_t)2 * g1 * 3 * kCols));
    L1LS_TRY(A.alloc(&p2, (size_t)g2 * 2 * kCols));
    L1LS_TRY(A.alloc(&pc, kCols));
    double* gsum = nullptr;
    L1LS_TRY(A.alloc(&gsum, (size_t)kGapBlocks * 5 * kCols));
    std::vector<PathCol> hc(kCols);
    for (int c = 0; c < kCols; ++c) {
        std::memset(&hc[c], 0, sizeof(PathCol));
        hc[c].tau = c < k ? taus[c] : 1.0;
        hc[c].thr = hc[c].tau / L;
        hc[c].conv_iter = -1;
        hc[c].done = c < k ? 0 : 1;
    }
    HIP_TRY(hipMemcpyAsync(pc, hc.data(), kCols * sizeof(PathCol), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(kp_fill, g1d((int64_t)n * kCols), dim3(L1LS_BLOCK), 0, s, X0, (int64_t)n * kCols);
    hipLaunchKernelGGL(kp_fill, g1d((int64_t)n * kCols), dim3(L1LS_BLOCK), 0, s, X1, (int64_t)n * kCols);
    const dim3 blk(kPathWaves * L1LS_WAVE);
    // R_x,0 = R_y,1 = A X_0 - b
    hipLaunchKernelGGL(kp_residual, dim3(g1), blk, 0, s, I->csr_ptr, I->csr_col, I->csr_v32, X0, I->b32_op, Rx, Ry,
                       0.f, 1, m, pc, k, p1, 1);
    const int check = o->check_every;
    double t = 1.0, beta_prev = 0.0;
    int64_t it = 0;
    std::vector<PathCol> got(kCols);
    while (it < o->max_iter) {
        const int64_t step = std::min<int64_t>((int64_t)check * 4, o->max_iter - it);
        for (int64_t q = 0; q < step; ++q) {
            const int64_t kk = it + 1;
            const double tn = next_t_host(t);
            const double beta = (t - 1.0) / tn;
            const float* Xc = (kk - 1) & 1 ? X1 : X0;
            float* Xs = kk & 1 ? X1 : X0;
            const int chk = (kk % check == 0 || kk == o->max_iter);
            const int st1 = chk || ((kk + 1) % check == 0) || (kk + 1 == o->max_iter);
            hipLaunchKernelGGL(kp_transpose, dim3(g2), blk, 0, s, I->csc_ptr, I->csc_row, I->csc_v32, Ry, Xc, Xs,
                               (float)beta_prev, (float)L, n, pc, k, p2, chk);
            hipLaunchKernelGGL(kp_residual, dim3(g1), blk, 0, s, I->csr_ptr, I->csr_col, I->csr_v32, Xs, I->b32_op,
                               Rx, Ry, (float)beta, 0, m, pc, k, p1 + (size_t)(kk & 1) * g1 * 3 * kCols, st1);
            if (chk) {
                hipLaunchKernelGGL(kp_gap_sum, dim3(kGapBlocks), dim3(1024), 0, s,
                                   p1 + (size_t)(kk & 1) * g1 * 3 * kCols,
                                   p1 + (size_t)((kk - 1) & 1) * g1 * 3 * kCols, g1, p2, g2, gsum);
                hipLaunchKernelGGL(kp_gap, dim3(1), dim3(kCols), 0, s, gsum, pc, k, o->rel_gap_tol, kk);
            }
            beta_prev = beta;
            t = tn;
            it = kk;
        }
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(got.data(), pc, kCols * sizeof(PathCol), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        bool all = true;
        for (int c = 0; c < k; ++c) all = all && got[c].done;
        if (all) break;
    }
    hipLaunchKernelGGL(kp_extract, g1d((int64_t)n * k), dim3(L1LS_BLOCK), 0, s, X0, X1, pc, it, I->op_col_pos, n, k,
                       X_out);
    HIP_TRY(hipMemcpyAsync(got.data(), pc, kCols * sizeof(PathCol), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    A.release();
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    bool all = true;
    for (int c = 0; c < k; ++c) {
        l1ls_report& r = reports[c];
        std::memset(&r, 0, sizeof(r));
        r.iterations = got[c].conv_iter >= 0 ? got[c].conv_iter : it;
        r.primal = got[c].P;
        r.dual = got[c].D;
        r.rel_gap = got[c].gap;
        r.converged = (got[c].conv_iter >= 0 && !got[c].nonfinite) ? 1 : 0;
        r.rel_err = -1.0;
        r.seconds = secs;
        all = all && r.converged;
        if (got[c].nonfinite) return L1LS_E_NONFINITE;
    }
    if (o->polish) {
        // FP64 finish of each column at its own tau: the FP64 gap of the FP32
        // result, the polish of the reduced problem (13) where that gap
        // misses the tolerance (polish = 2) or always (polish = 1), and the
        // FP64 gap of what is returned
        all = true;
        for (int c = 0; c < k; ++c) {
            l1ls_report& r = reports[c];
            double* xc = X_out + (size_t)c * n;
            double P, D, gap;
            L1LS_TRY(gap_fp64(I, taus[c], xc, &P, &D, &gap, s));
            if (o->polish == 1 || !(gap <= o->rel_gap_tol)) {
                int rounds = 0;
                int64_t pcg = 0;
                L1LS_TRY(polish_fp64(I, taus[c], xc, s, &rounds, &pcg, 0.0));
                L1LS_TRY(gap_fp64(I, taus[c], xc, &P, &D, &gap, s));
                r.polish_rounds = rounds;
                r.inner = pcg;
            }
            r.primal = P;
            r.dual = D;
            r.rel_gap = gap;
            r.converged = (gap <= o->rel_gap_tol) ? 1 : 0;
            r.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            all = all && r.converged;
        }
    }
    return all ? L1LS_OK : L1LS_NOT_CONVERGED;
}
