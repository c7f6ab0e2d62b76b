// FISTA (section 8.1) for an instance small enough that its stored FP64
// operator and iterates fit in the LDS of one compute unit (160 KB on
// gfx950): one workgroup of 1024 threads stages the CSR, the CSC, both x
// slots and r_y in LDS once and then runs every iteration, the duality-gap
// test included, without leaving the kernel.  At such sizes the
// multi-kernel driver is bound by launch latency (two launches per
// iteration); here an iteration is two LDS sweeps and two barriers.
//
// The arithmetic is that of k_residual / k_transpose_prox: every row and
// column sum adds the separately rounded products in storage order, and the
// epilogues are the same expressions, so the iterates equal the
// multi-kernel path's bit for bit.  Only the FP64 statistics of the gap are
// reduced in another order (one workgroup instead of per-workgroup
// partials).
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"

using namespace l1ls;

namespace {

constexpr int kOcThreads = 1024;
constexpr int kOcWaves = kOcThreads / L1LS_WAVE;
constexpr int kOcMaxPer = 4;                 // rows (columns) per thread: m, n <= 4096
constexpr int kOcLds = 160 * 1024;           // LDS of one workgroup
constexpr int kOcRed = kOcWaves * 5 * 8;     // reduction scratch (5 FP64 stats per wave)
constexpr int kOcData = kOcLds - kOcRed;

struct OcResult {
    double P, D, gap;
    int64_t iters;      // iterations run
    int64_t conv_iter;  // iteration at which the gap test passed (-1: never)
    int32_t nonfinite;
    int32_t pad;
};

// Bytes of the LDS image for (m, n, nnz): FP64 values first (8-byte aligned),
// then the int32 arrays.
inline int64_t onchip_bytes(int64_t m, int64_t n, int64_t nnz) {
    return 8 * (2 * nnz + 2 * n + m) + 4 * ((m + 1) + nnz + (n + 1) + nnz);
}

// Block reduction of NS FP64 stats (sums for index < NSUM, max otherwise);
// result valid in every thread.
template <int NS, int NSUM>
__device__ __forceinline__ void oc_reduce(double (&v)[NS], double* red) {
    const int lane = threadIdx.x % L1LS_WAVE, wid = threadIdx.x / L1LS_WAVE;
#pragma unroll
    for (int i = 0; i < NS; ++i) v[i] = (i < NSUM) ? wave_sum(v[i]) : wave_max(v[i]);
    __syncthreads();  // red may still be read by the previous reduction
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < NS; ++i) red[wid * NS + i] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        double a = red[i];
        for (int w = 1; w < kOcWaves; ++w) a = (i < NSUM) ? a + red[w * NS + i] : fmax(a, red[w * NS + i]);
        v[i] = a;
    }
}

// sum_k val[k] * vec[idx[k]] over [beg, end): products rounded on their own,
// then added in storage order (as the LDS-staged tile sums of the
// multi-kernel passes).
__device__ __forceinline__ double oc_dot(const int32_t* idx, const double* val, const double* vec, int32_t beg,
                                         int32_t end) {
#pragma clang fp contract(off)
    double acc = 0.0;
    for (int32_t k = beg; k < end; ++k) {
        const double p = val[k] * vec[idx[k]];
        acc += p;
    }
    return acc;
}

__global__ __launch_bounds__(kOcThreads) void k_fista_onchip(
    const int32_t* __restrict__ csr_ptr, const int32_t* __restrict__ csr_col, const double* __restrict__ csr_val,
    const int32_t* __restrict__ csc_ptr, const int32_t* __restrict__ csc_row, const double* __restrict__ csc_val,
    const double* __restrict__ b, double* __restrict__ x, const double* __restrict__ betas, int64_t m, int64_t n,
    int64_t nnz, double L, double thr, double tau, double tol, int64_t max_iter, int check,
    OcResult* __restrict__ res) {
    __shared__ __align__(16) unsigned char lds[kOcLds];
    double* sval = reinterpret_cast<double*>(lds);
    double* cval = sval + nnz;
    double* xs0 = cval + nnz;
    double* xs1 = xs0 + n;
    double* ry = xs1 + n;
    int32_t* sptr = reinterpret_cast<int32_t*>(ry + m);
    int32_t* scol = sptr + (m + 1);
    int32_t* cptr = scol + nnz;
    int32_t* crow = cptr + (n + 1);
    double* red = reinterpret_cast<double*>(lds + kOcData);
    const int tid = threadIdx.x;
    for (int64_t e = tid; e < nnz; e += kOcThreads) {
        sval[e] = csr_val[e];
        cval[e] = csc_val[e];
        scol[e] = csr_col[e];
        crow[e] = csc_row[e];
    }
    for (int64_t i = tid; i <= m; i += kOcThreads) sptr[i] = csr_ptr[i];
    for (int64_t j = tid; j <= n; j += kOcThreads) cptr[j] = csc_ptr[j];
    for (int64_t j = tid; j < n; j += kOcThreads) xs0[j] = xs1[j] = x[j];
    __syncthreads();
    // rows / columns of this thread, their b and r_x
    double bq[kOcMaxPer], rxq[kOcMaxPer];
#pragma unroll
    for (int q = 0; q < kOcMaxPer; ++q) {
        const int64_t i = tid + (int64_t)q * kOcThreads;
        bq[q] = (i < m) ? b[i] : 0.0;
        rxq[q] = 0.0;
    }
    // r_x,0 = A x_0 - b and r_y,1 = r_x,0 (beta_0 = 0)
    double s_res[3] = {0.0, 0.0, 0.0};  // ||r_x||^2, ||r_y||^2, b . r_y
#pragma unroll
    for (int q = 0; q < kOcMaxPer; ++q) {
        const int64_t i = tid + (int64_t)q * kOcThreads;
        if (i < m) {
            const double acc = oc_dot(scol, sval, xs0, sptr[i], sptr[i + 1]);
            const double r = acc - bq[q];
            rxq[q] = r;
            ry[i] = r;
            s_res[0] += r * r;
            s_res[1] += r * r;
            s_res[2] += bq[q] * r;
        }
    }
    oc_reduce<3, 3>(s_res, red);  // also the barrier that publishes r_y
    double ryy_prev = s_res[1], bry_prev = s_res[2];
    double P = 0.0, D = 0.0, gap = 0.0;
    int64_t conv = -1, k = 0;
    int32_t nonfinite = 0;
    for (k = 1; k <= max_iter; ++k) {
        const double beta_prev = betas[k - 1], beta_k = betas[k];
        double* xcur = ((k - 1) & 1) ? xs1 : xs0;  // x_{k-1}
        double* xslot = (k & 1) ? xs1 : xs0;       // x_{k-2} in, x_k out
        const bool chk = (k % check == 0) || k == max_iter;
        const bool res_stats = chk || ((k + 1) % check == 0) || k + 1 == max_iter;
        double s_tr[2] = {0.0, 0.0};  // sum |x_k|, max |g|
#pragma unroll
        for (int q = 0; q < kOcMaxPer; ++q) {
            const int64_t j = tid + (int64_t)q * kOcThreads;
            if (j < n) {
                const double acc = oc_dot(crow, cval, ry, cptr[j], cptr[j + 1]);
                const double xc = xcur[j];
                const double y = xc + beta_prev * (xc - xslot[j]);
                const double xn = soft_threshold<double>(y - acc / L, thr);
                xslot[j] = xn;
                s_tr[0] += fabs(xn);
                s_tr[1] = fmax(s_tr[1], fabs(acc));
            }
        }
        __syncthreads();  // x_k complete before the residual reads it
        double sr[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int q = 0; q < kOcMaxPer; ++q) {
            const int64_t i = tid + (int64_t)q * kOcThreads;
            if (i < m) {
                const double acc = oc_dot(scol, sval, xslot, sptr[i], sptr[i + 1]);
                const double r = acc - bq[q];
                const double yv = (1.0 + beta_k) * r - beta_k * rxq[q];
                rxq[q] = r;
                ry[i] = yv;
                sr[0] += r * r;
                sr[1] += yv * yv;
                sr[2] += bq[q] * yv;
            }
        }
        if (chk) {
            double st[5] = {sr[0], s_tr[0], 0.0, 0.0, s_tr[1]};  // rr, l1 | ginf
            oc_reduce<5, 4>(st, red);
            const double rr = st[0], l1 = st[1], ginf = st[4];
            P = tau * l1 + 0.5 * rr;
            const double theta = (ginf <= tau) ? 1.0 : tau / ginf;
            D = -0.5 * theta * theta * ryy_prev - theta * bry_prev;
            gap = (P - D) / fabs(P);
            const bool finite = (P == P) && (D == D) && (P - P == 0.0) && (D - D == 0.0);
            if (!finite) {
                nonfinite = 1;
                break;
            }
            if (tol > 0.0 && gap <= tol) {
                conv = k;
                break;
            }
        }
        if (res_stats) {
            double st[3] = {sr[0], sr[1], sr[2]};
            oc_reduce<3, 3>(st, red);  // also publishes r_y
            ryy_prev = st[1];
            bry_prev = st[2];
        } else {
            __syncthreads();  // r_y complete before the next transpose reads it
        }
    }
    const int64_t last = (conv >= 0) ? conv : std::min<int64_t>(k, max_iter);
    __syncthreads();
    const double* xf = (last & 1) ? xs1 : xs0;
    for (int64_t j = tid; j < n; j += kOcThreads) x[j] = xf[j];
    if (tid == 0) {
        res->P = P;
        res->D = D;
        res->gap = gap;
        res->iters = last;
        res->conv_iter = conv;
        res->nonfinite = nonfinite;
    }
}

}  // namespace

// Whether FISTA on (I, opts) runs in one workgroup: FP64 on the stored
// operator, the gap test on, at least one iteration, no kernel timing, and
// the stored A with both x slots and r_y within the LDS.
bool fista_onchip_fits(const l1ls_instance* I, const l1ls_solve_opts* o) {
    if (o->op != L1LS_OP_STORED || o->precision != L1LS_F64 || o->time_kernels || o->max_iter < 1) return false;
    if (!I->csr_v64 || !I->csc_v64) return false;
    if (I->m > (int64_t)kOcThreads * kOcMaxPer || I->n > (int64_t)kOcThreads * kOcMaxPer) return false;
    return onchip_bytes(I->m, I->n, I->nnz) <= kOcData;
}

// FISTA from x0 (or 0) with the multi-kernel driver's iteration, momentum
// sequence and gap test; x_out (original order) receives the last iterate
// (the converged one when the test passed).  Fills iterations, primal,
// dual, rel_gap and converged of *rep.
l1ls_status fista_onchip_run(const l1ls_instance* I, const l1ls_solve_opts* o, double tau, double L, double* x_out,
                             l1ls_report* rep) {
    hipStream_t s = (hipStream_t)o->stream;
    const int64_t n = I->n, K = o->max_iter;
    const int check = std::max(1, o->check_every);
    // beta_k = (t_k - 1) / t_{k+1}, t_1 = 1, t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2,
    // in the multi-kernel driver's operation order; betas[0] = 0
    std::vector<double> betas(K + 1);
    {
#pragma clang fp contract(off)
        double t = 1.0;
        betas[0] = 0.0;
        for (int64_t k = 1; k <= K; ++k) {
            const double t_next = (1.0 + std::sqrt(1.0 + 4.0 * t * t)) / 2.0;
            betas[k] = (t - 1.0) / t_next;
            t = t_next;
        }
    }
    // one device block: the result record, x (n) and the momentum table (K + 1)
    DevArena tmp;
    double* blk = nullptr;
    constexpr int64_t kRes = (sizeof(OcResult) + 7) / 8;
    auto done = [&](l1ls_status st) {
        (void)hipStreamSynchronize(s);
        tmp.release();
        return st;
    };
    l1ls_status st;
    if ((st = tmp.alloc(&blk, kRes + n + K + 1)) != L1LS_OK) return done(st);
    OcResult* res = reinterpret_cast<OcResult*>(blk);
    double* xb = blk + kRes;
    double* bt = xb + n;
    if (hipMemcpyAsync(bt, betas.data(), (K + 1) * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess)
        return done(L1LS_E_HIP);
    if (o->x0_dev)
        hipLaunchKernelGGL((k_gather_perm<double, double>), grid_1d(n), dim3(L1LS_BLOCK), 0, s, o->x0_dev, xb,
                           I->op_col_of, n);
    else if (hipMemsetAsync(xb, 0, n * sizeof(double), s) != hipSuccess)
        return done(L1LS_E_HIP);
    hipLaunchKernelGGL(k_fista_onchip, dim3(1), dim3(kOcThreads), 0, s, I->csr_ptr, I->csr_col, I->csr_v64,
                       I->csc_ptr, I->csc_row, I->csc_v64, I->b_op, xb, bt, I->m, n, I->nnz, L, tau / L, tau,
                       o->rel_gap_tol, K, check, res);
    hipLaunchKernelGGL((k_gather_perm<double, double>), grid_1d(n), dim3(L1LS_BLOCK), 0, s, xb, x_out,
                       I->op_col_pos, n);
    OcResult h;
    if (hipMemcpyAsync(&h, res, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess) return done(L1LS_E_HIP);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) return done(L1LS_E_HIP);
    rep->iterations = h.iters;
    rep->primal = h.P;
    rep->dual = h.D;
    rep->rel_gap = h.gap;
    rep->converged = (h.conv_iter >= 0) ? 1 : 0;
    rep->rel_err = -1.0;
    return done(h.nonfinite ? L1LS_E_NONFINITE : L1LS_OK);
}
