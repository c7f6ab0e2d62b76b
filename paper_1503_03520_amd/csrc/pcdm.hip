// PCDM on the stored FP64 operator (section 8.1 item PCDM; beta of section
// 8.3): step k updates a random set S_k of varpi coordinates, each by the
// exact minimiser of its separable model at the current x,
//     x_i <- soft(x_i - A_i^T r / (beta L_i), tau / (beta L_i)),
//     r = A x - b,  L_i = (A^T A)_ii,
//     beta = 1 + (omega - 1)(varpi - 1)/(n - 1)  (omega: most nonzeros in a row),
// then brings the residual up to date on the rows the changed columns touch.
// S_k is tau-nice: positions [(k mod q) varpi, (k mod q + 1) varpi) of a
// random bijection pi_e of the original indices, e = k div q, q = n div varpi
// (the Feistel bijection of the generator, tag 0x10000 + e, seed's key).
//
// The varpi updates of a step read the same x and r and write distinct
// coordinates, so a step is one workgroup's work for varpi <= 1024: one
// thread per sampled column, then one per (column, row) pair recomputing
// r_row = A_row x - b_row from the CSR (rows shared by two columns are
// recomputed twice to the same value).  A launch runs many steps with
// workgroup barriers between their phases.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "common.hpp"
#include "kernels.hpp"
#include "rng.hpp"

using namespace l1ls;

l1ls_status gap_fp64(const l1ls_instance* I, double tau, const double* x, double* P, double* D, double* gap,
                     hipStream_t s, DevAlloc* al = nullptr);
l1ls_status rel_err_planted(const l1ls_instance* I, const double* x, double* out, hipStream_t s);

namespace {

constexpr uint32_t kTagPcdmEpoch = 0x10000u;
constexpr int kPcdmMaxVarpi = 1024;
constexpr int kPcdmThreads = 1024;

inline dim3 g1d(int64_t N) { return dim3((unsigned)std::max<int64_t>(1, (N + L1LS_BLOCK - 1) / L1LS_BLOCK)); }

// r = A x - b over the rows (FP64, operator order), one thread per row.
__global__ void k_pcdm_residual(const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                                const double* __restrict__ val, const double* __restrict__ x,
                                const double* __restrict__ b, double* __restrict__ r, int64_t m) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    double acc = 0.0;
    for (int32_t e = ptr[i]; e < ptr[i + 1]; ++e) acc += val[e] * x[col[e]];
    r[i] = acc - b[i];
}

// omega: the largest row length of the CSR (a max reduction into *out).
__global__ void k_row_degree(const int32_t* __restrict__ ptr, int64_t m, int32_t* __restrict__ out) {
    int32_t w = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        w = max(w, ptr[i + 1] - ptr[i]);
#pragma unroll
    for (int o = L1LS_WAVE / 2; o > 0; o >>= 1) w = max(w, __shfl_xor(w, o, L1LS_WAVE));
    if (threadIdx.x % L1LS_WAVE == 0) atomicMax(out, w);
}

__global__ __launch_bounds__(kPcdmThreads) void k_pcdm_steps(
    const int32_t* __restrict__ csr_ptr, const int32_t* __restrict__ csr_col, const double* __restrict__ csr_val,
    const int32_t* __restrict__ csc_ptr, const int32_t* __restrict__ csc_row, const double* __restrict__ csc_val,
    const double* __restrict__ L, const double* __restrict__ b, const int32_t* __restrict__ col_pos,
    double* __restrict__ x, double* __restrict__ r, int64_t n, int varpi, double beta, double tau, Key key,
    int64_t step0, int64_t nsteps) {
    __shared__ int32_t sp[kPcdmMaxVarpi];
    __shared__ double sy[kPcdmMaxVarpi];
    const int t = threadIdx.x;
    const int64_t q = n / varpi;  // steps per epoch
    for (int64_t k = step0; k < step0 + nsteps; ++k) {
        const int64_t e = k / q, i0 = (k % q) * varpi;
        if (t < varpi) {
            const int64_t orig = bijection(i0 + t, n, kTagPcdmEpoch + (uint32_t)e, key);
            const int32_t p = (int32_t)(col_pos ? col_pos[orig] : orig);
            double g = 0.0;
            for (int32_t c = csc_ptr[p]; c < csc_ptr[p + 1]; ++c) g += csc_val[c] * r[csc_row[c]];
            const double v = beta * L[p];
            const double z = x[p] - g / v;
            sp[t] = p;
            sy[t] = soft_threshold<double>(z, tau / v);
        }
        __syncthreads();
        if (t < varpi) x[sp[t]] = sy[t];
        __syncthreads();
        for (int w = t; w < varpi * kMaxNnz; w += blockDim.x) {
            const int32_t p = sp[w / kMaxNnz];
            const int32_t c = csc_ptr[p] + w % kMaxNnz;
            if (c < csc_ptr[p + 1]) {
                const int32_t i = csc_row[c];
                double acc = 0.0;
                for (int32_t h = csr_ptr[i]; h < csr_ptr[i + 1]; ++h) acc += csr_val[h] * x[csr_col[h]];
                r[i] = acc - b[i];
            }
        }
        __syncthreads();
    }
}

}  // namespace

extern "C" l1ls_status l1ls_solve_pcdm(const l1ls_instance* I, const l1ls_solve_opts* o, double* x_out,
                                       l1ls_report* rep) {
    if (!I || !o || !x_out) return L1LS_E_ARG;
    if (o->precision != L1LS_F64 || o->op != L1LS_OP_STORED || o->polish != 0) return L1LS_E_UNSUPPORTED;
    if (!I->csr_v64 || !I->csc_v64) return L1LS_E_UNSUPPORTED;
    const int64_t n = I->n, m = I->m;
    const int varpi = o->pcdm_tau_nice > 0 ? o->pcdm_tau_nice : 40;
    if (varpi > kPcdmMaxVarpi || varpi > n || o->max_iter < 0 || o->check_every < 1) return L1LS_E_ARG;
    if (!(o->rel_gap_tol >= 0.0)) return L1LS_E_ARG;
    const double tau = o->tau > 0 ? o->tau : I->tau;
    if (!is_finite(tau)) return L1LS_E_ARG;
    // epochs are tagged 0x10000 + e with e < 2^16
    if (o->max_iter / (n / varpi) >= 0xFFFF) return L1LS_E_ARG;
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = (hipStream_t)o->stream;
    DevArena W;
    double *x = nullptr, *r = nullptr, *xo = nullptr;
    int32_t* deg = nullptr;
    L1LS_TRY(W.alloc(&x, n));
    L1LS_TRY(W.alloc(&r, m));
    L1LS_TRY(W.alloc(&xo, n));
    L1LS_TRY(W.alloc(&deg, 1));
    auto done = [&](l1ls_status st) {
        (void)hipStreamSynchronize(s);
        W.release();
        return st;
    };
    if (o->x0_dev)
        hipLaunchKernelGGL((k_gather_perm<double, double>), g1d(n), dim3(L1LS_BLOCK), 0, s, o->x0_dev, x, I->op_col_of,
                           n);
    else if (hipMemsetAsync(x, 0, n * sizeof(double), s) != hipSuccess)
        return done(L1LS_E_HIP);
    if (hipMemsetAsync(deg, 0, sizeof(int32_t), s) != hipSuccess) return done(L1LS_E_HIP);
    hipLaunchKernelGGL(k_row_degree, dim3(256), dim3(L1LS_BLOCK), 0, s, I->csr_ptr, m, deg);
    hipLaunchKernelGGL(k_pcdm_residual, g1d(m), dim3(L1LS_BLOCK), 0, s, I->csr_ptr, I->csr_col, I->csr_v64, x, I->b_op,
                       r, m);
    int32_t omega = 0;
    if (hipMemcpyAsync(&omega, deg, sizeof(omega), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return done(L1LS_E_HIP);
    const double beta = 1.0 + (double)(omega - 1) * (double)(varpi - 1) / (double)std::max<int64_t>(n - 1, 1);
    const Key key = seed_key(I->seed);
    l1ls_report rr;
    std::memset(&rr, 0, sizeof(rr));
    int64_t k = 0;
    l1ls_status st = L1LS_OK;
    while (k < o->max_iter) {
        const int64_t steps = std::min<int64_t>(o->check_every, o->max_iter - k);
        hipLaunchKernelGGL(k_pcdm_steps, dim3(1), dim3(kPcdmThreads), 0, s, I->csr_ptr, I->csr_col, I->csr_v64,
                           I->csc_ptr, I->csc_row, I->csc_v64, I->colnorm2_op, I->b_op, I->op_col_pos, x, r, n, varpi,
                           beta, tau, key, k, steps);
        if (hipGetLastError() != hipSuccess) return done(L1LS_E_HIP);
        k += steps;
        if (o->rel_gap_tol > 0.0 || k == o->max_iter) {
            hipLaunchKernelGGL((k_gather_perm<double, double>), g1d(n), dim3(L1LS_BLOCK), 0, s, x, xo, I->op_col_pos,
                               n);
            if ((st = gap_fp64(I, tau, xo, &rr.primal, &rr.dual, &rr.rel_gap, s)) != L1LS_OK) return done(st);
            if (o->rel_gap_tol > 0.0 && rr.rel_gap <= o->rel_gap_tol) {
                rr.converged = 1;
                break;
            }
        }
    }
    hipLaunchKernelGGL((k_gather_perm<double, double>), g1d(n), dim3(L1LS_BLOCK), 0, s, x, x_out, I->op_col_pos, n);
    if (hipGetLastError() != hipSuccess) return done(L1LS_E_HIP);
    if ((st = rel_err_planted(I, x_out, &rr.rel_err, s)) != L1LS_OK) return done(st);
    rr.iterations = k;
    rr.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (rep) *rep = rr;
    st = done(L1LS_OK);
    if (st != L1LS_OK) return st;
    return rr.converged ? L1LS_OK : L1LS_NOT_CONVERGED;
}
